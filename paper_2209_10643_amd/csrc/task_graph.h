// Host-side task-graph logic of libupir, free of HIP so that it also builds
// (and is checked under AddressSanitizer / UBSan) as plain C++:
//
//  * DepTable: predecessors of a new task from its depend list with OpenMP's
//    rules (paper sec. 3.3, the depend field "similar to the OpenMP depend
//    clause"): `in` on X waits for every earlier task with out / inout on X;
//    out / inout on X waits for every earlier task naming X.
//  * build_engine_tables: the tables the persistent task engine runs from
//    (sec. 3.3 tasks, sec. 5 taskwait): tile counts, successor / predecessor
//    lists (CSR), the initial work list, in-degrees, reduction-partial
//    ranges, and which tasks may move their data without device-coherent
//    accesses because no other task of the graph touches it.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <unordered_map>
#include <vector>

#include "upir.h"

namespace upir {

// ------------------------------------------------------------------ depend
struct AddrUse {
  std::vector<int64_t> writers;  // tasks with out / inout on the address
  std::vector<int64_t> all;      // every task naming the address
};

class DepTable {
 public:
  // Sorted, distinct predecessors of a task with this depend list (nothing is recorded).
  std::vector<int64_t> preds_of(const upir_depend *deps, int32_t ndeps) const;
  // Record task `id`'s uses; ids must be recorded in increasing order.
  void record(const upir_depend *deps, int32_t ndeps, int64_t id);
  void clear() { addr_.clear(); }

 private:
  std::unordered_map<uintptr_t, AddrUse> addr_;
};

// ------------------------------------------------------------ engine tables
// Data-movement mode of a task's operands inside the engine kernel.
enum : int32_t {
  MEM_COHERENT = 0,  // device-coherent accesses: another task of the graph touches the data
  MEM_PRIVATE = 1,   // plain accesses: no other task of the graph reads what this one writes,
                     // nor writes what this one reads
  MEM_PRIVATE_NT = 2 // as MEM_PRIVATE, with the non-temporal hint (large graphs)
};

// One task as the engine kernel sees it (shared with the device code).
struct TaskD {
  int32_t kind, red_op;
  int32_t ntiles, part_base;
  int32_t succ_begin, succ_end;
  int32_t pred_begin, pred_end;
  int64_t n, lb, step, tile;
  float a;
  int32_t vec;  // 16-byte aligned unit-step vector path allowed
  const float *x;
  float *y;
  const float *A;
  int64_t cols, lda;
  int32_t *cnt;
  double init;
  double *result;
  int32_t mem;  // MEM_*
  int32_t pad_;
};

// The engine's control block: line 0 holds the reserved-items counter
// (int32 at byte 0), the error flag (byte 4) and the stamp clock (uint64 at
// byte 16); line 1 + q holds the claim counter of work queue q (work items
// q, q + Q, q + 2Q, ... for Q queues), one 128-byte line each.
constexpr int ENGINE_QUEUES = 8;
constexpr size_t ENGINE_CTRL_LINE = 128;
constexpr size_t ENGINE_CTRL_BYTES = ENGINE_CTRL_LINE * (1 + ENGINE_QUEUES);

// Byte offsets of the engine's sections in its one device allocation (each
// 256-byte aligned). [0, static_bytes) is the image built on the host;
// the rest is mutable state the reset kernel initialises.
struct EngineLayout {
  size_t tasks, succ, pred, init_work, init_base, indeg0;  // static
  size_t indeg, tiles_done, task_base, work, ctrl, partials;  // mutable; work: 8 bytes per tile
  size_t static_bytes, total_bytes;
  int32_t ntasks, total_tiles, init_tiles;
  int64_t edges, parts;
};

// Tile (iterations per work item) the engine uses for a requested tile:
// MATVEC tiles count rows; other tiles are rounded up to a multiple of 4;
// every tile is clamped to [1, 2^24].
int64_t engine_tile(int32_t kind, int64_t requested);

// td[j] arrives with kind, red_op, n, lb, step, tile (requested), the data
// pointers, cols / lda, init and result filled in; preds[j] are the task's
// sorted predecessors (all < j). Sets tile, ntiles, part_base, the CSR
// ranges and mem (nt: the graph moves at least 64 MiB), and writes the
// static image (TaskD array, succ, pred, init work list, init bases,
// in-degrees). Returns false with `err` set if a limit is exceeded.
bool build_engine_tables(std::vector<TaskD> &td, const std::vector<std::vector<int64_t>> &preds,
                         std::vector<unsigned char> &image, EngineLayout &lay, std::string &err);

// Byte ranges [lo, hi) a task reads and writes (addresses as integers).
struct MemRange {
  uintptr_t lo, hi;
};
void task_ranges(const TaskD &t, std::vector<MemRange> &reads, std::vector<MemRange> &writes);

}  // namespace upir
