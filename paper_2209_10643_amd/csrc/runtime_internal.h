// Internal host-side state of libupir (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <set>
#include <string>
#include <array>
#include <unordered_map>
#include <vector>

#include "upir.h"
#include "upir_launch.h"
#include "task_graph.h"

struct Mapping {
  uintptr_t host;
  size_t bytes;
  void *dev;
  int32_t refs;
  int32_t map;
  int32_t access;
};

// Device scratch of one loop handle:
//   [0]  (unused)                  [8]  f64/i64 internal result slot
//   [16] i64 dynamic claim counter [24] u32 dynamic exit counter
//   [256] reduction slots, one 128-byte line per workgroup (value, flag)
constexpr size_t SCR_RESULT = 8, SCR_DYN = 16, SCR_DYNEXIT = 24, SCR_SLOTS = 256;
inline size_t scratch_bytes(int64_t cap) { return SCR_SLOTS + (size_t)cap * 8 * upir::SLOT_WORDS; }

struct upir_loop_obj {
  upir_ctx *ctx = nullptr;
  upir_loop loop{};
  upir_sched sched{};
  int32_t kind = 0;
  int32_t args_dev = 1;
  alignas(16) unsigned char args[128];
  size_t args_size = 0;
  bool has_red = false;
  upir_reduction red{};
  int64_t cnt[3] = {1, 1, 1};
  int64_t n = 0;
  unsigned char *scratch = nullptr;
  int64_t part_cap = 0;
  bool pending = false;   // async host-result reduction awaiting wait-release
  void *ws = nullptr;     // library-owned BF16 workspace
  size_t ws_bytes = 0;
  int32_t sum_dtype = UPIR_DT_F32;
  uint64_t key = 0;       // shape key for the tuning table
};

struct upir_graph_obj {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void *> owned;  // device buffers the graph's kernels use
};

struct TaskRec {
  upir_spmd spmd;
  upir_loop_h loop;
  std::vector<int64_t> preds;
  int64_t lo = 0, hi = -1;  // iteration block [lo, hi) of a taskloop task; hi < 0: the whole loop
  // data_update task (loop == nullptr): host range and direction
  void *host = nullptr;
  size_t bytes = 0;
  int32_t dir = 0;
};

// One timing-table row: features of (loop, candidate) and the measured time.
struct TuneRow {
  float feat[32];
  float log2_us;
  int64_t loop_key;
};

struct TunedChoice {
  upir_spmd spmd;
  upir_sched sched;
  double us;
};

struct ModelState;  // cost model (learned.hip)

// Deferred reduction folds (async reductions): a launch leaves one partial
// per wavefront in fold_buf[fold_flip] and flips; the fold is run by the
// next loop kernel on the stream (an extra workgroup of a streaming loop or
// a Jacobi sweep, else workgroup 0 after its own work), or by a
// one-workgroup kernel at the next synchronisation point. Two buffers, so a kernel can fold its predecessor's partials while
// writing its own.
struct PendingFold {
  bool on = false;
  upir::FoldK F{};
  upir_loop_obj *owner = nullptr;  // the loop that deferred it (F.result may be in its scratch)
};

struct upir_ctx {
  int device = -1;
  bool none = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t copy_stream[2] = {nullptr, nullptr};  // data_update tasks to / from the device (on first use)
  upir_alloc_fn alloc = nullptr;
  upir_free_fn free_fn = nullptr;
  void *user = nullptr;
  std::map<uintptr_t, Mapping> table;
  std::string err;
  std::set<upir_loop_obj *> loops;
  std::set<upir_graph_obj *> graphs;
  bool capturing = false;
  std::vector<TaskRec> tasks;
  upir::DepTable deps;                   // depend-clause uses of the pending tasks
  upir_task_trace trace{};
  int num_cus = 256;
  int max_lds = 160 * 1024;
  // schedule selection
  std::vector<TuneRow> db;
  std::unordered_map<uint64_t, TunedChoice> tuned;
  ModelState *model = nullptr;
  bool model_on = false;
  upir_loop_obj *reduce_loop = nullptr;  // cached handle for upir_reduce
  void *trace_clock = nullptr;           // device clock of the plain executor's trace
  PendingFold pend;
  unsigned long long *fold_buf[2] = {nullptr, nullptr};
  int64_t fold_cap = 0;                  // partials per buffer
  int fold_flip = 0;
  std::vector<void *> retired;           // outgrown fold buffers and loop scratch (graphs may use them)
  bool engine_set = false;               // the caller fixed the engine schedule
  upir_engine_sched engine_sched{};      // ... to this
  std::unordered_map<uint64_t, std::pair<upir_engine_sched, double>> tuned_engine;  // batch key -> best, us
  std::unordered_map<uint64_t, std::array<float, 12>> tuned_engine_graph;           // batch key -> graph features
  std::unordered_map<uint64_t, std::vector<float>> tuned_engine_rel;  // batch key -> log2(time / default) per candidate
  void *noalloc_scratch = nullptr;       // this device's static scratch (upir_reduce_noalloc)
  bool no_alloc = false;                 // inside a call that must not allocate (AUTO skips the model)
};

// helpers shared by the runtime translation units
upir_status upir_fail(upir_ctx *c, upir_status s, const char *fmt, ...);
upir_status upir_hipfail(upir_ctx *c, hipError_t e, const char *what);
void *upir_dalloc(upir_ctx *c, size_t bytes);
void upir_dfree(upir_ctx *c, void *p);
void upir_model_free(upir_ctx *c);
// Validate a loop description and fill *lp from it (no allocation).
upir_status describe_loop(upir_ctx *c, const upir_loop *loop, const upir_sched *sched, const upir_body *body,
                          const upir_reduction *red, upir_loop_obj *lp);
// Device address of [host, host + bytes) inside one mapping (bytes = 0: to
// the mapping's end, returned in *bytes).
upir_status upir_map_range(upir_ctx *c, const void *host, size_t *bytes, void **dev);

namespace upir {
struct Plan {
  int32_t variant;
  LoopK L;
  SchedK S;
  upir_spmd spmd;   // resolved teams / units
  upir_sched sched; // resolved schedule
};
upir_status resolve_plan(upir_ctx *c, const upir_spmd *spmd, upir_loop_obj *lp, Plan &out);
upir_status launch_plan(upir_ctx *c, upir_loop_obj *lp, const Plan &pl, bool for_task);
upir_status ensure_scratch(upir_ctx *c, upir_loop_obj *lp, int64_t parts);
// Run a pending deferred fold now (a one-workgroup kernel on the stream).
upir_status settle(upir_ctx *c);
upir_status clear_scratch(upir_ctx *c, upir_loop_obj *lp, unsigned char *scr, int64_t cap);
bool red_is_int(const upir_loop_obj *lp);
upir_status resolve_payload(upir_ctx *c, upir_loop_obj *lp, unsigned char *payload);
uint64_t loop_shape_key(const upir_loop_obj *lp);
// candidate schedules for the tuner / model
int candidate_count(upir_ctx *c, const upir_loop_obj *lp);
bool candidate_at(upir_ctx *c, const upir_loop_obj *lp, int idx, upir_spmd &sp, upir_sched &sc);
void candidate_features(upir_ctx *c, const upir_loop_obj *lp, const upir_spmd &sp, const upir_sched &sc,
                        float f[32]);
bool model_pick(upir_ctx *c, upir_loop_obj *lp, upir_spmd &sp, upir_sched &sc);
void default_choice(upir_ctx *c, const upir_loop_obj *lp, upir_spmd &sp, upir_sched &sc);
// Engine schedules of the batched executor: candidates (0 = default), the
// shape key of the pending task graph, features of (graph, candidate), and
// the cost model's pick among the candidates (false when the model is off).
std::vector<upir_engine_sched> engine_candidates();
uint64_t batch_key(const upir_ctx *c);
void batch_features(const upir_ctx *c, const upir_engine_sched &es, float f[32]);
bool model_pick_engine(upir_ctx *c, upir_engine_sched &es);
// Engine schedule of the pending graph and its source (UPIR_ENGINE_FROM_*).
upir_status resolve_engine_sched(upir_ctx *c, upir_engine_sched &es, int32_t &source);
// Address of the current device's static scratch array (looked up once per
// device; the device must be current).
hipError_t noalloc_setup(int device, void **out);
}  // namespace upir
