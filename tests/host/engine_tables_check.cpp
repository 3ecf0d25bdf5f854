// Host check of the task-graph logic (built with AddressSanitizer and UBSan
// by tests/test_host_sanitized.py; no GPU).
//
// Reads a task list, derives each task's predecessors from its depend list
// through DepTable, builds the persistent engine's tables and checks every
// table against a direct recomputation. Writes the predecessor lists (one
// line per task) to the output file for the caller to compare with the
// oracle's depend rules.
//
// Input, one task per line after a first line holding the task count:
//   kind n lb step tile red_op x y A cols lda ndeps (type addr)*
// (pointers as decimal integers; nothing is dereferenced).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "task_graph.h"

using namespace upir;

#define CHECK(cond, ...)                                    \
  do {                                                      \
    if (!(cond)) {                                          \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);  \
      fprintf(stderr, __VA_ARGS__);                         \
      fprintf(stderr, "\n");                                \
      exit(2);                                              \
    }                                                       \
  } while (0)

template <class T>
static const T *at(const std::vector<unsigned char> &img, size_t off) {
  return reinterpret_cast<const T *>(img.data() + off);
}

int main(int argc, char **argv) {
  CHECK(argc == 3, "usage: %s tasks.txt preds_out.txt", argv[0]);
  FILE *f = fopen(argv[1], "r");
  CHECK(f, "cannot open %s", argv[1]);
  long long n = 0;
  CHECK(fscanf(f, "%lld", &n) == 1 && n >= 0, "task count");
  std::vector<TaskD> td((size_t)n);
  std::vector<std::vector<int64_t>> preds((size_t)n);
  DepTable dt;
  std::vector<int64_t> requested((size_t)n);
  for (long long j = 0; j < n; ++j) {
    TaskD &d = td[(size_t)j];
    memset(&d, 0, sizeof d);
    long long kind, nn, lb, step, tile, red, x, y, A, cols, lda, nd;
    CHECK(fscanf(f, "%lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld", &kind, &nn, &lb, &step, &tile,
                 &red, &x, &y, &A, &cols, &lda, &nd) == 12,
          "task %lld", j);
    d.kind = (int32_t)kind;
    d.n = nn;
    d.lb = lb;
    d.step = step;
    d.tile = tile;
    requested[(size_t)j] = tile;
    d.red_op = (int32_t)red;
    d.x = (const float *)(uintptr_t)x;
    d.y = (float *)(uintptr_t)y;
    d.A = (const float *)(uintptr_t)A;
    d.cnt = (int32_t *)(uintptr_t)y;
    d.cols = cols;
    d.lda = lda;
    std::vector<upir_depend> deps((size_t)nd);
    for (long long q = 0; q < nd; ++q) {
      long long typ, addr;
      CHECK(fscanf(f, "%lld %lld", &typ, &addr) == 2, "depend %lld of task %lld", q, j);
      deps[(size_t)q].addr = (const void *)(uintptr_t)addr;
      deps[(size_t)q].type = (int32_t)typ;
    }
    preds[(size_t)j] = dt.preds_of(deps.data(), (int32_t)nd);
    dt.record(deps.data(), (int32_t)nd, j);
  }
  fclose(f);

  std::vector<unsigned char> img;
  EngineLayout L{};
  std::string err;
  CHECK(build_engine_tables(td, preds, img, L, err), "build_engine_tables: %s", err.c_str());

  // layout: aligned, ordered, non-overlapping sections
  const size_t offs[] = {L.tasks, L.succ, L.pred, L.init_work, L.init_base, L.indeg0, L.static_bytes,
                         L.indeg, L.tiles_done, L.task_base, L.work, L.ctrl, L.partials, L.total_bytes};
  for (size_t i = 0; i + 1 < sizeof offs / sizeof offs[0]; ++i) {
    CHECK(offs[i] % 256 == 0, "section %zu not aligned", i);
    CHECK(offs[i] <= offs[i + 1], "section %zu out of order", i);
  }
  CHECK(img.size() == L.static_bytes, "image size");
  CHECK(L.indeg == L.static_bytes, "mutable part starts after the image");
  CHECK(L.ntasks == n, "ntasks");
  CHECK(L.ctrl - L.work >= 8 * (size_t)L.total_tiles, "work list holds one 64-bit item per tile");
  CHECK(L.partials - L.ctrl >= ENGINE_CTRL_BYTES, "control block holds one line per work queue");

  // tasks: tiles, partial ranges, CSR ranges
  const TaskD *T = at<TaskD>(img, L.tasks);
  long long tiles = 0, parts = 0, edges = 0;
  for (long long j = 0; j < n; ++j) {
    const TaskD &d = T[j];
    CHECK(memcmp(&d, &td[(size_t)j], sizeof d) == 0, "image task %lld differs", j);
    CHECK(d.tile == engine_tile(d.kind, requested[(size_t)j]), "tile of %lld", j);
    CHECK(d.tile >= 1 && (d.kind == UPIR_BODY_MATVEC || d.tile % 4 == 0), "tile shape of %lld", j);
    const long long want_nt = d.n > 0 ? (d.n + d.tile - 1) / d.tile : 1;
    CHECK(d.ntiles == want_nt, "ntiles of %lld: %d vs %lld", j, d.ntiles, want_nt);
    CHECK((long long)(d.ntiles - 1) * d.tile < std::max<long long>(d.n, 1), "last tile of %lld is empty", j);
    if (d.red_op) {
      CHECK(d.part_base == parts, "part_base of %lld", j);
      parts += d.ntiles;
    }
    tiles += d.ntiles;
    CHECK(d.pred_begin == edges && d.pred_end - d.pred_begin == (long long)preds[(size_t)j].size(),
          "pred range of %lld", j);
    edges += d.pred_end - d.pred_begin;
    CHECK(d.mem >= MEM_COHERENT && d.mem <= MEM_PRIVATE_NT, "mem mode of %lld", j);
  }
  CHECK(tiles == L.total_tiles && parts == L.parts && edges == L.edges, "totals");
  // predecessor lists as given; successor lists are exactly the reversed edges, in order
  const int32_t *P = at<int32_t>(img, L.pred), *S = at<int32_t>(img, L.succ);
  std::vector<std::vector<int32_t>> succ_want((size_t)n);
  for (long long j = 0; j < n; ++j)
    for (size_t q = 0; q < preds[(size_t)j].size(); ++q) {
      CHECK(P[T[j].pred_begin + (long long)q] == preds[(size_t)j][q], "pred %zu of %lld", q, j);
      succ_want[(size_t)preds[(size_t)j][q]].push_back((int32_t)j);
    }
  long long so = 0;
  for (long long i = 0; i < n; ++i) {
    CHECK(T[i].succ_begin == so && T[i].succ_end - T[i].succ_begin == (long long)succ_want[(size_t)i].size(),
          "succ range of %lld", i);
    for (size_t q = 0; q < succ_want[(size_t)i].size(); ++q)
      CHECK(S[so + (long long)q] == succ_want[(size_t)i][q], "succ %zu of %lld", q, i);
    so += (long long)succ_want[(size_t)i].size();
  }
  // in-degrees, initial work list and bases
  const int32_t *I0 = at<int32_t>(img, L.indeg0), *IB = at<int32_t>(img, L.init_base);
  const int32_t *IW = at<int32_t>(img, L.init_work);
  long long w = 0;
  for (long long j = 0; j < n; ++j) {
    CHECK(I0[j] == (int32_t)preds[(size_t)j].size(), "indeg of %lld", j);
    if (preds[(size_t)j].empty()) {
      CHECK(IB[j] == w, "init base of %lld", j);
      for (int32_t q = 0; q < T[j].ntiles; ++q) CHECK(IW[w + q] == j, "init work item %lld", w + q);
      w += T[j].ntiles;
    } else {
      CHECK(IB[j] == -1, "init base of waiting task %lld", j);
    }
  }
  CHECK(w == L.init_tiles, "init tiles");
  // memory modes against a direct pairwise check (small graphs only)
  if (n <= 4096) {
    std::vector<std::vector<MemRange>> rd((size_t)n), wr((size_t)n);
    for (long long j = 0; j < n; ++j) task_ranges(T[j], rd[(size_t)j], wr[(size_t)j]);
    auto ov = [](const MemRange &a, const MemRange &b) { return a.lo < b.hi && b.lo < a.hi && a.lo < a.hi && b.lo < b.hi; };
    long long priv = 0;
    for (long long j = 0; j < n; ++j) {
      bool shared = false;
      for (long long i = 0; i < n && !shared; ++i) {
        if (i == j) continue;
        for (const MemRange &r : rd[(size_t)j])
          for (const MemRange &q : wr[(size_t)i]) shared = shared || ov(r, q);
        for (const MemRange &r : wr[(size_t)j]) {
          for (const MemRange &q : wr[(size_t)i]) shared = shared || ov(r, q);
          for (const MemRange &q : rd[(size_t)i]) shared = shared || ov(r, q);
        }
      }
      CHECK((T[j].mem == MEM_COHERENT) == shared, "mem mode of %lld: %d, shared %d", j, T[j].mem, (int)shared);
      priv += !shared;
    }
    printf("private_tasks %lld\n", priv);
  }

  FILE *o = fopen(argv[2], "w");
  CHECK(o, "cannot open %s", argv[2]);
  for (long long j = 0; j < n; ++j) {
    for (size_t q = 0; q < preds[(size_t)j].size(); ++q) fprintf(o, q ? " %lld" : "%lld", (long long)preds[(size_t)j][q]);
    fprintf(o, "\n");
  }
  fclose(o);
  printf("tasks %lld edges %lld tiles %lld parts %lld bytes %zu\n", n, (long long)L.edges, (long long)L.total_tiles,
         (long long)L.parts, L.total_bytes);
  return 0;
}
