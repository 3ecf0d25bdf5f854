// Host-side task-graph logic (no HIP): depend lists -> predecessors, and the
// persistent engine's tables. Paper sec. 3.3 (tasks, depend), sec. 5
// (taskwait).
#include "task_graph.h"

#include <string.h>

#include <algorithm>

namespace upir {

// ------------------------------------------------------------------ depend
std::vector<int64_t> DepTable::preds_of(const upir_depend *deps, int32_t ndeps) const {
  std::vector<int64_t> preds;
  for (int32_t i = 0; i < ndeps; ++i) {
    auto it = addr_.find((uintptr_t)deps[i].addr);
    if (it == addr_.end()) continue;
    const AddrUse &u = it->second;
    const std::vector<int64_t> &src = deps[i].type == UPIR_DEP_IN ? u.writers : u.all;
    preds.insert(preds.end(), src.begin(), src.end());
  }
  std::sort(preds.begin(), preds.end());
  preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
  return preds;
}

void DepTable::record(const upir_depend *deps, int32_t ndeps, int64_t id) {
  for (int32_t i = 0; i < ndeps; ++i) {
    AddrUse &u = addr_[(uintptr_t)deps[i].addr];
    if (u.all.empty() || u.all.back() != id) u.all.push_back(id);
    if (deps[i].type != UPIR_DEP_IN && (u.writers.empty() || u.writers.back() != id)) u.writers.push_back(id);
  }
}

// ------------------------------------------------------------ engine tables
int64_t engine_tile(int32_t kind, int64_t requested) {
  int64_t tile = requested;
  if (kind != UPIR_BODY_MATVEC) tile = std::max<int64_t>(4, (tile + 3) / 4 * 4);
  return std::max<int64_t>(1, std::min<int64_t>(tile, 1 << 24));
}

// Index range [first, last] of the elements k * step + lb, k < n.
static void idx_span(int64_t lb, int64_t step, int64_t n, int64_t &first, int64_t &last) {
  const int64_t end = lb + (n - 1) * step;
  first = std::min(lb, end);
  last = std::max(lb, end);
}

void task_ranges(const TaskD &t, std::vector<MemRange> &reads, std::vector<MemRange> &writes) {
  if (t.n <= 0) return;
  int64_t f, l;
  idx_span(t.lb, t.step, t.n, f, l);
  auto span = [](const void *base, int64_t first_elem, int64_t end_elem) {
    const uintptr_t b = (uintptr_t)base;
    return MemRange{b + (uintptr_t)(first_elem * 4), b + (uintptr_t)(end_elem * 4)};
  };
  switch (t.kind) {
    case UPIR_BODY_AXPY:
      reads.push_back(span(t.x, f, l + 1));
      reads.push_back(span(t.y, f, l + 1));
      writes.push_back(span(t.y, f, l + 1));
      break;
    case UPIR_BODY_SUM:
      reads.push_back(span(t.x, f, l + 1));
      break;
    case UPIR_BODY_MATVEC:
      reads.push_back(span(t.A, f * t.lda, l * t.lda + t.cols));
      reads.push_back(span(t.x, 0, t.cols));
      writes.push_back(span(t.y, f, l + 1));
      break;
    default:  // COVER: count[k] for the task's iteration numbers
      writes.push_back(span(t.cnt, 0, t.n));
  }
}

namespace {
// Intervals sorted by start, with the two largest ends seen so far that
// belong to different tasks: answers "does [lo, hi) overlap an interval of
// a task other than j" with one binary search.
struct IntervalIndex {
  struct Iv {
    uintptr_t lo, hi;
    int64_t task;
  };
  std::vector<Iv> iv;
  std::vector<uintptr_t> best_hi, second_hi;
  std::vector<int64_t> best_task;

  void build() {
    std::sort(iv.begin(), iv.end(), [](const Iv &a, const Iv &b) { return a.lo < b.lo; });
    const size_t n = iv.size();
    best_hi.resize(n);
    second_hi.resize(n);
    best_task.resize(n);
    uintptr_t bh = 0, sh = 0;
    int64_t bt = -1;
    for (size_t i = 0; i < n; ++i) {
      const Iv &v = iv[i];
      if (v.task == bt) {
        bh = std::max(bh, v.hi);
      } else if (v.hi > bh) {
        sh = bh;  // the old best is from another task than the new one and is >= every other end
        bh = v.hi;
        bt = v.task;
      } else {
        sh = std::max(sh, v.hi);
      }
      best_hi[i] = bh;
      second_hi[i] = sh;
      best_task[i] = bt;
    }
  }
  bool overlaps_other(const MemRange &q, int64_t j) const {
    if (q.hi <= q.lo) return false;
    size_t lo = 0, hi = iv.size();  // first interval with start >= q.hi
    while (lo < hi) {
      const size_t m = (lo + hi) / 2;
      if (iv[m].lo < q.hi) lo = m + 1;
      else hi = m;
    }
    if (lo == 0) return false;
    const size_t p = lo - 1;
    return (best_task[p] != j ? best_hi[p] : second_hi[p]) > q.lo;
  }
};
}  // namespace

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

bool build_engine_tables(std::vector<TaskD> &td, const std::vector<std::vector<int64_t>> &preds,
                         std::vector<unsigned char> &image, EngineLayout &lay, std::string &err) {
  const size_t n = td.size();
  if (preds.size() != n) {
    err = "predecessor lists do not match the tasks";
    return false;
  }
  if (n >= (1u << 30)) {
    err = "too many tasks";
    return false;
  }
  // CSR of predecessors and successors
  std::vector<int64_t> succ_off(n + 1, 0), pred_off(n + 1, 0);
  for (size_t j = 0; j < n; ++j) {
    for (int64_t p : preds[j]) {
      if (p < 0 || (size_t)p >= j) {
        err = "a predecessor must be an earlier task";
        return false;
      }
      succ_off[(size_t)p + 1]++;
    }
    pred_off[j + 1] = pred_off[j] + (int64_t)preds[j].size();
  }
  for (size_t j = 0; j < n; ++j) succ_off[j + 1] += succ_off[j];
  const int64_t edges = pred_off[n];
  if (edges >= (1LL << 31)) {
    err = "too many edges";
    return false;
  }
  std::vector<int32_t> succ((size_t)edges), pred((size_t)edges), fill(n, 0), indeg(n, 0);
  for (size_t j = 0; j < n; ++j) {
    int64_t q = pred_off[j];
    for (int64_t p : preds[j]) {
      pred[(size_t)q++] = (int32_t)p;
      succ[(size_t)(succ_off[(size_t)p] + fill[(size_t)p]++)] = (int32_t)j;
    }
    indeg[j] = (int32_t)preds[j].size();
  }
  // tiles, partial ranges
  int64_t parts = 0, total_tiles = 0;
  for (size_t j = 0; j < n; ++j) {
    TaskD &d = td[j];
    d.tile = engine_tile(d.kind, d.tile);
    const int64_t nt = std::max<int64_t>(1, (d.n + d.tile - 1) / d.tile);
    if (nt > (1LL << 30)) {
      err = "task " + std::to_string(j) + " has too many tiles";
      return false;
    }
    d.ntiles = (int32_t)nt;
    d.part_base = (int32_t)parts;
    if (d.red_op) parts += nt;
    if (parts >= (1LL << 31)) {
      err = "too many reduction tiles";
      return false;
    }
    total_tiles += nt;
    if (total_tiles >= (1LL << 31)) {
      err = "too many tiles";
      return false;
    }
    d.succ_begin = (int32_t)succ_off[j];
    d.succ_end = (int32_t)succ_off[j + 1];
    d.pred_begin = (int32_t)pred_off[j];
    d.pred_end = (int32_t)pred_off[j + 1];
  }
  // data-movement mode: private when no other task touches what this one
  // writes and no other task writes what this one reads
  {
    IntervalIndex W, A;
    std::vector<std::vector<MemRange>> rd(n), wr(n);
    uint64_t bytes = 0;
    for (size_t j = 0; j < n; ++j) {
      task_ranges(td[j], rd[j], wr[j]);
      for (const MemRange &r : wr[j]) {
        W.iv.push_back({r.lo, r.hi, (int64_t)j});
        A.iv.push_back({r.lo, r.hi, (int64_t)j});
      }
      for (const MemRange &r : rd[j]) {
        A.iv.push_back({r.lo, r.hi, (int64_t)j});
        bytes += r.hi - r.lo;
      }
      for (const MemRange &r : wr[j]) bytes += r.hi - r.lo;
    }
    W.build();
    A.build();
    const bool nt = bytes >= (64ull << 20);
    for (size_t j = 0; j < n; ++j) {
      bool shared = false;
      for (const MemRange &r : rd[j]) shared = shared || W.overlaps_other(r, (int64_t)j);
      for (const MemRange &r : wr[j]) shared = shared || A.overlaps_other(r, (int64_t)j);
      td[j].mem = shared ? MEM_COHERENT : (nt ? MEM_PRIVATE_NT : MEM_PRIVATE);
    }
  }
  // initially ready tasks take the front of the work list, in task order
  std::vector<int32_t> init_base(n, -1), init_work;
  for (size_t j = 0; j < n; ++j) {
    if (indeg[j] != 0) continue;
    init_base[j] = (int32_t)init_work.size();
    for (int32_t q = 0; q < td[j].ntiles; ++q) init_work.push_back((int32_t)j);
  }
  // layout
  EngineLayout L{};
  size_t o = 0;
  L.tasks = o;
  o += align256(sizeof(TaskD) * n);
  L.succ = o;
  o += align256(4 * succ.size() + 4);
  L.pred = o;
  o += align256(4 * pred.size() + 4);
  L.init_work = o;
  o += align256(4 * init_work.size() + 4);
  L.init_base = o;
  o += align256(4 * n + 4);
  L.indeg0 = o;
  o += align256(4 * n + 4);
  L.static_bytes = o;
  L.indeg = o;
  o += align256(4 * n + 4);
  L.tiles_done = o;
  o += align256(4 * n + 4);
  L.task_base = o;
  o += align256(4 * n + 4);
  L.work = o;  // one 64-bit item per tile: (tile index << 32) | (task + 1); 0 = not yet pushed
  o += align256(8 * (size_t)total_tiles + 8);
  L.ctrl = o;  // counters, each on its own 128-byte line (see ENGINE_CTRL_BYTES)
  o += align256(ENGINE_CTRL_BYTES);
  L.partials = o;
  o += align256(8 * (size_t)std::max<int64_t>(parts, 1));
  L.total_bytes = o;
  L.ntasks = (int32_t)n;
  L.total_tiles = (int32_t)total_tiles;
  L.init_tiles = (int32_t)init_work.size();
  L.edges = edges;
  L.parts = parts;
  image.assign(L.static_bytes, 0);
  if (n) memcpy(&image[L.tasks], td.data(), sizeof(TaskD) * n);
  if (!succ.empty()) memcpy(&image[L.succ], succ.data(), 4 * succ.size());
  if (!pred.empty()) memcpy(&image[L.pred], pred.data(), 4 * pred.size());
  if (!init_work.empty()) memcpy(&image[L.init_work], init_work.data(), 4 * init_work.size());
  if (n) memcpy(&image[L.init_base], init_base.data(), 4 * n);
  if (n) memcpy(&image[L.indeg0], indeg.data(), 4 * n);
  lay = L;
  return true;
}

}  // namespace upir
