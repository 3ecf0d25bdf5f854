// Tasks with depend (paper sec. 3.3) and taskwait (sec. 5): host side.
//
// upir_task records an offloaded task (one loop inside an SPMD region) and
// derives its predecessors from the depend list with OpenMP's rules. The
// graph is acyclic by construction: edges only go from earlier to later
// tasks, so creation order is a topological order.
//
// taskwait PLAIN launches one kernel per task in creation order on the
// context stream (stream order then satisfies every edge). taskwait BATCHED
// hands the whole graph to one persistent kernel (task_engine.hip).
#include <string.h>

#include <algorithm>

#include "runtime_internal.h"

using namespace upir;

upir_status upir_batched_run(upir_ctx *c, bool capture_only, upir_graph_obj **gout);  // task_engine.hip
upir_status upir_plain_trace(upir_ctx *c, int64_t task);                              // task_engine.hip

static bool task_body_ok(int32_t k) {
  return k == UPIR_BODY_AXPY || k == UPIR_BODY_SUM || k == UPIR_BODY_MATVEC || k == UPIR_BODY_COVER;
}

extern "C" upir_status upir_task(upir_ctx *c, const upir_spmd *spmd, upir_loop_h lp, const upir_depend *deps,
                                 int32_t ndeps, int64_t *task_id) {
  if (!c) return UPIR_EINVAL;
  if (!lp || !c->loops.count(lp)) return upir_fail(c, UPIR_EINVAL, "task: unknown loop handle");
  if (ndeps < 0 || (ndeps > 0 && !deps)) return upir_fail(c, UPIR_EDEPEND, "task: depend list");
  if (!task_body_ok(lp->kind))
    return upir_fail(c, UPIR_EUNSUPPORTED, "task: body %d is not offered as a task (AXPY, SUM, MATVEC, COVER)", lp->kind);
  if (lp->loop.collapse != 1) return upir_fail(c, UPIR_EUNSUPPORTED, "task: 1-D loops only");
  if (lp->has_red && lp->red.result_on_host && lp->red.async)
    return upir_fail(c, UPIR_EINVAL, "task: reductions of tasks complete at taskwait; async is meaningless");
  for (int32_t i = 0; i < ndeps; ++i)
    if (deps[i].type < UPIR_DEP_IN || deps[i].type > UPIR_DEP_INOUT)
      return upir_fail(c, UPIR_EDEPEND, "task: depend %d has type %d", i, deps[i].type);
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "task creation during graph capture");
  upir_spmd sp{0, 0, UPIR_TARGET_GPU};
  if (spmd) sp = *spmd;
  if (sp.target == 0) sp.target = UPIR_TARGET_GPU;
  if (sp.target != UPIR_TARGET_GPU) return upir_fail(c, UPIR_EUNSUPPORTED, "task: only offload to the GPU");
  const int64_t id = (int64_t)c->tasks.size();
  std::vector<int64_t> preds;
  for (int32_t i = 0; i < ndeps; ++i) {
    auto it = c->addr.find((uintptr_t)deps[i].addr);
    if (it == c->addr.end()) continue;
    const AddrUse &u = it->second;
    const std::vector<int64_t> &src = deps[i].type == UPIR_DEP_IN ? u.writers : u.all;
    preds.insert(preds.end(), src.begin(), src.end());
  }
  std::sort(preds.begin(), preds.end());
  preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
  // record this task's uses (once per address and kind)
  for (int32_t i = 0; i < ndeps; ++i) {
    AddrUse &u = c->addr[(uintptr_t)deps[i].addr];
    if (u.all.empty() || u.all.back() != id) u.all.push_back(id);
    if (deps[i].type != UPIR_DEP_IN && (u.writers.empty() || u.writers.back() != id)) u.writers.push_back(id);
  }
  c->tasks.push_back(TaskRec{sp, lp, std::move(preds)});
  if (task_id) *task_id = id;
  return UPIR_OK;
}

extern "C" upir_status upir_task_preds(upir_ctx *c, int64_t id, int64_t *preds, int32_t cap, int32_t *count) {
  if (!c || !count) return UPIR_EINVAL;
  if (id < 0 || id >= (int64_t)c->tasks.size()) return upir_fail(c, UPIR_EINVAL, "task id %lld", (long long)id);
  const auto &p = c->tasks[id].preds;
  *count = (int32_t)p.size();
  for (int32_t i = 0; i < cap && i < (int32_t)p.size(); ++i) preds[i] = p[i];
  return UPIR_OK;
}

extern "C" upir_status upir_set_task_trace(upir_ctx *c, const upir_task_trace *t) {
  if (!c) return UPIR_EINVAL;
  if (t)
    c->trace = *t;
  else
    c->trace = upir_task_trace{};
  return UPIR_OK;
}

static void clear_tasks(upir_ctx *c) {
  c->tasks.clear();
  c->addr.clear();
}

static upir_status run_plain(upir_ctx *c) {
  for (size_t j = 0; j < c->tasks.size(); ++j) {
    TaskRec &t = c->tasks[j];
    Plan pl;
    upir_status st = resolve_plan(c, &t.spmd, t.loop, pl);
    if (st) return st;
    st = launch_plan(c, t.loop, pl, true);
    if (st) return st;
    if (c->trace.tokens || c->trace.start_stamp || c->trace.done_stamp) {
      st = upir_plain_trace(c, (int64_t)j);
      if (st) return st;
    }
  }
  return UPIR_OK;
}

static upir_status deliver_task_results(upir_ctx *c) {
  bool any = false;
  for (auto &t : c->tasks) {
    upir_loop_obj *lp = t.loop;
    if (lp->has_red && lp->red.result_on_host) {
      hipError_t e = hipMemcpyAsync(lp->red.result, lp->scratch + SCR_RESULT, 8, hipMemcpyDeviceToHost, c->stream);
      if (e != hipSuccess) return upir_hipfail(c, e, "taskwait: result copy");
      any = true;
    }
  }
  (void)any;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return upir_hipfail(c, e, "taskwait");
  return UPIR_OK;
}

extern "C" upir_status upir_taskwait(upir_ctx *c, int32_t mode) {
  if (!c) return UPIR_EINVAL;
  if (mode != UPIR_TASKWAIT_PLAIN && mode != UPIR_TASKWAIT_BATCHED) return upir_fail(c, UPIR_EINVAL, "taskwait mode");
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context cannot run tasks");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "taskwait during graph capture (use upir_taskwait_graph)");
  // results that live on the host are copied from each loop's result slot
  for (auto &t : c->tasks)
    for (auto &u : c->tasks)
      if (&t != &u && t.loop == u.loop && t.loop->has_red && t.loop->red.result_on_host)
        return upir_fail(c, UPIR_EINVAL, "a loop with a host-result reduction can back only one task per taskwait");
  upir_status st = settle(c);  // a deferred fold of an earlier loop runs before the tasks
  if (st) return st;
  st = mode == UPIR_TASKWAIT_PLAIN ? run_plain(c) : upir_batched_run(c, false, nullptr);
  if (st == UPIR_OK) st = deliver_task_results(c);
  clear_tasks(c);
  return st;
}

extern "C" upir_status upir_taskwait_graph(upir_ctx *c, int32_t mode, upir_graph_h *out) {
  if (!c || !out) return UPIR_EINVAL;
  if (mode != UPIR_TASKWAIT_PLAIN && mode != UPIR_TASKWAIT_BATCHED) return upir_fail(c, UPIR_EINVAL, "taskwait mode");
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context cannot run tasks");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "already capturing");
  for (auto &t : c->tasks)
    if (t.loop->has_red && t.loop->red.result_on_host)
      return upir_fail(c, UPIR_EINVAL, "graph-built tasks need device results");
  upir_status st = settle(c);
  if (st) return st;
  if (mode == UPIR_TASKWAIT_BATCHED) {
    upir_graph_obj *g = nullptr;
    st = upir_batched_run(c, true, &g);
    if (st == UPIR_OK) *out = g;
  } else {
    // every plan is validated (and scratch grown) before capture starts
    for (auto &t : c->tasks) {
      Plan pl;
      st = resolve_plan(c, &t.spmd, t.loop, pl);
      if (st) {
        clear_tasks(c);
        return st;
      }
      if (t.loop->has_red) {
        st = ensure_scratch(c, t.loop, pl.S.T);
        if (st) {
          clear_tasks(c);
          return st;
        }
      }
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      clear_tasks(c);
      return upir_hipfail(c, e, "taskwait_graph");
    }
    st = upir_graph_begin(c);
    if (st == UPIR_OK) {
      upir_status rs = run_plain(c);
      upir_graph_h g = nullptr;
      st = upir_graph_end(c, &g);
      if (rs) st = rs;
      if (st == UPIR_OK) *out = g;
      else if (g) upir_graph_destroy(c, g);
    }
  }
  clear_tasks(c);
  return st;
}
