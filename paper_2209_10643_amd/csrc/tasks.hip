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
upir_status upir_plain_trace(upir_ctx *c, int64_t task, const int32_t *preds, int32_t np,
                             hipStream_t s);                                          // task_engine.hip
upir_status upir_plain_trace_start(upir_ctx *c);                                      // task_engine.hip
upir_status upir_plain_trace_preds(upir_ctx *c, int32_t **dev_out,
                                   std::vector<int64_t> &offsets);                    // task_engine.hip

static bool task_body_ok(int32_t k) {
  return k == UPIR_BODY_AXPY || k == UPIR_BODY_SUM || k == UPIR_BODY_MATVEC || k == UPIR_BODY_COVER;
}

// Checks shared by upir_task and upir_taskloop; resolves the SPMD shape.
static upir_status check_task(upir_ctx *c, const upir_spmd *spmd, upir_loop_h lp, const upir_depend *deps,
                              int32_t ndeps, upir_spmd &sp) {
  if (!lp || !c->loops.count(lp)) return upir_fail(c, UPIR_EINVAL, "task: unknown loop handle");
  if (ndeps < 0 || (ndeps > 0 && !deps)) return upir_fail(c, UPIR_EDEPEND, "task: depend list");
  if (!task_body_ok(lp->kind))
    return upir_fail(c, UPIR_EUNSUPPORTED, "task: body %d is not offered as a task (AXPY, SUM, MATVEC, COVER)", lp->kind);
  if (lp->loop.collapse != 1) return upir_fail(c, UPIR_EUNSUPPORTED, "task: 1-D loops only");
  for (int32_t i = 0; i < ndeps; ++i)
    if (deps[i].type < UPIR_DEP_IN || deps[i].type > UPIR_DEP_INOUT)
      return upir_fail(c, UPIR_EDEPEND, "task: depend %d has type %d", i, deps[i].type);
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "task creation during graph capture");
  sp = upir_spmd{0, 0, UPIR_TARGET_GPU};
  if (spmd) sp = *spmd;
  if (sp.target == 0) sp.target = UPIR_TARGET_GPU;
  if (sp.target != UPIR_TARGET_GPU) return upir_fail(c, UPIR_EUNSUPPORTED, "task: only offload to the GPU");
  return UPIR_OK;
}

extern "C" upir_status upir_taskloop(upir_ctx *c, const upir_spmd *spmd, upir_loop_h lp, int64_t grainsize,
                                     int64_t num_tasks, const upir_depend *deps, int32_t ndeps, int64_t *first_task,
                                     int64_t *count) {
  if (!c) return UPIR_EINVAL;
  upir_spmd sp;
  upir_status st = check_task(c, spmd, lp, deps, ndeps, sp);
  if (st) return st;
  if (grainsize < 0 || num_tasks < 0) return upir_fail(c, UPIR_EINVAL, "taskloop: negative grainsize / num_tasks");
  if (lp->kind == UPIR_BODY_SUM || lp->has_red)
    return upir_fail(c, UPIR_EUNSUPPORTED, "taskloop: loops with a reduction are not split into tasks");
  const int64_t n = lp->n;
  int64_t G = 0;
  if (n > 0) {
    G = INT64_MAX;
    if (num_tasks > 0) G = std::min(G, std::min(num_tasks, n));
    if (grainsize > 0) G = std::min(G, std::max<int64_t>(1, n / grainsize));
    if (G == INT64_MAX) G = std::min<int64_t>(n, std::max<int64_t>(1, (n + 65535) / 65536));
    G = std::max<int64_t>(1, G);
  }
  if (G > (1 << 20)) return upir_fail(c, UPIR_EINVAL, "taskloop: %lld tasks", (long long)G);
  const int64_t first = (int64_t)c->tasks.size();
  const std::vector<int64_t> preds = c->deps.preds_of(deps, ndeps);
  const int64_t q = G ? n / G : 0, r = G ? n % G : 0;
  for (int64_t t = 0; t < G; ++t) {
    TaskRec rec{sp, lp, preds};
    rec.lo = t * q + std::min(t, r);
    rec.hi = rec.lo + q + (t < r ? 1 : 0);
    c->tasks.push_back(std::move(rec));
  }
  for (int64_t t = 0; t < G; ++t) c->deps.record(deps, ndeps, first + t);
  if (first_task) *first_task = first;
  if (count) *count = G;
  return UPIR_OK;
}

extern "C" upir_status upir_task(upir_ctx *c, const upir_spmd *spmd, upir_loop_h lp, const upir_depend *deps,
                                 int32_t ndeps, int64_t *task_id) {
  if (!c) return UPIR_EINVAL;
  upir_spmd sp;
  upir_status st = check_task(c, spmd, lp, deps, ndeps, sp);
  if (st) return st;
  if (lp->has_red && lp->red.result_on_host && lp->red.async)
    return upir_fail(c, UPIR_EINVAL, "task: reductions of tasks complete at taskwait; async is meaningless");
  const int64_t id = (int64_t)c->tasks.size();
  c->tasks.push_back(TaskRec{sp, lp, c->deps.preds_of(deps, ndeps)});
  c->deps.record(deps, ndeps, id);  // once per address and kind
  if (task_id) *task_id = id;
  return UPIR_OK;
}

extern "C" upir_status upir_task_update(upir_ctx *c, void *host, size_t bytes, int32_t dir, const upir_depend *deps,
                                        int32_t ndeps, int64_t *task_id) {
  if (!c) return UPIR_EINVAL;
  if (!host) return upir_fail(c, UPIR_EINVAL, "task_update: null host address");
  if (dir != UPIR_TO_DEVICE && dir != UPIR_FROM_DEVICE) return upir_fail(c, UPIR_EINVAL, "task_update: direction");
  if (ndeps < 0 || (ndeps > 0 && !deps)) return upir_fail(c, UPIR_EDEPEND, "task_update: depend list");
  for (int32_t i = 0; i < ndeps; ++i)
    if (deps[i].type < UPIR_DEP_IN || deps[i].type > UPIR_DEP_INOUT)
      return upir_fail(c, UPIR_EDEPEND, "task_update: depend %d has type %d", i, deps[i].type);
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "task creation during graph capture");
  const int64_t id = (int64_t)c->tasks.size();
  TaskRec rec{upir_spmd{0, 0, UPIR_TARGET_GPU}, nullptr, c->deps.preds_of(deps, ndeps)};
  rec.host = host;
  rec.bytes = bytes;
  rec.dir = dir;
  c->tasks.push_back(std::move(rec));
  c->deps.record(deps, ndeps, id);
  if (task_id) *task_id = id;
  return UPIR_OK;
}

static bool has_copy_tasks(const upir_ctx *c) {
  for (const auto &t : c->tasks)
    if (!t.loop) return true;
  return false;
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
  c->deps.clear();
}

// The loop a task runs: the handle itself, or for a taskloop task a copy
// whose 1-D range is the task's iteration block (same body and scratch).
static upir_loop_obj task_view(const TaskRec &t) {
  upir_loop_obj v = *t.loop;
  if (t.hi >= 0) {
    const int64_t lb = v.loop.dim[0].lb, step = v.loop.dim[0].step;
    v.loop.dim[0].lb = lb + t.lo * step;
    v.loop.dim[0].ub = lb + t.hi * step;
    v.cnt[0] = t.hi - t.lo;
    v.n = t.hi - t.lo;
    if (v.kind == UPIR_BODY_COVER) {  // count[k] is indexed by iteration number
      upir_cover_args a;
      memcpy(&a, v.args, sizeof a);
      a.count += t.lo;
      memcpy(v.args, &a, sizeof a);
    }
  }
  return v;
}

// Loop tasks run on the context stream in creation order; data_update tasks
// run on two copy streams, one per direction (the link carries both
// directions at once). An edge between tasks on different streams becomes
// an event wait; an edge on one stream is kept by stream order. Creation
// order is a topological order, so every event waited for has been recorded.
static int task_queue(const TaskRec &t) { return !t.loop ? (t.dir == UPIR_TO_DEVICE ? 1 : 2) : 0; }

static bool tracing_on(const upir_ctx *c) { return c->trace.tokens || c->trace.start_stamp || c->trace.done_stamp; }

// Runs (or, during a capture, records) every pending task. With tracing on,
// `tpreds` holds the predecessor lists on the device (upir_plain_trace_preds,
// made before this call) and `toff` their offsets.
static upir_status run_plain(upir_ctx *c, const int32_t *tpreds, const std::vector<int64_t> &toff) {
  const size_t n = c->tasks.size();
  const bool copies = has_copy_tasks(c);
  const bool tracing = tracing_on(c);
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  };
  if (copies) {
    if (c->capturing) return upir_fail(c, UPIR_EUNSUPPORTED, "data_update tasks are not captured in graphs");
    for (int q = 0; q < 2; ++q)
      if (!c->copy_stream[q] && hipStreamCreateWithFlags(&c->copy_stream[q], hipStreamNonBlocking) != hipSuccess)
        return upir_fail(c, UPIR_EHIP, "copy stream");
    ev.resize(n + 1, nullptr);
    for (auto &e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        cleanup();
        return upir_fail(c, UPIR_EHIP, "task events");
      }
  }
  if (tracing) {
    upir_status st = upir_plain_trace_start(c);
    if (st) {
      cleanup();
      return st;
    }
  }
  hipStream_t qs[3] = {c->stream, c->copy_stream[0], c->copy_stream[1]};
  if (copies) {  // the copy streams start after the work already on the context stream
    hipError_t e = hipEventRecord(ev[n], c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(qs[1], ev[n], 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(qs[2], ev[n], 0);
    if (e != hipSuccess) {
      cleanup();
      return upir_hipfail(c, e, "copy stream start");
    }
  }
  for (size_t j = 0; j < n; ++j) {
    TaskRec &t = c->tasks[j];
    const bool is_copy = !t.loop;
    const int q = task_queue(t);
    hipStream_t s = qs[q];
    upir_status st = UPIR_OK;
    if (copies)
      for (int64_t p : t.preds)
        if (task_queue(c->tasks[p]) != q && hipStreamWaitEvent(s, ev[p], 0) != hipSuccess)
          st = upir_fail(c, UPIR_EHIP, "task %zu: event wait", j);
    if (!st && is_copy) {
      size_t bytes = t.bytes;
      void *dev = nullptr;
      st = upir_map_range(c, t.host, &bytes, &dev);
      if (!st) {
        hipError_t e = t.dir == UPIR_TO_DEVICE ? hipMemcpyAsync(dev, t.host, bytes, hipMemcpyHostToDevice, s)
                                               : hipMemcpyAsync(t.host, dev, bytes, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) st = upir_hipfail(c, e, "data_update task");
      }
    } else if (!st) {
      // a taskloop task (no reduction, so nothing in the copy's scratch is
      // resized) runs as a view; a whole-loop task runs its own handle
      upir_loop_obj view = task_view(t);
      upir_loop_obj *lp = t.hi >= 0 ? &view : t.loop;
      Plan pl;
      st = resolve_plan(c, &t.spmd, lp, pl);
      if (!st) st = launch_plan(c, lp, pl, true);
    }
    if (!st && tracing) {
      const int32_t np = (int32_t)(toff[j + 1] - toff[j]);
      st = upir_plain_trace(c, (int64_t)j, np ? tpreds + toff[j] : nullptr, np, s);
    }
    if (!st && copies && hipEventRecord(ev[j], s) != hipSuccess) st = upir_fail(c, UPIR_EHIP, "task event");
    if (st) {
      if (copies) {
        (void)hipStreamSynchronize(qs[1]);
        (void)hipStreamSynchronize(qs[2]);
      }
      cleanup();
      return st;
    }
  }
  if (copies) {  // let all three streams drain before the events go
    hipError_t e = hipSuccess;
    for (int q = 0; q < 3; ++q) {
      const hipError_t eq = hipStreamSynchronize(qs[q]);
      if (e == hipSuccess) e = eq;
    }
    cleanup();
    if (e != hipSuccess) return upir_hipfail(c, e, "copy streams");
  }
  return UPIR_OK;
}

static upir_status deliver_task_results(upir_ctx *c) {
  bool any = false;
  for (auto &t : c->tasks) {
    upir_loop_obj *lp = t.loop;
    if (lp && lp->has_red && lp->red.result_on_host) {
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
      if (&t != &u && t.loop && t.loop == u.loop && t.loop->has_red && t.loop->red.result_on_host)
        return upir_fail(c, UPIR_EINVAL, "a loop with a host-result reduction can back only one task per taskwait");
  if (mode == UPIR_TASKWAIT_BATCHED && has_copy_tasks(c))
    return upir_fail(c, UPIR_EUNSUPPORTED, "data_update tasks run with taskwait PLAIN");
  upir_status st = settle(c);  // a deferred fold of an earlier loop runs before the tasks
  if (st) return st;
  if (mode == UPIR_TASKWAIT_PLAIN) {
    int32_t *tpreds = nullptr;
    std::vector<int64_t> toff;
    if (tracing_on(c)) st = upir_plain_trace_preds(c, &tpreds, toff);
    if (!st) st = run_plain(c, tpreds, toff);
    if (st == UPIR_OK) st = deliver_task_results(c);  // synchronises: the trace kernels are done
    else (void)hipStreamSynchronize(c->stream);
    upir_dfree(c, tpreds);
  } else {
    st = upir_batched_run(c, false, nullptr);
    if (st == UPIR_OK) st = deliver_task_results(c);
  }
  clear_tasks(c);
  return st;
}

extern "C" upir_status upir_taskwait_graph(upir_ctx *c, int32_t mode, upir_graph_h *out) {
  if (!c || !out) return UPIR_EINVAL;
  if (mode != UPIR_TASKWAIT_PLAIN && mode != UPIR_TASKWAIT_BATCHED) return upir_fail(c, UPIR_EINVAL, "taskwait mode");
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context cannot run tasks");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "already capturing");
  if (has_copy_tasks(c)) return upir_fail(c, UPIR_EUNSUPPORTED, "data_update tasks are not captured in graphs");
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
    // the trace's predecessor lists go to the device before the capture; the
    // graph owns that buffer
    int32_t *tpreds = nullptr;
    std::vector<int64_t> toff;
    if (tracing_on(c)) st = upir_plain_trace_preds(c, &tpreds, toff);
    if (st == UPIR_OK) st = upir_graph_begin(c);
    if (st == UPIR_OK) {
      upir_status rs = run_plain(c, tpreds, toff);
      upir_graph_h g = nullptr;
      st = upir_graph_end(c, &g);
      if (rs) st = rs;
      if (st == UPIR_OK) {
        if (tpreds) g->owned.push_back(tpreds);
        tpreds = nullptr;
        *out = g;
      } else if (g) {
        upir_graph_destroy(c, g);
      }
    }
    upir_dfree(c, tpreds);
  }
  clear_tasks(c);
  return st;
}
