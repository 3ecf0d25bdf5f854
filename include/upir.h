/*
 * upir.h -- C ABI of libupir, an MI355X (gfx950) executor for the
 * data-parallel pattern of the UPIR paper (Wang, Yi, Yan, "UPIR: Toward the
 * Design of Unified Parallel Intermediate Representation for Parallel
 * Programming Models", arXiv 2209.10643).
 *
 * The calls mirror the paper's IR nodes (Table 1 maps each programming
 * model onto spmd / loop, loop_parallel / task / data / sync):
 *
 *   upir_spmd_launch      sec. 3.1  SPMD region: target, num_teams, num_units
 *   upir_loop_parallel    sec. 3.2  canonical loop (lb, ub, step, collapse) +
 *                                   worksharing schedule and distribute
 *   upir_reduce*          sec. 5    reduction sync (arrive-compute, wait-release)
 *   upir_data_*           sec. 4    data mapping to/from/tofrom/allocate,
 *                                   explicit data_update, mm allocator hook
 *   upir_task / taskwait  sec. 3.3  offloaded tasks ordered by depend; taskwait
 *   upir_taskloop         sec. 3.2  taskloop(grainsize, num_tasks) over the tasks
 *   upir_task_update      sec. 4    data_update with depend, as a copy task
 *
 * There is no compiler here to outline user code, so a loop body is one of
 * a closed set of built-in bodies (upir_body_kind). Loops and reductions run
 * in hand-written HIP kernels; nothing here computes on the host.
 *
 * Conventions for every call:
 *  - Return value: UPIR_OK (0) or a negative upir_status. No call aborts,
 *    throws or exits. After an error, upir_last_error() describes it.
 *  - Validation happens before anything is enqueued: a call that fails
 *    enqueues nothing and leaks nothing.
 *  - Work is enqueued on the context's stream in call order (stream order is
 *    the implicit barrier that ends every loop, sec. 5). Calls whose effect
 *    must be visible on the host (unmap with FROM, update FROM_DEVICE,
 *    reduce_wait, taskwait) have completed that effect when they return.
 *  - One context per host thread; contexts are not thread-safe.
 *  - "host pointer" = an address in the caller's address space that was
 *    registered with upir_data_map; "device pointer" = HIP device memory.
 */
#ifndef UPIR_H
#define UPIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef int32_t upir_status;
#define UPIR_OK            0
#define UPIR_EINVAL       -1   /* malformed argument or descriptor */
#define UPIR_ENOTMAPPED   -2   /* host pointer not present in the data table */
#define UPIR_EOVERLAP     -3   /* new mapping partially overlaps an existing one */
#define UPIR_ENOMEM       -4   /* allocator returned NULL */
#define UPIR_EHIP         -5   /* a HIP runtime call failed (text in last_error) */
#define UPIR_EUNSUPPORTED -6   /* valid in the IR, not provided by this library */
#define UPIR_EDEPEND      -7   /* bad depend list, or the task graph did not drain */
#define UPIR_ESTATE       -8   /* call not allowed in the current state */

typedef struct upir_ctx upir_ctx;
typedef struct upir_loop_obj *upir_loop_h;
typedef struct upir_graph_obj *upir_graph_h;

/* --------------------------------------------------------------- context */
/* Open a context on HIP device `device`. `hip_stream` is a hipStream_t to
 * enqueue on (the caller keeps ownership), or NULL for a stream the context
 * creates and destroys. device = UPIR_DEVICE_NONE opens a host-only context
 * in which descriptors, the data table (ALLOC mappings through a caller
 * allocator) and the task graph can be built and checked, but every call
 * that would touch a GPU returns UPIR_ESTATE. */
#define UPIR_DEVICE_NONE (-1)
upir_status upir_init(int device, void *hip_stream, upir_ctx **out);
/* Release everything the context owns: loop handles, graphs, mappings
 * (device copies are freed without copying back), task lists. */
upir_status upir_finalize(upir_ctx *ctx);
const char *upir_strerror(upir_status s);
const char *upir_last_error(const upir_ctx *ctx);
/* Run a deferred (async) reduction fold if one is pending, then block until
 * all work enqueued on the context's stream has finished. */
upir_status upir_sync(upir_ctx *ctx);
/* Library version string. */
const char *upir_version(void);

/* ------------------------------------------ memory management (sec. 4.2) */
/* The mm_allocator / mm_deallocator pair used for every device buffer the
 * library creates (mapped copies, reduction scratch, BF16 workspaces, task
 * tables). Default: hipMalloc / hipFree. alloc returns NULL on failure. */
typedef void *(*upir_alloc_fn)(size_t bytes, void *user);
typedef void (*upir_free_fn)(void *ptr, void *user);
upir_status upir_set_allocator(upir_ctx *ctx, upir_alloc_fn alloc, upir_free_fn free_fn, void *user);

/* ------------------------------------------- data attributes (sec. 4.1) */
#define UPIR_MAP_TO     1   /* copy host -> device when the mapping is created */
#define UPIR_MAP_FROM   2   /* copy device -> host when the mapping ends */
#define UPIR_MAP_TOFROM 3
#define UPIR_MAP_ALLOC  4   /* device buffer only, no copies */
#define UPIR_ACCESS_RO  1
#define UPIR_ACCESS_WO  2
#define UPIR_ACCESS_RW  3
/* Present-table semantics (reading of the mapping attribute, "similar to
 * OpenMP map"): if [host, host+bytes) lies inside an existing mapping its
 * reference count grows and nothing is copied; if it partially overlaps one
 * the call fails with UPIR_EOVERLAP; otherwise a device buffer of `bytes`
 * is allocated and, for TO/TOFROM, filled asynchronously from host (the host
 * buffer must not change until the next synchronising call). *dev_out
 * (optional) receives the device address of `host`. An ACCESS_RO mapping
 * is never copied back. */
upir_status upir_data_map(upir_ctx *ctx, void *host, size_t bytes, int32_t map, int32_t access, void **dev_out);
/* Drop one reference of the mapping that starts at `host`. When the count
 * reaches zero and `map` includes FROM (and access is not RO), the device
 * buffer is copied back (complete on return), then freed. */
upir_status upir_data_unmap(upir_ctx *ctx, void *host, int32_t map);
/* Explicit data movement (data_update): copy `bytes` at `host` (0 = to the
 * end of its mapping) in direction dir. FROM_DEVICE is complete on return. */
#define UPIR_TO_DEVICE   1
#define UPIR_FROM_DEVICE 2
upir_status upir_data_update(upir_ctx *ctx, void *host, size_t bytes, int32_t dir);
/* Device address of a host address that lies inside a mapping. */
upir_status upir_data_lookup(upir_ctx *ctx, const void *host, void **dev_out);

/* ------------------------------------------------ SPMD region (sec. 3.1) */
#define UPIR_TARGET_GPU     1
#define UPIR_TARGET_CPU     2   /* UPIR_EUNSUPPORTED */
#define UPIR_TARGET_CLUSTER 3   /* UPIR_EUNSUPPORTED */
typedef struct {
    int32_t num_teams;   /* workgroups; 0 = chosen by the library */
    int32_t num_units;   /* work-items per team, 1..1024; 0 = chosen */
    int32_t target;      /* UPIR_TARGET_GPU */
} upir_spmd;

/* ------------------------------------------ loops and worksharing (3.2) */
typedef struct { int64_t lb, ub, step; } upir_dim;   /* ub exclusive, step != 0 */
typedef struct {
    int32_t collapse;          /* 1..3 dimensions, row-major linearisation */
    int32_t pad_;
    upir_dim dim[3];
} upir_loop;

#define UPIR_SCHED_STATIC       0  /* near-equal contiguous blocks, teams then units */
#define UPIR_SCHED_STATIC_CHUNK 1  /* chunks of `chunk` iterations dealt cyclically */
#define UPIR_SCHED_DYNAMIC      2  /* chunks claimed at run time from a device counter */
#define UPIR_SCHED_GUIDED       3  /* like DYNAMIC with decreasing chunk sizes */
#define UPIR_SCHED_RUNTIME      4  /* policy taken from env UPIR_SCHEDULE at launch */
#define UPIR_SCHED_AUTO         5  /* library choice: tuned table, else cost model, else default */
#define UPIR_DIST_TEAMS_UNITS   0
#define UPIR_DIST_TEAMS         1  /* each team's share run by its unit 0 */
#define UPIR_DIST_UNITS         2  /* one team; iterations split over its units */
typedef struct {
    int32_t policy;      /* UPIR_SCHED_* */
    int32_t distribute;  /* UPIR_DIST_* */
    int64_t chunk;       /* STATIC_CHUNK / DYNAMIC / GUIDED chunk (>= 1) */
    int32_t tile[3];     /* tiling before worksharing; 0 = untiled. Tiles are
                            anchored at induction value 0, need unit steps, and
                            the innermost extent must be a multiple of 4. Tiles
                            go to teams by `policy`; inside a tile, group p/4 of
                            its row-major points goes to unit (p/4) mod U. */
    int32_t pad_;
} upir_sched;

/* ------------------------------------------------------ reduction (sec. 5) */
#define UPIR_RED_NONE 0
#define UPIR_RED_SUM  1
#define UPIR_RED_MAX  2
#define UPIR_RED_MIN  3
typedef struct {
    int32_t op;              /* UPIR_RED_* */
    int32_t result_on_host;  /* 1: result is a host address, delivered by
                                upir_reduce_wait (or at launch if !async) */
    double init;             /* folded in once */
    void *result;            /* double (float data) or int64_t (integer data) */
    int32_t async;           /* 1: launch = arrive-compute only (sec. 5 split
                                sync): the kernel leaves one partial per
                                wavefront and the cross-workgroup fold is
                                deferred to the next loop kernel on the
                                context (one of its workgroups) or to the next
                                upir_reduce_wait / upir_sync / graph end /
                                taskwait / data_update / unmap (wait-release).
                                A device result is valid after that point, a
                                host result after upir_reduce_wait. Loops run
                                as tasks ignore the flag. */
    int32_t pad_;
} upir_reduction;

/* -------------------------------------------------------- built-in bodies */
#define UPIR_BODY_AXPY          1  /* 1-D: y[i] = fma(a, x[i], y[i]); reduces y'[i] */
#define UPIR_BODY_SUM           2  /* 1-D: reduces x[i] (needs a reduction) */
#define UPIR_BODY_JACOBI5       3  /* 2-D: dst[i][j] = ((N+S)+(W+E))*0.25 of src;
                                      reduces |dst - src| in float64 */
#define UPIR_BODY_MATMUL_F32    4  /* 2-D over C: C[i][j] = sum_k A[i][k] B[k][j] */
#define UPIR_BODY_MATMUL_BF16   5  /* same with A, B rounded to bfloat16 (RNE),
                                      float32 accumulation */
#define UPIR_BODY_MATMUL_SPLIT3 6  /* A_lo B_hi + A_hi B_lo + A_hi B_hi, hi/lo the
                                      bfloat16 split, float32 accumulation */
#define UPIR_BODY_MATVEC        7  /* 1-D over rows: y[r] = sum_c A[r][c] x[c];
                                      the unit is a 64-lane wavefront */
#define UPIR_BODY_OWNER         8  /* any: out[k] = team * U + unit of iteration k */
#define UPIR_BODY_COVER         9  /* any: count[k] += 1 (atomic) */
#define UPIR_BODY_FILTER7      10  /* 2-D (sec. 6 stencil, filter size 7):
                                      dst[i][j] = sum_{m,n<7} w[m][n] *
                                      src[i+m-3][j+n-3], float32 fma chain with
                                      m outer, n inner, from 0; no reduction.
                                      The loop box must keep the reads inside
                                      the array (lb >= 3, ub <= extent - 3). */

typedef struct { float a; int32_t pad_; const float *x; float *y; } upir_axpy_args;
typedef struct { const void *x; int32_t dtype; int32_t pad_; } upir_sum_args;    /* dtype UPIR_DT_* */
typedef struct { const float *src; float *dst; int64_t ld; } upir_jacobi5_args;
typedef struct {
    const float *A; const float *B; float *C;
    int64_t K, lda, ldb, ldc;
    void *workspace;          /* BF16 hi/lo copies; NULL = library allocates */
    size_t workspace_bytes;   /* see upir_matmul_workspace_bytes */
} upir_matmul_args;
typedef struct { const float *A; const float *x; float *y; int64_t cols, lda; } upir_matvec_args;
typedef struct { int32_t *out; } upir_owner_args;
typedef struct { int32_t *count; } upir_cover_args;
typedef struct { const float *src; float *dst; const float *w; int64_t ld; } upir_filter7_args;
                                   /* w: 49 float32 weights, row-major 7 x 7;
                                      src and dst row-major with pitch ld, distinct */
#define UPIR_DT_F32 1
#define UPIR_DT_F64 2
#define UPIR_DT_I32 3
#define UPIR_DT_I64 4

typedef struct {
    int32_t kind;                  /* UPIR_BODY_* */
    int32_t args_are_device_ptrs;  /* 1: pointers in args are device pointers
                                      (is_device_ptr); 0: host pointers resolved
                                      through the data table at each launch */
    const void *args;              /* one of the *_args structs; copied */
    size_t args_size;              /* sizeof that struct */
} upir_body;

/* Create a loop handle: validates loop, schedule, body and reduction and
 * allocates the reduction scratch. The handle is owned by the library until
 * upir_loop_free or upir_finalize. `red` may be NULL. */
upir_status upir_loop_parallel(upir_ctx *ctx, const upir_loop *loop, const upir_sched *sched,
                               const upir_body *body, const upir_reduction *red, upir_loop_h *out);
upir_status upir_loop_free(upir_ctx *ctx, upir_loop_h loop);
/* Point the handle's reduction at another result address (e.g. one slot per
 * sweep); same kind of address (host/device) as at creation. */
upir_status upir_loop_set_result(upir_ctx *ctx, upir_loop_h loop, void *result);
/* Replace the body arguments of a handle (same body kind and size). */
upir_status upir_loop_set_args(upir_ctx *ctx, upir_loop_h loop, const void *args, size_t args_size);

/* Run `nloops` loops in order inside one SPMD region on the context stream.
 * Each loop ends with the implicit barrier (stream order). Enqueue-only,
 * except that a synchronous host-result reduction waits for its value. */
upir_status upir_spmd_launch(upir_ctx *ctx, const upir_spmd *spmd, const upir_loop_h *loops, int32_t nloops);
/* Wait-release step of a loop's reduction: waits for the loop's last launch
 * and, for a host result, copies the value to the result address. */
upir_status upir_reduce_wait(upir_ctx *ctx, upir_loop_h loop);
/* Standalone reduction of `n` device elements of type dtype (UPIR_DT_*):
 * float data reduce to a double, integer data to an exact int64. */
upir_status upir_reduce(upir_ctx *ctx, int32_t op, int32_t dtype, const void *dev_in, int64_t n,
                        const upir_spmd *spmd, const upir_sched *sched, upir_reduction *red);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reduction of upir_reduce, with the same arguments, kernels and results,
 * that allocates nothing. Its reduction scratch is a static device array of
 * 256 + 128 x UPIR_REDUCE_NOALLOC_MAX_TEAMS bytes that every GPU the library
 * runs on holds until the process ends. Differences from upir_reduce:
 *  - red->result must be a device address (result_on_host = 0; else
 *    UPIR_EINVAL); the call only enqueues, and the result is defined in
 *    stream order after the call's kernels (no synchronisation);
 *  - schedule AUTO resolves to the tuned table or the library default, never
 *    the cost model (its inference allocates);
 *  - a resolved launch of more than UPIR_REDUCE_NOALLOC_MAX_TEAMS workgroups
 *    fails with UPIR_EINVAL before anything is enqueued;
 *  - all calls on one GPU share the array (each call clears what it uses
 *    first, with a kernel): calls that may overlap on one GPU (other
 *    streams, contexts or threads) race and give undefined results. */
#define UPIR_REDUCE_NOALLOC_MAX_TEAMS 4096
upir_status upir_reduce_noalloc(upir_ctx *ctx, int32_t op, int32_t dtype, const void *dev_in, int64_t n,
                                const upir_spmd *spmd, const upir_sched *sched, upir_reduction *red);
/* The launch geometry and kernel variant the library would use (after AUTO
 * resolution): teams, units and the resolved schedule. */
upir_status upir_loop_resolve(upir_ctx *ctx, const upir_spmd *spmd, upir_loop_h loop,
                              upir_spmd *spmd_out, upir_sched *sched_out, int32_t *variant_out);
/* Bytes of BF16 workspace a MATMUL_BF16 / MATMUL_SPLIT3 body needs:
 * (M + N) x K' x 2 (x 2 again for the split's low parts), K' = K rounded up
 * to a multiple of 32. */
size_t upir_matmul_workspace_bytes(int32_t kind, int64_t M, int64_t N, int64_t K);

/* ------------------------------------------------- graphs (stream replay) */
/* Capture everything enqueued on the context stream between begin and end
 * into a replayable HIP graph (no data mapping, no host results inside). */
upir_status upir_graph_begin(upir_ctx *ctx);
upir_status upir_graph_end(upir_ctx *ctx, upir_graph_h *out);
upir_status upir_graph_launch(upir_ctx *ctx, upir_graph_h g);
upir_status upir_graph_destroy(upir_ctx *ctx, upir_graph_h g);

/* ------------------------------------------------------- tasks (sec. 3.3) */
#define UPIR_DEP_IN    1
#define UPIR_DEP_OUT   2
#define UPIR_DEP_INOUT 3
typedef struct { const void *addr; int32_t type; int32_t pad_; } upir_depend;
/* Create an offloaded task that runs `loop` (an AXPY, SUM, MATVEC or COVER
 * 1-D loop) inside `spmd`. Depend semantics follow OpenMP: `in` on X waits
 * for every earlier task with out/inout on X; out/inout on X waits for every
 * earlier task naming X. Addresses are opaque keys. *task_id receives the
 * task's index (0, 1, ... since the last taskwait). The loop handle must
 * stay alive until taskwait. */
upir_status upir_task(upir_ctx *ctx, const upir_spmd *spmd, upir_loop_h loop,
                      const upir_depend *deps, int32_t ndeps, int64_t *task_id);
/* Taskloop (sec. 3.2, loop parallelization by tasking: fields grainsize and
 * num_tasks). The 1-D `loop` (AXPY, MATVEC or COVER; no reduction) is cut
 * into G tasks of near-equal contiguous iteration blocks, the first n mod G
 * one longer: num_tasks > 0 asks for min(num_tasks, n) tasks, grainsize > 0
 * for max(1, n / grainsize) (each task then has at least grainsize and fewer
 * than 2 x grainsize iterations); with both the smaller count; with neither
 * one task per 65536 iterations (at least one). No iterations: no tasks.
 * `deps` apply to the taskloop as a whole: every generated task waits for
 * what a single task with these deps would wait for, the generated tasks do
 * not wait for each other, and later tasks that name an address wait for all
 * of them. *first_task gets the first task id, *count the number G; ids are
 * consecutive. Tasks run at the next taskwait, in either mode. */
upir_status upir_taskloop(upir_ctx *ctx, const upir_spmd *spmd, upir_loop_h loop, int64_t grainsize,
                          int64_t num_tasks, const upir_depend *deps, int32_t ndeps, int64_t *first_task,
                          int64_t *count);
/* data_update as a task (sec. 4 explicit data movement with its depend
 * field): copy `bytes` of the mapped range starting at `host` to the device
 * (UPIR_TO_DEVICE) or back (UPIR_FROM_DEVICE), ordered only by `deps` with
 * the rules of upir_task. It runs at the next upir_taskwait(PLAIN) on the
 * context's copy queue, so it overlaps loop tasks it is not ordered with
 * (host memory should be pinned for the copy engine to run asynchronously).
 * bytes = 0: to the end of the mapping. The range must be mapped when the
 * task runs (UPIR_ENOTMAPPED otherwise). Graphs and the BATCHED executor
 * take no copy tasks (UPIR_EUNSUPPORTED at taskwait). */
upir_status upir_task_update(upir_ctx *ctx, void *host, size_t bytes, int32_t dir, const upir_depend *deps,
                             int32_t ndeps, int64_t *task_id);
/* Predecessors of task `id` as computed from the depend lists (sorted). */
upir_status upir_task_preds(upir_ctx *ctx, int64_t id, int64_t *preds, int32_t cap, int32_t *count);
#define UPIR_TASKWAIT_PLAIN   0  /* one kernel launch per task, in index order */
#define UPIR_TASKWAIT_BATCHED 1  /* one persistent kernel runs the whole graph */
/* Optional per-task trace (device arrays of ntasks uint64): token chain
 * tok[j] = mix(j, tok[p] for p in preds(j)) and start/done stamps from one
 * device-wide counter. NULL pointers disable tracing. */
typedef struct { uint64_t *tokens; uint64_t *start_stamp; uint64_t *done_stamp; } upir_task_trace;
upir_status upir_set_task_trace(upir_ctx *ctx, const upir_task_trace *trace);
/* Run every pending task, wait for completion, clear the task list. */
upir_status upir_taskwait(upir_ctx *ctx, int32_t mode);
/* Build the pending tasks into a replayable graph instead of running them
 * (the task list is cleared). Each upir_graph_launch re-runs the batch. */
upir_status upir_taskwait_graph(upir_ctx *ctx, int32_t mode, upir_graph_h *out);

/* --------------------------------------- schedule selection (AUTO policy) */
/* Exhaustive tuner: time every candidate schedule of `loop` (on scratch
 * copies of its outputs), record rows in the context's timing table and
 * remember the fastest for AUTO. best_us (optional) gets its time. */
upir_status upir_tune(upir_ctx *ctx, const upir_spmd *spmd, upir_loop_h loop, int32_t reps,
                      upir_sched *best, upir_spmd *best_spmd, double *best_us);
/* Candidate count for a loop and the feature vector (32 floats) of one. */
upir_status upir_candidates(upir_ctx *ctx, upir_loop_h loop, int32_t *count);
upir_status upir_candidate_features(upir_ctx *ctx, upir_loop_h loop, int32_t idx, float *feat32,
                                    upir_spmd *spmd_out, upir_sched *sched_out);
/* Timing table I/O: append-only text file, one row per measurement. */
upir_status upir_tune_db_save(upir_ctx *ctx, const char *path);
upir_status upir_tune_db_load(upir_ctx *ctx, const char *path);
upir_status upir_tune_db_size(upir_ctx *ctx, int64_t *rows);
upir_status upir_tune_db_row(upir_ctx *ctx, int64_t row, float *feat32, float *log2_us, int64_t *loop_key);

/* Engine schedule of the batched executor (taskwait BATCHED): the tile
 * (work item) of every task whose schedule is AUTO with no tile of its own,
 * per body: elements per tile for AXPY and COVER tasks, for SUM tasks, and
 * rows per tile for MATVEC tasks. A task graph resolves it, in order, to
 * the schedule the caller set, the exhaustive batch tuner's best for a graph
 * of the same shape, the cost model's choice (among the tuner's best
 * schedules of the ten tuned graphs most like this one, and the default,
 * the one with the lowest sum of the model's prediction and its mean time
 * measured on those graphs), or the default {16384, 16384, 64}. The candidates are the 27 combinations of AXPY
 * {8192, 16384, 32768}, SUM {16384, 32768, 65536} and MATVEC {32, 64, 128};
 * candidate 0 is the default. */
typedef struct { int64_t tile_axpy, tile_sum, rows_matvec; } upir_engine_sched;
#define UPIR_ENGINE_CANDIDATES     27
#define UPIR_ENGINE_FROM_DEFAULT   0
#define UPIR_ENGINE_FROM_TUNER     1
#define UPIR_ENGINE_FROM_MODEL     2
#define UPIR_ENGINE_FROM_CALLER    3
/* Fix the engine schedule (NULL: back to automatic resolution). Tiles must
 * be >= 1 and <= 2^24 (UPIR_EINVAL otherwise). */
upir_status upir_engine_sched_set(upir_ctx *ctx, const upir_engine_sched *sched);
/* The engine schedule the pending tasks would run with, and its source
 * (UPIR_ENGINE_FROM_*). May run the cost model (a forward pass on the GPU). */
upir_status upir_engine_sched_resolve(upir_ctx *ctx, upir_engine_sched *out, int32_t *source);
/* Candidate idx of the engine schedule and the 32 features of (pending task
 * graph, candidate) the cost model sees (feat32 may be NULL). */
upir_status upir_engine_candidate(upir_ctx *ctx, int32_t idx, upir_engine_sched *out, float *feat32);
/* Exhaustive batch tuner: run the pending task graph with the batched
 * executor once per candidate and then `reps` times between HIP events,
 * record one timing-table row per candidate (log2 of its median time over
 * the default candidate's: graph rows hold relative costs) and remember the
 * fastest for graphs of this shape. The tasks stay pending. The runs execute
 * the tasks: a task that updates its data in place (AXPY) is applied
 * (reps + 1) x 27 times, so callers restore such data before the taskwait
 * that counts. UPIR_ESTATE during capture or with no pending tasks. */
upir_status upir_tune_batched(upir_ctx *ctx, int32_t reps, upir_engine_sched *best, double *best_us);

/* Cost model: MLP 32 -> 64 -> 64 -> 1 (float32), trained on the GPU by
 * the library's own forward / backward / Adam kernels. */
#define UPIR_MLP_PARAMS 6337
upir_status upir_model_init(upir_ctx *ctx, uint64_t seed);
upir_status upir_model_set_params(upir_ctx *ctx, const float *host_params);
upir_status upir_model_get_params(upir_ctx *ctx, float *host_params);
/* Forward pass on n device feature rows (n x 32) -> n device predictions. */
upir_status upir_model_forward(upir_ctx *ctx, const float *dev_x, int64_t n, float *dev_y);
/* One step on a device batch: loss (host out), gradients into dev_grad
 * (UPIR_MLP_PARAMS floats, may be NULL), and an Adam update when adam != 0. */
upir_status upir_model_step(upir_ctx *ctx, const float *dev_x, const float *dev_t, int64_t n,
                            float lr, int32_t adam, float *dev_grad, float *loss_out);
/* Train on the context's timing table: epochs over minibatches of `batch`
 * rows, rows whose loop_key % 5 == holdout_mod held out. Returns final
 * train / holdout mean squared errors. */
upir_status upir_model_train(upir_ctx *ctx, int32_t epochs, int32_t batch, float lr, int32_t holdout_mod,
                             float *train_mse, float *holdout_mse);
/* Let AUTO use the model for loops (and task graphs) the tuner has not seen
 * (1) or not (0). */
upir_status upir_model_enable(upir_ctx *ctx, int32_t on);
upir_status upir_model_save(upir_ctx *ctx, const char *path);
upir_status upir_model_load(upir_ctx *ctx, const char *path);

#ifdef __cplusplus
}
#endif
#endif /* UPIR_H */
