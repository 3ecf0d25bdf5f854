// Batched task engine: one persistent kernel runs a whole task graph.
//
// Paper: sec. 3.3 treats an offloaded kernel launch as an asynchronous task
// ordered by depend clauses; sec. 5 lists taskwait. Launching one kernel per
// task pays the launch and synchronisation cost the paper's evaluation
// blames for lost time (sec. 6.2) once per task. Here a grid sized to the
// resident capacity of the GPU runs every task of the graph:
//
//  * each task's loop is cut into tiles of `tile` iterations;
//  * the tiles of every task that becomes ready get a contiguous range of
//    a global work list (one atomic reservation per task); workgroups claim
//    work items with one global counter and wait, if needed, until the item
//    they hold has been filled in by the push that reserved it;
//  * the workgroup that finishes a task's last tile combines the task's
//    reduction (float64, tile order), writes its trace token and stamps, and
//    decrements the remaining in-degree of each successor, pushing those
//    that reach zero;
//  * every wait is bounded: a workgroup that sees no progress for a long
//    time raises an error flag and leaves, so the kernel always drains.
//
// The XCDs' L2 caches are not coherent with each other. Counters, tokens,
// results and reduction partials move with relaxed device-coherent (agent
// scope) atomics, each publisher first waiting for its own accesses to
// complete; no agent-scope fence (a write-back of the whole L2) is used. A
// task whose data another task of the graph also touches reads and writes
// it device-coherently too; a task whose data no other task touches uses
// plain accesses (non-temporal for large graphs), since its tiles touch
// disjoint elements and the kernel's end publishes them.
#include <string.h>

#include <algorithm>
#include <vector>

#include "runtime_internal.h"
#include "task_graph.h"

namespace upir {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct EngineD {
  const TaskD *tasks;
  int32_t ntasks, total_tiles, init_tiles, pad_;
  const int32_t *succ, *pred, *init_work, *init_base, *indeg0;
  int32_t *indeg, *tiles_done, *task_base;
  unsigned long long *work;  // per item: (tile << 32) | (task + 1); 0 until pushed
  int32_t *ctrl;  // control block: [0] work items reserved, [1] error; queue q's claim
                  // counter at int index (q + 1) * ENGINE_CTRL_LINE / 4
  int32_t nq;     // work queues in use (<= ENGINE_QUEUES, <= grid)
  int32_t pad2_;
  unsigned long long *clock;
  double *partials;
  uint64_t *tok, *tstart, *tdone;
  long long spin_limit;
};

__device__ inline uint64_t mix64(uint64_t z) {
  // SplitMix64 finalizer (Steele, Lea, Flood 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Relaxed agent-scope accesses (device-coherent, no cache maintenance).
__device__ inline int ld_i(int32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_i(int32_t *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline int add_i(int32_t *p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long ld_u64(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_u64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long work_item(int task, int tile) {
  return ((unsigned long long)(unsigned)tile << 32) | (unsigned)(task + 1);
}
__device__ inline unsigned long long tick(unsigned long long *p) {
  return __hip_atomic_fetch_add(p, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Task data accesses in one of the MEM_* modes (fixed per instantiation).
// Coherent: relaxed agent-scope atomics (pairs of floats as 64-bit
// accesses) and buffer accesses with the sc1 policy, the level those atomics
// use, so values neither stay in nor come from one XCD's L2. Private: plain
// accesses; private-nt: with the non-temporal hint.
typedef float f32x4e __attribute__((ext_vector_type(4)));
typedef unsigned u32x4e __attribute__((ext_vector_type(4)));
constexpr int mem_aux(int mem) { return mem == MEM_COHERENT ? 16 : (mem == MEM_PRIVATE_NT ? 2 : 0); }

template <int MEM>
__device__ inline float ld1(const float *p) {
  if constexpr (MEM == MEM_COHERENT) return __hip_atomic_load((float *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else if constexpr (MEM == MEM_PRIVATE_NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <int MEM>
__device__ inline void st1(float *p, float v) {
  if constexpr (MEM == MEM_COHERENT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else if constexpr (MEM == MEM_PRIVATE_NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <int MEM>
__device__ inline float2 ld2(const float *p) {
  if constexpr (MEM == MEM_COHERENT) {
    const unsigned long long v =
        __hip_atomic_load((unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, v);
  } else {
    return float2{ld1<MEM>(p), ld1<MEM>(p + 1)};
  }
}

// 16-byte accesses through a buffer resource over one tile's range (the
// resource's record count also bounds the accesses to the tile). A tile is
// run by the whole workgroup, so base and size are the same in every lane;
// the task descriptor they come from is read with vector loads, though, and
// the compiler would wrap every access through a resource it cannot prove
// uniform in a per-lane loop. Taking both from the first active lane makes
// the resource scalar.
__device__ inline __amdgpu_buffer_rsrc_t tile_rsrc(const void *base, int64_t bytes) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  const int n = __builtin_amdgcn_readfirstlane((int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0, n, 0x00020000);
}
template <int MEM>
__device__ inline f32x4e ld4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(f32x4e, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, mem_aux(MEM)));
}
template <int MEM>
__device__ inline void st4(__amdgpu_buffer_rsrc_t r, uint32_t off, f32x4e v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4e, v), r, off, 0, mem_aux(MEM));
}

// Reset the mutable engine state (a kernel, so graphs hold no memset node)
// and lay out the tiles of the initially ready tasks at the front of the
// work list.
__global__ void k_engine_reset(EngineD E) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, st = gridDim.x * blockDim.x;
  for (int i = i0; i < E.ntasks; i += st) {
    st_i(&E.indeg[i], E.indeg0[i]);
    st_i(&E.tiles_done[i], 0);
    st_i(&E.task_base[i], E.init_base[i]);
  }
  for (int w = i0; w < E.total_tiles; w += st) {
    unsigned long long v = 0;
    if (w < E.init_tiles) {
      const int task = E.init_work[w];
      v = work_item(task, w - E.init_base[task]);
    }
    st_u64(&E.work[w], v);
  }
  if (i0 == 0) {
    st_i(&E.ctrl[0], E.init_tiles);
    st_i(&E.ctrl[1], 0);
    for (int q = 0; q < ENGINE_QUEUES; ++q) st_i(&E.ctrl[(q + 1) * (ENGINE_CTRL_LINE / 4)], 0);
    __hip_atomic_store(E.clock, 0ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One tile of a task, executed by the whole workgroup; `acc` collects this
// lane's contribution to the task's reduction. OP (the task's reduction, or
// RED_NONE) is a template constant so the per-element fold is one
// instruction; several chunks (rows for MATVEC) are loaded before any is
// used, to keep loads in flight.
template <int OP>
__device__ inline void fold_op(float &acc, float v) {
  if (OP != RED_NONE) acc = red_apply(OP, acc, v);
}

template <int OP, int MEM>
__device__ inline void run_tile_op(const TaskD &t, int64_t tile, float &acc) {
  constexpr int UN = 4;
  const int64_t lo = tile * t.tile;
  const int64_t hi = lo + t.tile < t.n ? lo + t.tile : t.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (t.kind == UPIR_BODY_MATVEC) {
    // same arithmetic as the loop kernel's row: lane l takes columns
    // 4l .. 4l+3 of each 256-column block in order, then a fixed tree
    const int lane = tid % WAVE, w = tid / WAVE, nw = nt / WAVE;
    auto row_dot = [&](int64_t r) {
      const float *a = t.A + r * t.lda;
      float s = 0.0f;
      for (int64_t c0 = 0; c0 < t.cols; c0 += 256) {
        const int64_t c = c0 + 4 * lane;
        if (t.vec && c + 3 < t.cols) {
          const float2 a0 = ld2<MEM>(a + c), a1 = ld2<MEM>(a + c + 2), x0 = ld2<MEM>(t.x + c), x1 = ld2<MEM>(t.x + c + 2);
          s = __builtin_fmaf(a0.x, x0.x, s);
          s = __builtin_fmaf(a0.y, x0.y, s);
          s = __builtin_fmaf(a1.x, x1.x, s);
          s = __builtin_fmaf(a1.y, x1.y, s);
        } else {
          for (int q = 0; q < 4; ++q)
            if (c + q < t.cols) s = __builtin_fmaf(ld1<MEM>(a + c + q), ld1<MEM>(t.x + c + q), s);
        }
      }
      return s;
    };
    int64_t k = lo + w;
    if (t.vec && t.cols == 256 && t.step == 1 && 4 * (hi - lo) * t.lda < (1LL << 31)) {
      // the common shape: four rows in flight per wavefront
      const int c = 4 * lane;
      const float2 x0 = ld2<MEM>(t.x + c), x1 = ld2<MEM>(t.x + c + 2);
      const __amdgpu_buffer_rsrc_t ra = tile_rsrc(t.A + (t.lb + lo) * t.lda, 4 * (hi - lo) * t.lda);
      for (; k + (UN - 1) * nw < hi; k += UN * nw) {
        f32x4e av[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) av[u] = ld4<MEM>(ra, (uint32_t)(4 * ((k + u * nw - lo) * t.lda + c)));
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          float s = 0.0f;
          s = __builtin_fmaf(av[u].x, x0.x, s);
          s = __builtin_fmaf(av[u].y, x0.y, s);
          s = __builtin_fmaf(av[u].z, x1.x, s);
          s = __builtin_fmaf(av[u].w, x1.y, s);
          s = wave_reduce(RED_SUM, s);
          if (lane == 0) {
            st1<MEM>(t.y + t.lb + k + u * nw, s);
            fold_op<OP>(acc, s);
          }
        }
      }
    }
    for (; k < hi; k += nw) {
      const int64_t r = t.lb + k * t.step;
      const float s = wave_reduce(RED_SUM, row_dot(r));
      if (lane == 0) {
        st1<MEM>(t.y + r, s);
        fold_op<OP>(acc, s);
      }
    }
    return;
  }
  if (t.vec) {  // unit step, 16-byte aligned start of every tile
    const int64_t b = t.lb + lo;
    const int64_t len = hi - lo, nc = len >> 2;
    int64_t m = tid;
    if (t.kind == UPIR_BODY_AXPY) {
      const __amdgpu_buffer_rsrc_t rx = tile_rsrc(t.x + b, 16 * nc), ry = tile_rsrc(t.y + b, 16 * nc);
      for (; m + (UN - 1) * nt < nc; m += UN * nt) {
        f32x4e xv[UN], yv[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          xv[u] = ld4<MEM>(rx, (uint32_t)(16 * (m + u * nt)));
          yv[u] = ld4<MEM>(ry, (uint32_t)(16 * (m + u * nt)));
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          f32x4e r;
          r.x = __builtin_fmaf(t.a, xv[u].x, yv[u].x);
          r.y = __builtin_fmaf(t.a, xv[u].y, yv[u].y);
          r.z = __builtin_fmaf(t.a, xv[u].z, yv[u].z);
          r.w = __builtin_fmaf(t.a, xv[u].w, yv[u].w);
          st4<MEM>(ry, (uint32_t)(16 * (m + u * nt)), r);
          fold_op<OP>(acc, r.x);
          fold_op<OP>(acc, r.y);
          fold_op<OP>(acc, r.z);
          fold_op<OP>(acc, r.w);
        }
      }
      for (; m < nc; m += nt) {
        const f32x4e xv = ld4<MEM>(rx, (uint32_t)(16 * m)), yv = ld4<MEM>(ry, (uint32_t)(16 * m));
        f32x4e r;
        r.x = __builtin_fmaf(t.a, xv.x, yv.x);
        r.y = __builtin_fmaf(t.a, xv.y, yv.y);
        r.z = __builtin_fmaf(t.a, xv.z, yv.z);
        r.w = __builtin_fmaf(t.a, xv.w, yv.w);
        st4<MEM>(ry, (uint32_t)(16 * m), r);
        fold_op<OP>(acc, r.x);
        fold_op<OP>(acc, r.y);
        fold_op<OP>(acc, r.z);
        fold_op<OP>(acc, r.w);
      }
    } else if (t.kind == UPIR_BODY_SUM) {
      const __amdgpu_buffer_rsrc_t rx = tile_rsrc(t.x + b, 16 * nc);
      for (; m + (2 * UN - 1) * nt < nc; m += 2 * UN * nt) {
        f32x4e xv[2 * UN];
#pragma unroll
        for (int u = 0; u < 2 * UN; ++u) xv[u] = ld4<MEM>(rx, (uint32_t)(16 * (m + u * nt)));
#pragma unroll
        for (int u = 0; u < 2 * UN; ++u) {
          fold_op<OP>(acc, xv[u].x);
          fold_op<OP>(acc, xv[u].y);
          fold_op<OP>(acc, xv[u].z);
          fold_op<OP>(acc, xv[u].w);
        }
      }
      for (; m < nc; m += nt) {
        const f32x4e xv = ld4<MEM>(rx, (uint32_t)(16 * m));
        fold_op<OP>(acc, xv.x);
        fold_op<OP>(acc, xv.y);
        fold_op<OP>(acc, xv.z);
        fold_op<OP>(acc, xv.w);
      }
    } else {
      for (; m < nc; m += nt)
        for (int q = 0; q < 4; ++q) atomicAdd(&t.cnt[lo + 4 * m + q], 1);
    }
    for (int64_t k = lo + 4 * nc + tid; k < hi; k += nt) {  // ragged end of the tile
      const int64_t i = t.lb + k;
      if (t.kind == UPIR_BODY_AXPY) {
        const float r = __builtin_fmaf(t.a, ld1<MEM>(t.x + i), ld1<MEM>(t.y + i));
        st1<MEM>(t.y + i, r);
        fold_op<OP>(acc, r);
      } else if (t.kind == UPIR_BODY_SUM) {
        fold_op<OP>(acc, ld1<MEM>(t.x + i));
      } else {
        atomicAdd(&t.cnt[k], 1);
      }
    }
    return;
  }
  for (int64_t k = lo + tid; k < hi; k += nt) {
    const int64_t i = t.lb + k * t.step;
    if (t.kind == UPIR_BODY_AXPY) {
      const float r = __builtin_fmaf(t.a, ld1<MEM>(t.x + i), ld1<MEM>(t.y + i));
      st1<MEM>(t.y + i, r);
      fold_op<OP>(acc, r);
    } else if (t.kind == UPIR_BODY_SUM) {
      fold_op<OP>(acc, ld1<MEM>(t.x + i));
    } else {
      atomicAdd(&t.cnt[k], 1);
    }
  }
}

template <int MEM>
__device__ inline void run_tile_mem(const TaskD &t, int64_t tile, float &acc) {
  switch (t.red_op) {
    case RED_SUM: return run_tile_op<RED_SUM, MEM>(t, tile, acc);
    case RED_MAX: return run_tile_op<RED_MAX, MEM>(t, tile, acc);
    case RED_MIN: return run_tile_op<RED_MIN, MEM>(t, tile, acc);
    default: return run_tile_op<RED_NONE, MEM>(t, tile, acc);
  }
}

__device__ inline void run_tile(const TaskD &t, int64_t tile, float &acc) {
  switch (t.mem) {
    case MEM_PRIVATE: return run_tile_mem<MEM_PRIVATE>(t, tile, acc);
    case MEM_PRIVATE_NT: return run_tile_mem<MEM_PRIVATE_NT>(t, tile, acc);
    default: return run_tile_mem<MEM_COHERENT>(t, tile, acc);
  }
}

__global__ void __launch_bounds__(256) k_engine(EngineD E) {
  __shared__ int s_task, s_tile, s_last;
  __shared__ float s_red[16];
  __shared__ double s_red64[16];
  // Work items are dealt round-robin over nq queues, each with its own claim
  // counter (one atomic per claim; a single counter for the whole chip
  // serialised the claims). Workgroup b claims from queue b mod nq, items
  // q, q + nq, q + 2 nq, ... in order. Thread 0 claims one item ahead: the
  // claim for the next item is issued before the current tile runs, so its
  // round trip overlaps the tile's memory traffic. A workgroup finishes its
  // current tile before it waits for a claimed item to be pushed, so holding
  // one claimed item per workgroup cannot stall the graph.
  const int q = (int)(blockIdx.x % (unsigned)E.nq);
  int32_t *next = &E.ctrl[(q + 1) * (ENGINE_CTRL_LINE / 4)], *reserved = &E.ctrl[0], *err = &E.ctrl[1];
  int w = 0;
  if (threadIdx.x == 0) w = q + E.nq * add_i(next, 1);
  for (;;) {
    if (threadIdx.x == 0) {
      int task = -1, tile = 0;
      if (w < E.total_tiles) {
        // wait until the push that reserves item w has filled it in
        long long spins = 0;
        int seen = -1;
        for (;;) {
          const unsigned long long v = ld_u64(&E.work[w]);
          if (v != 0) {
            task = (int)(unsigned)(v & 0xffffffffULL) - 1;
            tile = (int)(v >> 32);
            if (tile == 0 && E.tstart) E.tstart[task] = tick(E.clock);
            break;
          }
          if (ld_i(err)) break;
          const int r = ld_i(reserved);
          if (r != seen) {
            seen = r;
            spins = 0;
          }
          __builtin_amdgcn_s_sleep(2);
          if (++spins > E.spin_limit) {
            st_i(err, 1);
            break;
          }
        }
        if (task >= 0) w = q + E.nq * add_i(next, 1);
      }
      s_task = task;
      s_tile = tile;
    }
    __syncthreads();
    const int t = s_task, k = s_tile;
    if (t < 0) break;
    const TaskD &d = E.tasks[t];
    float acc = d.red_op ? red_identity<float>(d.red_op) : 0.0f;
    run_tile(d, k, acc);
    if (d.red_op) {
      const float wg = block_reduce(d.red_op, acc, s_red);
      if (threadIdx.x == 0)
        coh_store((unsigned long long *)&E.partials[d.part_base + k], __builtin_bit_cast(unsigned long long, (double)wg));
    }
    // Before the tile counts as done: a task whose data another task touches
    // has every thread's tile stores at the coherent level; otherwise only
    // the reduction partial (thread 0's store) must have landed: no other
    // task reads the data, and the kernel's end publishes it.
    if (d.mem == MEM_COHERENT || (d.red_op && threadIdx.x == 0)) complete_own_accesses();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (add_i(&E.tiles_done[t], 1) == d.ntiles - 1);
    __syncthreads();
    if (s_last) {
      if (d.red_op) {
        double v = red_identity<double>(d.red_op);
        for (int i = threadIdx.x; i < d.ntiles; i += blockDim.x)
          v = red_apply(d.red_op, v,
                        __builtin_bit_cast(double, coh_load((unsigned long long *)&E.partials[d.part_base + i])));
        v = block_reduce(d.red_op, v, s_red64);
        if (threadIdx.x == 0)
          coh_store((unsigned long long *)d.result, __builtin_bit_cast(unsigned long long, red_apply(d.red_op, d.init, v)));
      }
      if (threadIdx.x == 0) {
        if (E.tok) {
          uint64_t hsh = mix64((uint64_t)(t + 1) * 0x9E3779B97F4A7C15ULL);
          for (int i = d.pred_begin; i < d.pred_end; ++i)
            hsh = mix64(hsh ^ coh_load((unsigned long long *)&E.tok[E.pred[i]]));
          coh_store((unsigned long long *)&E.tok[t], hsh);
        }
        if (E.tdone) E.tdone[t] = tick(E.clock);
        complete_own_accesses();  // result, token and stamp before any successor starts
        for (int i = d.succ_begin; i < d.succ_end; ++i) {
          const int s = E.succ[i];
          if (add_i(&E.indeg[s], -1) == 1) {
            const int nt = E.tasks[s].ntiles;
            const int base = add_i(reserved, nt);
            for (int q = 0; q < nt; ++q) st_u64(&E.work[base + q], work_item(s, q));
          }
        }
      }
    }
    __syncthreads();
  }
}

// Token and stamps of one task of the plain executor (runs after its kernel).
__global__ void k_plain_trace(int32_t t, const int32_t *preds, int32_t np, uint64_t *tok, uint64_t *tstart,
                              uint64_t *tdone, unsigned long long *clock) {
  if (threadIdx.x != 0) return;
  if (tstart) tstart[t] = atomicAdd(clock, 1ULL);
  if (tok) {
    uint64_t h = mix64((uint64_t)(t + 1) * 0x9E3779B97F4A7C15ULL);
    for (int i = 0; i < np; ++i) h = mix64(h ^ tok[preds[i]]);
    tok[t] = h;
  }
  if (tdone) tdone[t] = atomicAdd(clock, 1ULL);
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ULL; }

}  // namespace upir

using namespace upir;

// Tile of a task in the engine: the task's own schedule tile if it gives
// one; for an AUTO schedule the graph's engine schedule (per body); else the
// default (16384 elements, 64 KiB of each array, or 64 MATVEC rows).
static int64_t task_tile(upir_loop_obj *lp, const upir_engine_sched &es) {
  if (lp->sched.tile[0] > 0) return lp->sched.tile[0];
  // a copy: engine_candidates() returns a temporary
  const upir_engine_sched use = lp->sched.policy == UPIR_SCHED_AUTO ? es : engine_candidates()[0];
  switch (lp->kind) {
    case UPIR_BODY_MATVEC: return use.rows_matvec;
    case UPIR_BODY_SUM: return use.tile_sum;
    default: return use.tile_axpy;
  }
}

// Per-context device clock for the plain executor's trace stamps.
static upir_status plain_trace_buf(upir_ctx *c, unsigned long long **clock) {
  if (!c->trace_clock) {
    c->trace_clock = upir_dalloc(c, 64);
    if (!c->trace_clock) return upir_fail(c, UPIR_ENOMEM, "trace clock");
  }
  *clock = (unsigned long long *)c->trace_clock;
  return UPIR_OK;
}

upir_status upir_plain_trace_start(upir_ctx *c) {
  unsigned long long *clock = nullptr;
  upir_status st = plain_trace_buf(c, &clock);
  if (st) return st;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, c->stream, clock);
  return UPIR_OK;
}

// Predecessor lists of every pending task, concatenated in task order, in
// one device array (the plain executor's trace kernels read their task's
// slice). Copied before any task runs and before a graph capture starts, so
// no copy or synchronisation happens while tasks are enqueued or captured.
upir_status upir_plain_trace_preds(upir_ctx *c, int32_t **dev_out, std::vector<int64_t> &offsets) {
  *dev_out = nullptr;
  const size_t n = c->tasks.size();
  offsets.assign(n + 1, 0);
  for (size_t j = 0; j < n; ++j) offsets[j + 1] = offsets[j] + (int64_t)c->tasks[j].preds.size();
  if (offsets[n] == 0) return UPIR_OK;
  if (offsets[n] >= (1LL << 31)) return upir_fail(c, UPIR_EINVAL, "too many task edges to trace");
  std::vector<int32_t> hp((size_t)offsets[n]);
  for (size_t j = 0; j < n; ++j)
    for (size_t i = 0; i < c->tasks[j].preds.size(); ++i) hp[(size_t)offsets[j] + i] = (int32_t)c->tasks[j].preds[i];
  int32_t *dp = (int32_t *)upir_dalloc(c, hp.size() * 4);
  if (!dp) return upir_fail(c, UPIR_ENOMEM, "trace preds");
  hipError_t e = hipMemcpyAsync(dp, hp.data(), hp.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    upir_dfree(c, dp);
    return upir_hipfail(c, e, "trace preds copy");
  }
  *dev_out = dp;
  return UPIR_OK;
}

// Token and stamps of task `task` after its kernel, on stream s; its
// predecessors are preds[0 .. np).
upir_status upir_plain_trace(upir_ctx *c, int64_t task, const int32_t *preds, int32_t np, hipStream_t s) {
  unsigned long long *clock = nullptr;
  upir_status st = plain_trace_buf(c, &clock);
  if (st) return st;
  hipLaunchKernelGGL(k_plain_trace, dim3(1), dim3(64), 0, s, (int32_t)task, preds, np, c->trace.tokens,
                     c->trace.start_stamp, c->trace.done_stamp, clock);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return upir_hipfail(c, e, "trace kernel");
  return UPIR_OK;
}

// The engine's device state for the pending tasks under one engine
// schedule: one allocation (tables, then mutable state) and the launch shape.
struct EnginePrep {
  unsigned char *dev = nullptr;
  EngineD E{};
  int grid = 0, rgrid = 0;
  int64_t total_tiles = 0;
};

static upir_status engine_prepare(upir_ctx *c, const upir_engine_sched &es, EnginePrep &P) {
  const int32_t n = (int32_t)c->tasks.size();
  // ---- host tables (task_graph.cpp builds and lays them out)
  std::vector<TaskD> td(n);
  std::vector<std::vector<int64_t>> preds(n);
  for (int32_t j = 0; j < n; ++j) {
    upir_loop_obj *lp = c->tasks[j].loop;
    preds[j] = c->tasks[j].preds;
    alignas(16) unsigned char pay[sizeof(MatmulP) + 16];
    upir_status st = resolve_payload(c, lp, pay);
    if (st) return st;
    TaskD &d = td[j];
    memset(&d, 0, sizeof d);
    d.kind = lp->kind;
    d.red_op = lp->has_red ? lp->red.op : 0;
    d.n = lp->n;
    d.lb = lp->loop.dim[0].lb;
    d.step = lp->loop.dim[0].step;
    if (c->tasks[j].hi >= 0) {  // a taskloop task: its block of the loop's iterations
      d.lb += c->tasks[j].lo * d.step;
      d.n = c->tasks[j].hi - c->tasks[j].lo;
    }
    d.tile = task_tile(lp, es);
    if (lp->has_red) {
      d.init = lp->red.init;
      d.result = (double *)(lp->red.result_on_host ? (void *)(lp->scratch + SCR_RESULT) : lp->red.result);
    }
    if (lp->kind == UPIR_BODY_AXPY) {
      const AxpyP &p = *(const AxpyP *)pay;
      d.a = p.a;
      d.x = p.x;
      d.y = p.y;
      d.vec = d.step == 1 && ((uintptr_t)(p.x + d.lb) % 16 == 0) && ((uintptr_t)(p.y + d.lb) % 16 == 0);
    } else if (lp->kind == UPIR_BODY_SUM) {
      const SumP &p = *(const SumP *)pay;
      if (p.dtype != UPIR_DT_F32) return upir_fail(c, UPIR_EUNSUPPORTED, "batched SUM tasks take float32 data");
      d.x = (const float *)p.x;
      d.vec = d.step == 1 && ((uintptr_t)(d.x + d.lb) % 16 == 0);
    } else if (lp->kind == UPIR_BODY_MATVEC) {
      const MatvecP &p = *(const MatvecP *)pay;
      d.A = p.A;
      d.x = p.x;
      d.y = p.y;
      d.cols = p.cols;
      d.lda = p.lda;
      d.vec = (p.lda % 4 == 0) && ((uintptr_t)p.A % 16 == 0) && ((uintptr_t)p.x % 16 == 0);
    } else {
      const CoverP &p = *(const CoverP *)pay;
      // count[k] is indexed by the loop's iteration number: a taskloop task's
      // local numbering starts at its block
      d.cnt = p.count + (c->tasks[j].hi >= 0 ? c->tasks[j].lo : 0);
      d.vec = d.step == 1 && lp->loop.dim[0].lb == 0 && (uintptr_t)d.cnt % 16 == 0;
    }
  }
  std::vector<unsigned char> host;
  EngineLayout lay{};
  std::string why;
  if (!build_engine_tables(td, preds, host, lay, why)) return upir_fail(c, UPIR_EINVAL, "task engine: %s", why.c_str());
  const int64_t total_tiles = lay.total_tiles;
  // ---- device buffer: the static image, then mutable state
  unsigned char *dev = (unsigned char *)upir_dalloc(c, lay.total_bytes);
  P.dev = dev;
  if (!dev) return upir_fail(c, UPIR_ENOMEM, "task engine tables (%zu bytes)", lay.total_bytes);
  hipError_t e = hipMemcpyAsync(dev, host.data(), lay.static_bytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    upir_dfree(c, dev);
    P.dev = nullptr;
    return upir_hipfail(c, e, "task table copy");
  }
  EngineD E{};
  E.tasks = (const TaskD *)(dev + lay.tasks);
  E.succ = (const int32_t *)(dev + lay.succ);
  E.pred = (const int32_t *)(dev + lay.pred);
  E.init_work = (const int32_t *)(dev + lay.init_work);
  E.init_base = (const int32_t *)(dev + lay.init_base);
  E.indeg0 = (const int32_t *)(dev + lay.indeg0);
  E.indeg = (int32_t *)(dev + lay.indeg);
  E.tiles_done = (int32_t *)(dev + lay.tiles_done);
  E.task_base = (int32_t *)(dev + lay.task_base);
  E.work = (unsigned long long *)(dev + lay.work);
  E.ctrl = (int32_t *)(dev + lay.ctrl);
  E.clock = (unsigned long long *)(dev + lay.ctrl + 16);
  static_assert(ENGINE_CTRL_LINE >= 24, "control line holds the counters and the clock");
  E.partials = (double *)(dev + lay.partials);
  E.ntasks = n;
  E.total_tiles = (int32_t)total_tiles;
  E.init_tiles = lay.init_tiles;
  E.tok = c->trace.tokens;
  E.tstart = c->trace.start_stamp;
  E.tdone = c->trace.done_stamp;
  E.spin_limit = 1LL << 22;
  const char *gs = getenv("UPIR_ENGINE_GRID");
  int grid = c->num_cus * 4;
  if (gs && atoi(gs) > 0) grid = atoi(gs);
  E.nq = std::min(grid, ENGINE_QUEUES);
  const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (std::max<int64_t>(n, total_tiles) + 255) / 256));
  P.E = E;
  P.grid = grid;
  P.rgrid = rgrid;
  P.total_tiles = total_tiles;
  return UPIR_OK;
}

static void engine_launch(upir_ctx *c, const EnginePrep &P) {
  hipLaunchKernelGGL(k_engine_reset, dim3(P.rgrid), dim3(256), 0, c->stream, P.E);
  hipLaunchKernelGGL(k_engine, dim3(P.grid), dim3(256), 0, c->stream, P.E);
}

// Wait for the engine and read its error flag.
static upir_status engine_check(upir_ctx *c, const EnginePrep &P) {
  hipError_t e = hipStreamSynchronize(c->stream);
  int32_t ctrl[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(ctrl, P.E.ctrl, sizeof ctrl, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return upir_hipfail(c, e, "task engine");
  if (ctrl[1]) return upir_fail(c, UPIR_EDEPEND, "task graph did not drain (%d of %d work items reserved)", ctrl[0], (int)P.total_tiles);
  return UPIR_OK;
}

upir_status upir_batched_run(upir_ctx *c, bool capture_only, upir_graph_obj **gout) {
  const int32_t n = (int32_t)c->tasks.size();
  if (n == 0) {
    if (capture_only) {
      upir_status st = upir_graph_begin(c);
      if (st) return st;
      upir_graph_h g;
      st = upir_graph_end(c, &g);
      if (st == UPIR_OK) *gout = g;
      return st;
    }
    return UPIR_OK;
  }
  upir_engine_sched es{};
  int32_t src = 0;
  upir_status st = resolve_engine_sched(c, es, src);  // before any capture: the model may run
  if (st) return st;
  EnginePrep P;
  st = engine_prepare(c, es, P);
  if (st) return st;
  if (capture_only) {
    st = upir_graph_begin(c);
    if (st) {
      upir_dfree(c, P.dev);
      return st;
    }
    engine_launch(c, P);
    const hipError_t e = hipGetLastError();
    upir_graph_h g = nullptr;
    st = upir_graph_end(c, &g);
    if (e != hipSuccess && st == UPIR_OK) {
      upir_graph_destroy(c, g);
      st = upir_hipfail(c, e, "task engine launch");
    }
    if (st == UPIR_OK) {
      g->owned.push_back(P.dev);
      *gout = g;
    } else {
      upir_dfree(c, P.dev);
    }
    return st;
  }
  engine_launch(c, P);
  const hipError_t e = hipGetLastError();
  st = e != hipSuccess ? upir_hipfail(c, e, "task engine launch") : engine_check(c, P);
  if (st) (void)hipStreamSynchronize(c->stream);
  upir_dfree(c, P.dev);
  return st;
}

extern "C" upir_status upir_tune_batched(upir_ctx *c, int32_t reps, upir_engine_sched *best, double *best_us) {
  if (!c) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "tuning during graph capture");
  if (c->tasks.empty()) return upir_fail(c, UPIR_ESTATE, "no pending tasks to tune");
  if (reps < 1 || reps > 1000) return upir_fail(c, UPIR_EINVAL, "reps");
  for (const TaskRec &t : c->tasks)
    if (!t.loop) return upir_fail(c, UPIR_EUNSUPPORTED, "data_update tasks run with taskwait PLAIN");
  upir_status st = settle(c);
  if (st) return st;
  const auto cs = engine_candidates();
  const uint64_t key = batch_key(c);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return upir_fail(c, UPIR_EHIP, "event create");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return upir_fail(c, UPIR_EHIP, "event create");
  }
  double bus = 1e300;
  int bi = -1;
  std::vector<TuneRow> rows;
  for (size_t i = 0; i < cs.size() && st == UPIR_OK; ++i) {
    EnginePrep P;
    st = engine_prepare(c, cs[i], P);
    if (st) break;
    engine_launch(c, P);  // warm-up
    st = engine_check(c, P);
    std::vector<float> ms;
    for (int r = 0; r < reps && st == UPIR_OK; ++r) {
      float t = 0;
      if (hipEventRecord(a, c->stream) != hipSuccess) st = upir_fail(c, UPIR_EHIP, "event record");
      if (st == UPIR_OK) engine_launch(c, P);
      if (st == UPIR_OK && (hipEventRecord(b, c->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                            hipEventElapsedTime(&t, a, b) != hipSuccess))
        st = upir_fail(c, UPIR_EHIP, "event wait");
      if (st == UPIR_OK) st = engine_check(c, P);
      ms.push_back(t);
    }
    (void)hipStreamSynchronize(c->stream);
    upir_dfree(c, P.dev);
    if (st) break;
    std::sort(ms.begin(), ms.end());
    const double us = 1e3 * ms[ms.size() / 2];
    TuneRow row{};
    batch_features(c, cs[i], row.feat);
    row.log2_us = (float)log2(std::max(us, 1e-3));
    row.loop_key = (int64_t)(key & 0x7FFFFFFFFFFFFFFFULL);
    rows.push_back(row);
    if (us < bus) {
      bus = us;
      bi = (int)i;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st) return st;
  // A graph row records its time relative to the default schedule (candidate
  // 0): the candidates of one graph differ by a few percent while whole
  // graphs differ by orders of magnitude, so relative costs are what the
  // model can learn to rank (and ranking is all the choice needs).
  const float base = rows[0].log2_us;
  for (TuneRow &r : rows) r.log2_us -= base;
  c->db.insert(c->db.end(), rows.begin(), rows.end());
  c->tuned_engine[key] = std::make_pair(cs[bi], bus);
  std::array<float, 12> gf;  // the candidate-independent graph features (slots 0-11)
  for (int q = 0; q < 12; ++q) gf[(size_t)q] = rows[0].feat[q];
  c->tuned_engine_graph[key] = gf;
  std::vector<float> rel(rows.size());
  for (size_t i = 0; i < rows.size(); ++i) rel[i] = rows[i].log2_us;
  c->tuned_engine_rel[key] = rel;
  if (best) *best = cs[bi];
  if (best_us) *best_us = bus;
  return UPIR_OK;
}
