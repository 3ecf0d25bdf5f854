// Internal device-side definitions shared by the runtime and the kernels.
//
// Worksharing (paper sec. 3.2): a loop of n collapsed iterations runs in an
// SPMD region of T teams (workgroups) x U units (work-items). The functions
// here enumerate the iterations a (team, unit) pair owns under each schedule;
// every kernel that honours a schedule goes through them or through a fast
// path that owns exactly the same iterations.
//
// Reduction (sec. 5; sec. 3.1 on fusing a reduction with the region's
// barrier): lane values are combined inside a wavefront by DPP steps (lane
// shuffles for a partial last wavefront), across the wavefronts of a
// workgroup through LDS, and across workgroups in float64 (or exact int64)
// by the last workgroup launched, which reads every workgroup's partial in a
// fixed order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace upir {

enum : int32_t { POL_STATIC = 0, POL_CHUNK = 1, POL_DYNAMIC = 2, POL_GUIDED = 3 };
enum : int32_t { DIST_TU = 0, DIST_T = 1, DIST_U = 2 };
enum : int32_t { RED_NONE = 0, RED_SUM = 1, RED_MAX = 2, RED_MIN = 3 };

constexpr int WAVE = 64;
constexpr int UNIT_GROUP = 4;  // consecutive points per unit slice inside a tile

struct LoopK {
  int32_t nd;
  int32_t pad_;
  int64_t lb[3], step[3], cnt[3];
  int64_t n;  // product of cnt
};

struct SchedK {
  int32_t policy, dist;
  int64_t chunk;
  int32_t tiled;
  int32_t tile[3];
  int64_t t0[3], nt[3], ntiles;  // tile grid (tiled only)
  int32_t T, U;                   // teams, units of the launch
  long long *dyn_next;            // DYNAMIC / GUIDED claim counter (self-resetting)
  unsigned *dyn_exit;             // workgroups that finished claiming
};

// A reduction whose cross-workgroup fold was deferred: the partial values
// (float64 or int64 bits) a finished kernel left behind, and where the
// folded result goes. count == 0: nothing pending.
struct FoldK {
  const unsigned long long *part;
  long long count;
  int32_t op, is_int;
  double init;
  long long init_i;
  void *result;
};

struct RedK {
  int32_t op;                 // RED_*
  int32_t is_int;             // accumulate exactly in int64
  double init;
  long long init_i;
  void *result;               // device double* or long long*
  unsigned long long *slots;  // two words per workgroup: value, flag
  long long spin_limit;       // bound on the combiner's wait per slot
  unsigned long long *defer;  // non-null: leave one partial per wavefront here, fold later
  FoldK fold;                 // an earlier loop's deferred fold, run by one workgroup
};

// Empty float slot: all ones, a NaN that neither arithmetic nor a float32 to
// float64 conversion produces. Integer slots carry a separate flag word.
// Each workgroup's slot has a 128-byte cache line of its own: device-coherent
// stores to one line from many workgroups are serialised.
constexpr unsigned long long SLOT_EMPTY = ~0ULL;
constexpr int SLOT_WORDS = 16;  // 64-bit words between slots

// ------------------------------------------------------------------ helpers
__host__ __device__ inline void block_range(int64_t n, int64_t parts, int64_t p, int64_t &lo, int64_t &hi) {
  int64_t q = n / parts, r = n % parts;
  lo = p * q + (p < r ? p : r);
  hi = lo + q + (p < r ? 1 : 0);
}

// Team id of this workgroup. Teams are logical; hardware hands workgroups
// to the 8 XCDs round-robin, so consecutive team ids are placed on the same
// XCD (each XCD owns a contiguous run of team ids) to share its L2.
__device__ inline int xcd_team(int b, int G) {
  const int X = 8;
  int q = G / X, r = G % X;
  int x = b % X, i = b / X;
  int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return base + i;
}

// Collapsed index -> induction values (row-major).
__device__ inline void decode(const LoopK &L, int64_t k, int64_t iv[3]) {
  if (L.nd == 1) {
    iv[0] = L.lb[0] + k * L.step[0];
  } else if (L.nd == 2) {
    int64_t a = k / L.cnt[1], b = k - a * L.cnt[1];
    iv[0] = L.lb[0] + a * L.step[0];
    iv[1] = L.lb[1] + b * L.step[1];
  } else {
    int64_t c = k % L.cnt[2];
    int64_t t = k / L.cnt[2];
    int64_t b = t % L.cnt[1];
    int64_t a = t / L.cnt[1];
    iv[0] = L.lb[0] + a * L.step[0];
    iv[1] = L.lb[1] + b * L.step[1];
    iv[2] = L.lb[2] + c * L.step[2];
  }
}

// Visit k in [lo, hi) with induction values advanced as an odometer.
template <class F>
__device__ inline void visit_range(const LoopK &L, int64_t lo, int64_t hi, F &f) {
  if (lo >= hi) return;
  int64_t iv[3] = {0, 0, 0};
  int64_t idx[3] = {0, 0, 0};
  int64_t r = lo;
  for (int d = L.nd - 1; d >= 0; --d) {
    idx[d] = r % L.cnt[d];
    r /= L.cnt[d];
    iv[d] = L.lb[d] + idx[d] * L.step[d];
  }
  for (int64_t k = lo; k < hi; ++k) {
    f(k, iv);
    for (int d = L.nd - 1; d >= 0; --d) {
      ++idx[d];
      iv[d] += L.step[d];
      if (idx[d] < L.cnt[d]) break;
      idx[d] = 0;
      iv[d] = L.lb[d];
    }
  }
}

// Every iteration owned by (team, unit) under static / static-chunk (untiled).
template <class F>
__device__ inline void for_owned_untiled(const LoopK &L, const SchedK &S, int team, int unit, F &f) {
  const int64_t n = L.n;
  if (S.policy == POL_STATIC) {
    if (S.dist == DIST_U) {
      int64_t lo, hi;
      block_range(n, S.U, unit, lo, hi);
      visit_range(L, lo, hi, f);
      return;
    }
    int64_t tlo, thi;
    block_range(n, S.T, team, tlo, thi);
    if (S.dist == DIST_T) {
      if (unit == 0) visit_range(L, tlo, thi, f);
      return;
    }
    int64_t ulo, uhi;
    block_range(thi - tlo, S.U, unit, ulo, uhi);
    visit_range(L, tlo + ulo, tlo + uhi, f);
  } else {  // POL_CHUNK
    // first chunk and chunk stride of this unit; selected without nested
    // branches (an if / else-if chain here was compiled into code that ran
    // no iteration for distribute(units) on gfx950)
    const int64_t c = S.chunk;
    const bool tu = S.dist == DIST_TU, tt = S.dist == DIST_T;
    if (tt && unit != 0) return;
    const int64_t first = tu ? (int64_t)team * S.U + unit : (tt ? (int64_t)team : (int64_t)unit);
    const int64_t stride = tu ? (int64_t)S.T * S.U : (tt ? (int64_t)S.T : (int64_t)S.U);
    for (int64_t m = first; m * c < n; m += stride) {
      int64_t lo = m * c, hi = lo + c < n ? lo + c : n;
      visit_range(L, lo, hi, f);
    }
  }
}

// Tiled schedules: tiles -> teams by policy, 4-point groups -> units.
template <class F>
__device__ inline void for_owned_tile(const LoopK &L, const SchedK &S, int64_t m, int unit, F &f) {
  int64_t tc[3] = {0, 0, 0};
  int64_t rem = m;
  for (int d = L.nd - 1; d >= 0; --d) {
    tc[d] = S.t0[d] + rem % S.nt[d];
    rem /= S.nt[d];
  }
  int64_t vol = 1;
  for (int d = 0; d < L.nd; ++d) vol *= S.tile[d];
  for (int64_t g = unit; g * UNIT_GROUP < vol; g += S.U) {
    for (int q = 0; q < UNIT_GROUP; ++q) {
      int64_t p = g * UNIT_GROUP + q;
      if (p >= vol) break;
      int64_t off[3] = {0, 0, 0};
      int64_t pr = p;
      for (int d = L.nd - 1; d >= 0; --d) {
        off[d] = pr % S.tile[d];
        pr /= S.tile[d];
      }
      int64_t iv[3] = {0, 0, 0};
      bool in = true;
      int64_t k = 0;
      for (int d = 0; d < L.nd; ++d) {
        iv[d] = tc[d] * S.tile[d] + off[d];
        int64_t ub = L.lb[d] + L.cnt[d];  // unit steps
        in = in && iv[d] >= L.lb[d] && iv[d] < ub;
        k = k * L.cnt[d] + (iv[d] - L.lb[d]);
      }
      if (in) f(k, iv);
    }
  }
}

template <class F>
__device__ inline void for_owned_tiled(const LoopK &L, const SchedK &S, int team, int unit, F &f) {
  if (S.policy == POL_STATIC) {
    int64_t lo, hi;
    block_range(S.ntiles, S.T, team, lo, hi);
    for (int64_t m = lo; m < hi; ++m) for_owned_tile(L, S, m, unit, f);
  } else {
    const int64_t c = S.chunk;
    for (int64_t m0 = (int64_t)team * c; m0 < S.ntiles; m0 += (int64_t)S.T * c)
      for (int64_t m = m0; m < m0 + c && m < S.ntiles; ++m) for_owned_tile(L, S, m, unit, f);
  }
}

// ---------------------------------------------------- wavefront reductions
template <class T> struct OpSum { __device__ static T apply(T a, T b) { return a + b; } };
template <class T> struct OpMax { __device__ static T apply(T a, T b) { return a > b ? a : b; } };
template <class T> struct OpMin { __device__ static T apply(T a, T b) { return a < b ? a : b; } };

template <class T>
__device__ inline T red_apply(int op, T a, T b) {
  if (op == RED_SUM) return a + b;
  if (op == RED_MAX) return a > b ? a : b;
  return a < b ? a : b;
}

template <class T>
__device__ inline T red_identity(int op);
template <> __device__ inline float red_identity<float>(int op) {
  return op == RED_SUM ? 0.0f : (op == RED_MAX ? -__builtin_inff() : __builtin_inff());
}
template <> __device__ inline double red_identity<double>(int op) {
  return op == RED_SUM ? 0.0 : (op == RED_MAX ? -__builtin_inf() : __builtin_inf());
}
template <> __device__ inline long long red_identity<long long>(int op) {
  return op == RED_SUM ? 0LL : (op == RED_MAX ? (long long)0x8000000000000000ULL : 0x7FFFFFFFFFFFFFFFLL);
}

// Lane v moved by one DPP step; lanes the row mask leaves out get `id`.
template <int CTRL, int RM, class T>
__device__ inline T dpp_move(T v, T id) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, id), __builtin_bit_cast(int, v), CTRL, RM, 0xF, false));
  } else {
    const unsigned long long vb = __builtin_bit_cast(unsigned long long, v), ib = __builtin_bit_cast(unsigned long long, id);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)ib, (int)(unsigned)vb, CTRL, RM, 0xF, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(ib >> 32), (int)(unsigned)(vb >> 32), CTRL, RM, 0xF, false);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}
template <class T>
__device__ inline T read_lane63(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), WAVE - 1));
  } else {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, WAVE - 1);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), WAVE - 1);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// Reduction over the lanes of a wavefront, returned to every lane; a fixed
// tree, so the result is deterministic. Wavefronts of a workgroup made of
// whole wavefronts (every lane present) use DPP steps: pairs and quads, the
// two halves of each row of 16 lanes, then rows 0 + 1 and 2 + 3 and finally
// all four rows into lane 63. The last wavefront of any other workgroup has
// only `act` < 64 lanes (lanes 0 .. act-1); there a butterfly over lane
// shuffles (xor 32, 16, ..., 1) takes the op's identity for every partner
// lane >= act (such a lane does not exist and its register is undefined), so
// lane 0 ends with the reduction over the present lanes, which is then read
// back from lane 0 by every lane.
template <class T>
__device__ inline T wave_reduce(int op, T v) {
  const T id = red_identity<T>(op);
  if (blockDim.x % WAVE == 0) {
    v = red_apply(op, v, dpp_move<0xB1, 0xF>(v, id));   // quad_perm [1,0,3,2]
    v = red_apply(op, v, dpp_move<0x4E, 0xF>(v, id));   // quad_perm [2,3,0,1]
    v = red_apply(op, v, dpp_move<0x141, 0xF>(v, id));  // row_half_mirror
    v = red_apply(op, v, dpp_move<0x140, 0xF>(v, id));  // row_mirror
    v = red_apply(op, v, dpp_move<0x142, 0xA>(v, id));  // row_bcast:15 into rows 1 and 3
    v = red_apply(op, v, dpp_move<0x143, 0xC>(v, id));  // row_bcast:31 into rows 2 and 3
    return read_lane63(v);
  }
  const int lane = (int)(threadIdx.x % WAVE);
  const int first = (int)(threadIdx.x - (unsigned)lane);
  const int act = (int)blockDim.x - first < WAVE ? (int)blockDim.x - first : WAVE;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const T o = __shfl_xor(v, s, WAVE);
    v = red_apply(op, v, (lane ^ s) < act ? o : id);
  }
  return __shfl(v, 0, WAVE);
}

// Block reduce: every thread passes its value; returns the block value in
// thread 0 (other threads get an unspecified value). `lds` holds >= 16 T.
template <class T>
__device__ inline T block_reduce(int op, T v, T *lds) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int nw = (blockDim.x + WAVE - 1) / WAVE;
  v = wave_reduce(op, v);
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  T r = red_identity<T>(op);
  if (threadIdx.x < WAVE) {
    r = (int)threadIdx.x < nw ? lds[threadIdx.x] : red_identity<T>(op);
    r = wave_reduce(op, r);
  }
  return r;
}

// Device-coherent accesses. The XCDs' L2 caches are not coherent with each
// other; atomic accesses at agent scope are performed at the device-coherent
// level, so values published through them need no L2 write-back.
// complete_own_accesses() waits until this thread's earlier memory
// operations have completed (a coherent store has then reached the
// device-coherent level), which orders a published value before the counter
// update that announces it. A workgroup-scope fence alone does not do this:
// it emits no wait for global stores, because within one workgroup the
// stores are already ordered. The agent-scope release fence would add a
// write-back of the whole L2 of the XCD, about a microsecond per fence.
__device__ inline void coh_store(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long coh_load(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void complete_own_accesses() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // no compiler reordering across this point
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");        // loads and stores of this thread complete
}
__device__ inline unsigned ticket_add(unsigned *t) {
  return __hip_atomic_fetch_add(t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-workgroup combine. Every workgroup but the last one launched
// publishes its value in its slot with one device-coherent store and
// retires. The last workgroup (launched last, so the others are already
// running or done) waits for every slot in turn, folds them in workgroup
// order (each thread a fixed stride, then a fixed tree), adds `init`,
// writes the result and empties the slots for the next launch. Integer
// values are followed by a flag word, written after the value has
// completed; float values mark their own slot, since an empty slot holds a
// NaN pattern no float value takes. Waits are bounded (a NaN result reports
// a slot that never arrived).
template <class T>
__device__ inline void combine_slots(const RedK &R, T wg, T *lds) {
  constexpr bool INT = std::is_same<T, long long>::value;
  const int G = gridDim.x, b = blockIdx.x;
  unsigned long long *sl = R.slots;
  if (b != G - 1) {
    if (threadIdx.x == 0) {
      coh_store(&sl[SLOT_WORDS * b], __builtin_bit_cast(unsigned long long, wg));
      if (INT) {
        complete_own_accesses();
        coh_store(&sl[SLOT_WORDS * b + 1], 1ULL);
      }
    }
    return;
  }
  __shared__ int s_missing;
  if (threadIdx.x == 0) s_missing = 0;
  __syncthreads();
  // Each thread folds slots tid, tid + U, tid + 2U, ... in that order. The
  // slots of a batch are loaded together (one memory round trip for the
  // batch); only slots that are still empty are polled again.
  constexpr int BATCH = 8;
  const int U = blockDim.x;
  T v = red_identity<T>(R.op);
  for (int i0 = threadIdx.x; i0 < G - 1; i0 += BATCH * U) {
    unsigned long long bits[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = i0 + q * U;
      bits[q] = i < G - 1 ? coh_load(&sl[SLOT_WORDS * i + (INT ? 1 : 0)]) : 0ULL;
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = i0 + q * U;
      if (i >= G - 1) break;
      long long spins = 0;
      while (INT ? bits[q] == 0ULL : bits[q] == SLOT_EMPTY) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > R.spin_limit) {
          s_missing = 1;
          break;
        }
        bits[q] = coh_load(&sl[SLOT_WORDS * i + (INT ? 1 : 0)]);
      }
    }
    if (INT) {  // flags seen: now the values
#pragma unroll
      for (int q = 0; q < BATCH; ++q) {
        const int i = i0 + q * U;
        if (i < G - 1) bits[q] = coh_load(&sl[SLOT_WORDS * i]);
      }
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = i0 + q * U;
      if (i >= G - 1) break;
      v = red_apply(R.op, v, __builtin_bit_cast(T, bits[q]));
      coh_store(&sl[SLOT_WORDS * i], INT ? 0ULL : SLOT_EMPTY);
      if (INT) coh_store(&sl[SLOT_WORDS * i + 1], 0ULL);
    }
  }
  if (threadIdx.x == 0) v = red_apply(R.op, v, wg);  // this workgroup's own value, last
  v = block_reduce(R.op, v, lds);
  if (threadIdx.x == 0) {
    if constexpr (std::is_same<T, double>::value) {
      *(double *)R.result = s_missing ? __builtin_nan("") : red_apply(R.op, R.init, v);
    } else {
      *(long long *)R.result = red_apply(R.op, R.init_i, v);
    }
  }
}

__device__ inline void combine_f64(const RedK &R, double wg, double *lds) { combine_slots<double>(R, wg, lds); }
__device__ inline void combine_i64(const RedK &R, long long wg, long long *lds) { combine_slots<long long>(R, wg, lds); }

// Deferred finish: one partial per wavefront, stored at
// defer[workgroup * wavefronts-per-workgroup + wavefront]; no barrier and no
// cross-workgroup traffic in this kernel.
template <class T>
__device__ inline void defer_partial(const RedK &R, T lane) {
  const T w = wave_reduce(R.op, lane);
  if (threadIdx.x % WAVE == 0) {
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    unsigned long long bits;
    if constexpr (std::is_same<T, long long>::value) bits = (unsigned long long)w;
    else bits = __builtin_bit_cast(unsigned long long, (double)w);
    R.defer[(long long)blockIdx.x * nw + threadIdx.x / WAVE] = bits;
  }
}

// Lane value -> workgroup value -> cross-workgroup combine.
template <class A>
__device__ inline void finish_reduction(const RedK &R, A lane);

template <>
__device__ inline void finish_reduction<float>(const RedK &R, float lane) {
  if (R.defer) return defer_partial<float>(R, lane);
  __shared__ float lf[16];
  __shared__ double ld[16];
  float wg = block_reduce(R.op, lane, lf);
  combine_f64(R, (double)wg, ld);
}
template <>
__device__ inline void finish_reduction<double>(const RedK &R, double lane) {
  if (R.defer) return defer_partial<double>(R, lane);
  __shared__ double ld[16];
  double wg = block_reduce(R.op, lane, ld);
  combine_f64(R, wg, ld);
}
template <>
__device__ inline void finish_reduction<long long>(const RedK &R, long long lane) {
  if (R.defer) return defer_partial<long long>(R, lane);
  __shared__ long long li[16];
  long long wg = block_reduce(R.op, lane, li);
  combine_i64(R, wg, li);
}

// Fold of a deferred reduction by one whole workgroup: thread t takes
// partials t, t + U, ... in order, then a fixed tree; `init` is applied
// once. A thread's partials are loaded FB at a time, all in flight
// together. The partials were written by an earlier kernel on the same
// stream, so plain loads see them.
template <class V>
__device__ inline V fold_value(unsigned long long b) {
  if constexpr (std::is_same<V, long long>::value) return (long long)b;
  else return __builtin_bit_cast(double, b);
}

template <class V>
__device__ inline void fold_typed(const FoldK &F, V *lds) {
  constexpr int FB = 8;
  const long long U = blockDim.x;
  V v = red_identity<V>(F.op);
  unsigned long long b[FB];
  for (long long i0 = threadIdx.x; i0 < F.count; i0 += FB * U) {
#pragma unroll
    for (int q = 0; q < FB; ++q) b[q] = i0 + q * U < F.count ? F.part[i0 + q * U] : 0ULL;
#pragma unroll
    for (int q = 0; q < FB; ++q)
      if (i0 + q * U < F.count) v = red_apply(F.op, v, fold_value<V>(b[q]));
  }
  v = block_reduce(F.op, v, lds);
  if (threadIdx.x == 0) {
    if constexpr (std::is_same<V, long long>::value) *(long long *)F.result = red_apply(F.op, F.init_i, v);
    else *(double *)F.result = red_apply(F.op, F.init, v);
  }
}

__device__ inline void run_fold(const FoldK &F) {
  __shared__ double fd[16];
  __shared__ long long fi[16];
  if (F.is_int) fold_typed<long long>(F, fi);
  else fold_typed<double>(F, fd);
}

// The tiled Jacobi kernel launches one extra workgroup for its
// cross-workgroup work: an earlier loop's fold, its own synchronous combine.
__host__ __device__ inline bool jacobi_extra_wg(const RedK &R) {
  return R.fold.count > 0 || (R.op != RED_NONE && R.defer == nullptr);
}

// Called by every thread at the very end of a loop kernel: workgroup 0 runs
// the fold an earlier loop deferred, after its own work. (The streaming and
// Jacobi kernels give the fold an extra workgroup instead, which runs beside
// the others rather than at the end of workgroup 0.)
__device__ inline void fold_hook(const RedK &R) {
  if (R.fold.count > 0 && blockIdx.x == 0) run_fold(R.fold);
}

}  // namespace upir
