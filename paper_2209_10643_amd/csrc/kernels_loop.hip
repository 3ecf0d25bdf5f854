// Worksharing-loop kernels for the built-in bodies (gfx950).
//
// Paper: sec. 3.2 (canonical loop + worksharing with schedule, distribute and
// collapse inside an SPMD region), sec. 5 (reduction), sec. 6 (the AXPY loop
// body; matrix-vector, matrix multiplication and stencil kernels).
//
// Two kinds of kernels:
//  * k_generic<Body>: executes exactly the iterations each (team, unit) owns
//    under any static / static-chunk / tiled schedule, any distribute and
//    collapse 1..3, decoding induction values as it goes. Correct for every
//    body, used for anything the fast kernels do not cover.
//  * fast kernels that own the same iterations with wide, coalesced access:
//    k_stream4 (1-D, chunk 4: one f32x4 per chunk, chunks dealt over the
//    flat unit id -- the classic grid-stride loop), k_jacobi_tile (tiles of
//    TH x 256 points; each wavefront streams a strip of rows through
//    registers, west / east neighbours from adjacent lanes, no LDS),
//    k_filter7_tile (the same strips for the 7 x 7 filter), k_matvec (one
//    64-lane wavefront per row).
// All kernels fuse their reduction (lane -> wavefront -> LDS -> last
// workgroup combines in float64 in workgroup order).
#include "upir_launch.h"

namespace upir {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ body functors
struct BAxpy {
  using Acc = float;
  AxpyP p;
  __device__ void operator()(int64_t, const int64_t *iv, int, int, Acc &acc, int op) const {
    const int64_t i = iv[0];
    const float v = __builtin_fmaf(p.a, p.x[i], p.y[i]);
    p.y[i] = v;
    if (op) acc = red_apply(op, acc, v);
  }
};

template <class T, class A>
struct BSum {
  using Acc = A;
  const T *x;
  __device__ void operator()(int64_t, const int64_t *iv, int, int, Acc &acc, int op) const {
    acc = red_apply(op, acc, (A)x[iv[0]]);
  }
};

struct BJacobi {
  using Acc = double;
  JacobiP p;
  __device__ void operator()(int64_t, const int64_t *iv, int, int, Acc &acc, int op) const {
    const int64_t i = iv[0], j = iv[1], ld = p.ld;
    const float *s = p.src;
    const float v = ((s[(i - 1) * ld + j] + s[(i + 1) * ld + j]) + (s[i * ld + j - 1] + s[i * ld + j + 1])) * 0.25f;
    p.dst[i * ld + j] = v;
    if (op) acc = red_apply(op, acc, fabs((double)v - (double)s[i * ld + j]));
  }
};

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

struct BMatmul {
  using Acc = float;
  MatmulP p;
  __device__ void operator()(int64_t, const int64_t *iv, int, int, Acc &, int) const {
    const int64_t i = iv[0], j = iv[1];
    float acc = 0.0f;
    if (p.kind == 4) {
      for (int64_t k = 0; k < p.K; ++k) acc = __builtin_fmaf(p.A[i * p.lda + k], p.B[k * p.ldb + j], acc);
    } else if (p.kind == 5) {
      for (int64_t k = 0; k < p.K; ++k)
        acc = __builtin_fmaf(bf16_to_f32(p.ah[i * p.K + k]), bf16_to_f32(p.bh[j * p.K + k]), acc);
    } else {
      for (int64_t k = 0; k < p.K; ++k) {
        const float ah = bf16_to_f32(p.ah[i * p.K + k]), al = bf16_to_f32(p.al[i * p.K + k]);
        const float bh = bf16_to_f32(p.bh[j * p.K + k]), bl = bf16_to_f32(p.bl[j * p.K + k]);
        acc = __builtin_fmaf(al, bh, acc);
        acc = __builtin_fmaf(ah, bl, acc);
        acc = __builtin_fmaf(ah, bh, acc);
      }
    }
    p.C[i * p.ldc + j] = acc;
  }
};

// 7 x 7 filter, one point: the fused multiply-add chain of the definition.
struct BFilter7 {
  using Acc = float;
  Filter7P p;
  __device__ void operator()(int64_t, const int64_t *iv, int, int, Acc &, int) const {
    const int64_t i = iv[0], j = iv[1], ld = p.ld;
    float s = 0.0f;
    for (int m = 0; m < 7; ++m)
      for (int n = 0; n < 7; ++n) s = __builtin_fmaf(p.w[m * 7 + n], p.src[(i + m - 3) * ld + j + n - 3], s);
    p.dst[i * ld + j] = s;
  }
};

struct BOwner {
  using Acc = float;
  OwnerP p;
  int U;
  __device__ void operator()(int64_t k, const int64_t *, int team, int unit, Acc &, int) const {
    p.out[k] = team * U + unit;
  }
};

struct BCover {
  using Acc = float;
  CoverP p;
  __device__ void operator()(int64_t k, const int64_t *, int, int, Acc &, int) const {
    atomicAdd(&p.count[k], 1);
  }
};

// ----------------------------------------------------------- generic kernel
template <class B>
__global__ void __launch_bounds__(1024) k_generic(LoopK L, SchedK S, RedK R, B body) {
  using A = typename B::Acc;
  const int team = blockIdx.x, unit = threadIdx.x;
  A acc = red_identity<A>(R.op ? R.op : RED_SUM);
  auto f = [&](int64_t k, const int64_t *iv) { body(k, iv, team, unit, acc, R.op); };
  if (S.tiled)
    for_owned_tiled(L, S, team, unit, f);
  else
    for_owned_untiled(L, S, team, unit, f);
  if (R.op != RED_NONE) finish_reduction<A>(R, acc);
  fold_hook(R);
}

// Dynamic / guided: each team claims a range of iterations from a device
// counter and splits it among its units in near-equal blocks. The last team
// to finish re-arms the counter so graph replays start from zero.
template <class B>
__global__ void __launch_bounds__(1024) k_dynamic(LoopK L, SchedK S, RedK R, B body) {
  using A = typename B::Acc;
  __shared__ long long s_lo, s_hi;
  const int team = blockIdx.x, unit = threadIdx.x;
  A acc = red_identity<A>(R.op ? R.op : RED_SUM);
  auto f = [&](int64_t k, const int64_t *iv) { body(k, iv, team, unit, acc, R.op); };
  const long long n = L.n;
  for (;;) {
    if (threadIdx.x == 0) {
      long long lo, hi;
      if (S.policy == POL_DYNAMIC) {
        long long len = S.chunk * (long long)S.U;
        lo = atomicAdd((unsigned long long *)S.dyn_next, (unsigned long long)len);
        hi = lo + len < n ? lo + len : n;
      } else {  // guided: claim max(chunk*U, remaining / (2T))
        long long cur = __hip_atomic_load(S.dyn_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
          if (cur >= n) { lo = hi = n; break; }
          long long rem = n - cur;
          long long len = rem / (2LL * S.T);
          long long mn = S.chunk * (long long)S.U;
          if (len < mn) len = mn;
          long long want = cur + len < n ? cur + len : n;
          if (__hip_atomic_compare_exchange_strong(S.dyn_next, &cur, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)) {
            lo = cur;
            hi = want;
            break;
          }
        }
      }
      s_lo = lo < n ? lo : n;
      s_hi = hi;
    }
    __syncthreads();
    const long long lo = s_lo, hi = s_hi;
    __syncthreads();
    if (lo >= hi) break;
    int64_t ulo, uhi;
    block_range(hi - lo, S.U, unit, ulo, uhi);
    visit_range(L, lo + ulo, lo + uhi, f);
  }
  if (threadIdx.x == 0) {
    // every claim of this team is done; the last team re-arms both counters
    unsigned t = ticket_add(S.dyn_exit);
    if (t == gridDim.x - 1) {
      __hip_atomic_store(S.dyn_next, 0LL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(S.dyn_exit, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (R.op != RED_NONE) finish_reduction<A>(R, acc);
  fold_hook(R);
}

template <class B>
static hipError_t go_generic(const B &b, const LoopK &L, const SchedK &S, const RedK &R, hipStream_t st) {
  if (S.policy == POL_DYNAMIC || S.policy == POL_GUIDED)
    hipLaunchKernelGGL(k_dynamic<B>, dim3(S.T), dim3(S.U), 0, st, L, S, R, b);
  else
    hipLaunchKernelGGL(k_generic<B>, dim3(S.T), dim3(S.U), 0, st, L, S, R, b);
  return hipGetLastError();
}

hipError_t launch_generic(int32_t body, const void *payload, const LoopK &L, const SchedK &S, const RedK &R,
                          hipStream_t st) {
  switch (body) {
    case 1: return go_generic(BAxpy{*(const AxpyP *)payload}, L, S, R, st);
    case 2: {
      const SumP &p = *(const SumP *)payload;
      switch (p.dtype) {
        case 1: return go_generic(BSum<float, float>{(const float *)p.x}, L, S, R, st);
        case 2: return go_generic(BSum<double, double>{(const double *)p.x}, L, S, R, st);
        case 3: return go_generic(BSum<int32_t, long long>{(const int32_t *)p.x}, L, S, R, st);
        case 4: return go_generic(BSum<long long, long long>{(const long long *)p.x}, L, S, R, st);
      }
      return hipErrorInvalidValue;
    }
    case 3: return go_generic(BJacobi{*(const JacobiP *)payload}, L, S, R, st);
    case 4:
    case 5:
    case 6: return go_generic(BMatmul{*(const MatmulP *)payload}, L, S, R, st);
    case 8: return go_generic(BOwner{*(const OwnerP *)payload, S.U}, L, S, R, st);
    case 9: return go_generic(BCover{*(const CoverP *)payload}, L, S, R, st);
    case 10: return go_generic(BFilter7{*(const Filter7P *)payload}, L, S, R, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------- 1-D streaming, chunk 4
// Ownership: chunk m (4 iterations) belongs to flat unit m mod (T U), flat =
// team U + unit, exactly the static-chunk-4 schedule. x and y point at the
// element of the first iteration and are 16-byte aligned. Four owned chunks
// of each input (eight for SUM) are loaded before any is used to keep
// several loads in flight. NT: loads and stores carry the non-temporal hint
// (streamed through rather than kept).
template <bool NT>
__device__ __forceinline__ f32x4 ld4(const f32x4 *p) {
  if (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT>
__device__ __forceinline__ void st4(f32x4 *p, f32x4 v) {
  if (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// OP is the reduction (RED_NONE for none), fixed at compile time so the
// per-element fold is one instruction.
// An earlier loop's deferred fold gets one extra workgroup, launched last and
// given no chunks: it runs beside the others instead of after workgroup 0's
// own chunks (which put the fold's memory round trips on the kernel's
// critical path, about 2 us of a 4 us loop at 2^20). When this loop's own
// reduction is synchronous, that workgroup is also the combiner.
template <int BODY, int OP, bool NT>
__global__ void __launch_bounds__(1024) k_stream4(int64_t n, float a, const float *__restrict__ x,
                                                  float *__restrict__ y, int32_t *__restrict__ cnt, RedK R) {
  constexpr bool RED = OP != RED_NONE;
  const bool xwg = R.fold.count > 0;
  const int G = xwg ? (int)gridDim.x - 1 : (int)gridDim.x;  // workgroups that take chunks
  if (xwg && (int)blockIdx.x == G) {
    run_fold(R.fold);
    if (RED && !R.defer) finish_reduction<float>(R, red_identity<float>(OP));
    return;
  }
  const int64_t F = (int64_t)G * blockDim.x;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nc = n >> 2;
  float acc = RED ? red_identity<float>(OP) : 0.0f;
  const f32x4 *x4 = (const f32x4 *)x;
  f32x4 *y4 = (f32x4 *)y;
  auto fold = [&](float v) {
    if (RED) acc = red_apply(OP, acc, v);
  };
  int64_t m = f;
  if (BODY == 1) {  // AXPY
    for (; m + 3 * F < nc; m += 4 * F) {
      f32x4 xv[4], yv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xv[u] = ld4<NT>(&x4[m + u * F]);
        yv[u] = ld4<NT>(&y4[m + u * F]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        f32x4 r;
        r.x = __builtin_fmaf(a, xv[u].x, yv[u].x);
        r.y = __builtin_fmaf(a, xv[u].y, yv[u].y);
        r.z = __builtin_fmaf(a, xv[u].z, yv[u].z);
        r.w = __builtin_fmaf(a, xv[u].w, yv[u].w);
        st4<NT>(&y4[m + u * F], r);
        fold(r.x); fold(r.y); fold(r.z); fold(r.w);
      }
    }
    for (; m < nc; m += F) {
      f32x4 xv = x4[m], yv = y4[m];
      f32x4 r;
      r.x = __builtin_fmaf(a, xv.x, yv.x);
      r.y = __builtin_fmaf(a, xv.y, yv.y);
      r.z = __builtin_fmaf(a, xv.z, yv.z);
      r.w = __builtin_fmaf(a, xv.w, yv.w);
      y4[m] = r;
      fold(r.x); fold(r.y); fold(r.z); fold(r.w);
    }
    if ((n & 3) && f == nc % F) {
      for (int64_t i = nc * 4; i < n; ++i) {
        float r = __builtin_fmaf(a, x[i], y[i]);
        y[i] = r;
        fold(r);
      }
    }
  } else if (BODY == 2) {  // SUM over float32: eight chunks in flight (one input stream)
    for (; m + 7 * F < nc; m += 8 * F) {
      f32x4 xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = ld4<NT>(&x4[m + u * F]);
#pragma unroll
      for (int u = 0; u < 8; ++u) { fold(xv[u].x); fold(xv[u].y); fold(xv[u].z); fold(xv[u].w); }
    }
    for (; m < nc; m += F) {
      f32x4 xv = x4[m];
      fold(xv.x); fold(xv.y); fold(xv.z); fold(xv.w);
    }
    if ((n & 3) && f == nc % F)
      for (int64_t i = nc * 4; i < n; ++i) fold(x[i]);
  } else {  // COVER: count[k] += 1
    for (; m < nc; m += F) {
#pragma unroll
      for (int q = 0; q < 4; ++q) atomicAdd(&cnt[4 * m + q], 1);
    }
    if ((n & 3) && f == nc % F)
      for (int64_t i = nc * 4; i < n; ++i) atomicAdd(&cnt[i], 1);
  }
  if (RED) finish_reduction<float>(R, acc);
}

template <int BODY, int OP>
static void go_stream4(bool nt, dim3 g, dim3 b, hipStream_t st, int64_t n, float a, const float *x, float *y,
                       int32_t *cnt, const RedK &R) {
  if (nt)
    hipLaunchKernelGGL((k_stream4<BODY, OP, true>), g, b, 0, st, n, a, x, y, cnt, R);
  else
    hipLaunchKernelGGL((k_stream4<BODY, OP, false>), g, b, 0, st, n, a, x, y, cnt, R);
}

template <int BODY>
static void go_stream4_op(bool nt, dim3 g, dim3 b, hipStream_t st, int64_t n, float a, const float *x, float *y,
                          int32_t *cnt, const RedK &R) {
  switch (R.op) {
    case RED_SUM: return go_stream4<BODY, RED_SUM>(nt, g, b, st, n, a, x, y, cnt, R);
    case RED_MAX: return go_stream4<BODY, RED_MAX>(nt, g, b, st, n, a, x, y, cnt, R);
    case RED_MIN: return go_stream4<BODY, RED_MIN>(nt, g, b, st, n, a, x, y, cnt, R);
    default: return go_stream4<BODY, RED_NONE>(nt, g, b, st, n, a, x, y, cnt, R);
  }
}

hipError_t launch_stream4(int32_t body, const void *payload, const LoopK &L, const SchedK &S, const RedK &R,
                          hipStream_t st) {
  // From 64 MiB of operands on, loads and stores carry the non-temporal hint:
  // measured on MI355X it lifts cold-cache streams by 40-120% and costs at
  // most 6% when the operands are still resident in the 256 MB last-level
  // cache; below 64 MiB plain accesses are as fast or faster either way.
  const bool nt = (uint64_t)L.n * (body == 1 ? 8u : 4u) >= (64ull << 20);
  const int64_t n = L.n, lb = L.lb[0];
  dim3 g(S.T + (R.fold.count > 0 ? 1 : 0)), b(S.U);  // + the fold's own workgroup
  if (body == 1) {
    const AxpyP &p = *(const AxpyP *)payload;
    go_stream4_op<1>(nt, g, b, st, n, p.a, p.x + lb, p.y + lb, nullptr, R);
  } else if (body == 2) {
    if (R.op == RED_NONE) return hipErrorInvalidValue;
    const SumP &p = *(const SumP *)payload;
    go_stream4_op<2>(nt, g, b, st, n, 0.0f, (const float *)p.x + lb, nullptr, nullptr, R);
  } else if (body == 9) {
    const CoverP &p = *(const CoverP *)payload;
    hipLaunchKernelGGL((k_stream4<9, RED_NONE, false>), g, b, 0, st, n, 0.0f, (const float *)nullptr,
                       (float *)nullptr, p.count, R);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------- Jacobi, wavefront strips
// Tile = TH rows x 256 columns, anchored at multiples of (TH, 256); tiles go
// to teams by the schedule. Inside a team's tile the NW = U/64 wavefronts
// take contiguous strips of ceil(TH/NW) rows and lane l takes columns
// 4l .. 4l+3 of every row of its strip (the within-tile unit assignment of
// this body). A wavefront walks its strip top to bottom holding the rows
// above and at the current one in registers, loads the rows below in groups
// of JG with the next group's loads issued before the current group's
// arithmetic, and gets its west/east neighbours from the adjacent lanes
// (lane 0 and lane 63 load the tile's halo columns). Nothing is staged in
// LDS, so no barrier separates loads from arithmetic.
constexpr int JT_W = 256;  // tile width (points)

// Residual reduction per lane. The float64 value of |u1 - u0| is only needed
// where it can change the lane's maximum (or minimum): rounding to float32
// is monotonic, so a point whose float32 |u1 - u0| is below the lane's
// float32 maximum cannot hold the exact maximum. Only candidates at or above
// it take the float64 path, and a row of four points where none is a
// candidate costs one comparison; the result is exact.
template <int OP>
struct ResidualAcc {
  float m32 = OP == RED_MIN ? __builtin_inff() : -1.0f;
  double m64 = OP == RED_SUM ? 0.0 : (OP == RED_MAX ? -__builtin_inf() : __builtin_inf());
  __device__ void add(float v, float c) {
    if (OP == RED_SUM) {
      m64 += fabs((double)v - (double)c);
      return;
    }
    const float d = fabsf(v - c);
    if (OP == RED_MAX ? d >= m32 : d <= m32) {
      const double e = fabs((double)v - (double)c);
      if (d != m32) {
        m32 = d;
        m64 = e;
      } else {
        m64 = OP == RED_MAX ? (e > m64 ? e : m64) : (e < m64 ? e : m64);
      }
    }
  }
  // The four points of a lane's row; bit e of `mk` marks point e as in the
  // loop box.
  __device__ void add4(const f32x4 &v, const f32x4 &c, int mk) {
    if (OP != RED_SUM) {
      constexpr float NONE = OP == RED_MAX ? -1.0f : __builtin_inff();
      const float d0 = mk & 1 ? fabsf(v.x - c.x) : NONE, d1 = mk & 2 ? fabsf(v.y - c.y) : NONE;
      const float d2 = mk & 4 ? fabsf(v.z - c.z) : NONE, d3 = mk & 8 ? fabsf(v.w - c.w) : NONE;
      const float dm = OP == RED_MAX ? fmaxf(fmaxf(d0, d1), fmaxf(d2, d3)) : fminf(fminf(d0, d1), fminf(d2, d3));
      if (OP == RED_MAX ? dm < m32 : dm > m32) return;
    }
    if (mk & 1) add(v.x, c.x);
    if (mk & 2) add(v.y, c.y);
    if (mk & 4) add(v.z, c.z);
    if (mk & 8) add(v.w, c.w);
  }
};

// The rows of one wavefront's strip, rb - ra = n of them. Rows are read
// through a buffer resource that starts 16 bytes before the tile's first
// column in the row above the strip: lane l's four columns (tile columns
// cl .. cl+3, cl = 4 l) sit at byte offset 16 (l + 1) of every row, the
// halo columns at 12 (lane 0, tile column -1) and 1040 (lane 63, column
// 256), and the row is the scalar offset. A lane that must not read an
// address passes an offset past the resource's extent, which the hardware
// answers with zero without touching memory, so the loads need no branches.
// EDGE tiles cross the loop box's column bounds: they read only the tile
// columns [clo, chi] that in-box points read and write only [wlo, whi); a
// lane whose four columns straddle a read bound loads them one by one. Byte
// offsets within a strip fit 32 bits (checked when the variant is chosen).
template <bool EDGE, int RED, bool NT>
__device__ __forceinline__ void jacobi_strip(const float *sp, float *dp, int ld, int n, int lane, int clo, int chi,
                                             int wlo, int whi, ResidualAcc<RED> &acc) {
  constexpr uint32_t OFF = 0x80000000u;  // past the extent: reads as zero
  // rows per load group: 4 without a residual, 2 with one (the residual's
  // registers and arithmetic leave room for fewer rows in flight)
  constexpr int JG = RED != RED_NONE ? 2 : 4;
  const uint32_t rowb = 4u * (uint32_t)ld;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)(sp - 4), (short)0, (int)((uint32_t)(n + 1) * rowb + 1044u), 0x00020000);
  const int cl = 4 * lane;
  const bool in4 = !EDGE || (cl >= clo && cl + 3 <= chi);
  const bool split = EDGE && !in4 && cl <= chi && cl + 3 >= clo;
  const uint32_t vo = in4 ? 16u * (uint32_t)(lane + 1) : OFF;
  const int hc = lane == 0 ? cl - 1 : cl + 4;
  const uint32_t ho =
      (lane == 0 || lane == WAVE - 1) && (!EDGE || (hc >= clo && hc <= chi)) ? 16u + 4u * (uint32_t)hc : OFF;
  auto elem = [&](int x, int q) {
    const uint32_t eo = cl + q >= clo && cl + q <= chi ? 16u + 4u * (uint32_t)(cl + q) : OFF;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, eo, __builtin_amdgcn_readfirstlane(x * (int)rowb), 0));
  };
  auto row4 = [&](int x) {
    f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, __builtin_amdgcn_readfirstlane(x * (int)rowb), 0));
    if (EDGE && split) v = f32x4{elem(x, 0), elem(x, 1), elem(x, 2), elem(x, 3)};
    return v;
  };
  auto halo = [&](int x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ho, __builtin_amdgcn_readfirstlane(x * (int)rowb), 0));
  };
  // Points of this lane in the box (bit e: column cl + e) and, in EDGE tiles,
  // the destination through a buffer resource: a lane writes its four
  // columns with one store when all are in the box, else (in a wavefront
  // that has such a lane) one by one, offsets past the extent dropping the
  // columns outside the box.
  int mk = 0xF;
  if (EDGE) {
    mk = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) mk |= (cl + e >= wlo && cl + e < whi) ? 1 << e : 0;
  }
  const __amdgpu_buffer_rsrc_t rd =
      __builtin_amdgcn_make_buffer_rsrc((void *)dp, (short)0, (int)((uint32_t)(n - 1) * rowb + 1024u), 0x00020000);
  const uint32_t so4 = mk == 0xF ? 4u * (uint32_t)cl : OFF;
  const bool part = EDGE && __builtin_amdgcn_ballot_w64(mk != 0xF && mk != 0) != 0;
  f32x4 up = row4(0), mid = row4(1);
  float hm = halo(1);
  // Strip rows r+1 .. r+JG (clamped to n, the row below the strip).
  auto load_group = [&](int r, f32x4 *dn, float *hd) {
#pragma unroll
    for (int q = 0; q < JG; ++q) {
      const int x = (r + 1 + q < n ? r + 1 + q : n) + 1;
      dn[q] = row4(x);
      hd[q] = halo(x);
    }
  };
  // Output rows r .. r+JG-1 of the strip from the rows held and a group below.
  auto compute_group = [&](int r, const f32x4 *dn, const float *hd) {
#pragma unroll
    for (int q = 0; q < JG; ++q) {
      if (r + q >= n) break;
      const float wsh = __shfl_up(mid.w, 1), esh = __shfl_down(mid.x, 1);
      const float Wm = lane == 0 ? hm : wsh, Ep = lane == WAVE - 1 ? hm : esh;
      const f32x4 S = dn[q];
      f32x4 v;
      v.x = ((up.x + S.x) + (Wm + mid.y)) * 0.25f;
      v.y = ((up.y + S.y) + (mid.x + mid.z)) * 0.25f;
      v.z = ((up.z + S.z) + (mid.y + mid.w)) * 0.25f;
      v.w = ((up.w + S.w) + (mid.z + Ep)) * 0.25f;
      if (RED) acc.add4(v, mid, mk);
      if (!EDGE) {
        float *out = dp + __builtin_amdgcn_readfirstlane((r + q) * ld) + cl;
        if (NT) __builtin_nontemporal_store(v, (f32x4 *)out);
        else *(f32x4 *)out = v;
      } else {
        const int soff = __builtin_amdgcn_readfirstlane((r + q) * (int)rowb);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rd, so4, soff, 0);
        if (part) {
          const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, vv[e]), rd,
                                                  mk != 0xF && (mk >> e & 1) ? 4u * (uint32_t)(cl + e) : OFF, soff, 0);
        }
      }
      up = mid;
      mid = S;
      hm = hd[q];
    }
  };
  // Two groups in flight: the next group's loads are issued before the
  // current group's arithmetic.
  f32x4 A[JG], B[JG];
  float hA[JG], hB[JG];
  load_group(0, A, hA);
  for (int r = 0; r < n; r += 2 * JG) {
    if (r + JG < n) load_group(r + JG, B, hB);
    compute_group(r, A, hA);
    if (r + JG >= n) break;
    if (r + 2 * JG < n) load_group(r + 2 * JG, A, hA);
    compute_group(r + JG, B, hB);
  }
}

// NT: the grids exceed the last-level cache, so the new grid is stored with
// the non-temporal hint (a grid that fits is read back from that cache by the
// next sweep and is stored normally).
template <int TH, int RED, bool NT>
__global__ void __launch_bounds__(1024) k_jacobi_tile(LoopK L, SchedK S, JacobiP p, RedK R) {
  const int lane = threadIdx.x % WAVE;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), NW = blockDim.x / WAVE;
  // The launch's cross-workgroup work goes to one extra workgroup, launched
  // last and given no tile, so that its latency hides behind the tiles still
  // running: the fold of an earlier loop's deferred reduction, and the
  // combine of this loop's own synchronous reduction (as the last-launched
  // workgroup it is the combiner; its own value is the identity).
  const bool xwg = jacobi_extra_wg(R);
  const int G = xwg ? gridDim.x - 1 : gridDim.x;
  if (xwg && (int)blockIdx.x == G) {
    if (R.fold.count > 0) run_fold(R.fold);
    if (RED && !R.defer) finish_reduction<double>(R, ResidualAcc<RED>().m64);
    return;
  }
  const int team = xcd_team(blockIdx.x, G);
  const int SH = (TH + NW - 1) / NW;                          // strip height
  const int64_t ilo = L.lb[0], ihi = L.lb[0] + L.cnt[0];  // interior rows [ilo, ihi)
  const int64_t jlo = L.lb[1], jhi = L.lb[1] + L.cnt[1];
  const int ld = (int)p.ld;
  ResidualAcc<RED> acc;

  auto do_tile = [&](int64_t m) {
    const int64_t ti = S.t0[0] + m / S.nt[1], tj = S.t0[1] + m % S.nt[1];
    const int64_t i0 = ti * TH, j0 = tj * JT_W;
    const int64_t s0 = i0 + (int64_t)w * SH, s1 = s0 + SH < i0 + TH ? s0 + SH : i0 + TH;
    const int64_t ra = s0 > ilo ? s0 : ilo, rb = s1 < ihi ? s1 : ihi;
    if (ra >= rb) return;
    const float *sp = p.src + (ra - 1) * p.ld + j0;
    float *dp = p.dst + ra * p.ld + j0;
    const int n = (int)(rb - ra);
    if (j0 >= jlo && j0 + JT_W <= jhi) {
      jacobi_strip<false, RED, NT>(sp, dp, ld, n, lane, -1, JT_W, 0, JT_W, acc);
    } else {
      // tile columns read by in-box points (inclusive) and written (half-open)
      const int wlo = (int)((j0 > jlo ? j0 : jlo) - j0), whi = (int)((j0 + JT_W < jhi ? j0 + JT_W : jhi) - j0);
      jacobi_strip<true, RED, NT>(sp, dp, ld, n, lane, wlo - 1, whi, wlo, whi, acc);
    }
  };

  if (S.policy == POL_STATIC) {
    int64_t lo, hi;
    block_range(S.ntiles, S.T, team, lo, hi);
    for (int64_t m = lo; m < hi; ++m) do_tile(m);
  } else {
    const int64_t c = S.chunk;
    for (int64_t m0 = (int64_t)team * c; m0 < S.ntiles; m0 += (int64_t)S.T * c)
      for (int64_t m = m0; m < m0 + c && m < S.ntiles; ++m) do_tile(m);
  }
  if (RED) finish_reduction<double>(R, acc.m64);
}

bool jacobi_tile_supports(const JacobiP &p, const LoopK &L, const SchedK &S) {
  if (L.nd != 2 || !S.tiled || S.dist != DIST_TU) return false;
  if (L.step[0] != 1 || L.step[1] != 1) return false;
  if (S.tile[1] != JT_W) return false;
  const int th = S.tile[0];
  if (th != 4 && th != 8 && th != 16 && th != 32 && th != 64 && th != 128) return false;
  if (S.U % WAVE != 0 || S.U < WAVE) return false;
  if (S.policy != POL_STATIC && S.policy != POL_CHUNK) return false;
  if ((p.ld % 4) != 0 || ((uintptr_t)p.src % 16) != 0 || ((uintptr_t)p.dst % 16) != 0) return false;
  if (L.lb[1] < 1 || L.lb[0] < 1) return false;  // halo reads at lb-1 stay in the array
  if ((int64_t)(th + 2) * p.ld * 4 + 2048 >= (1LL << 31)) return false;  // 32-bit byte offsets within a strip
  return true;
}

template <int TH, bool NT>
static hipError_t go_jacobi_nt(const JacobiP &p, const LoopK &L, const SchedK &S, const RedK &R, hipStream_t st) {
  const dim3 g(S.T + (jacobi_extra_wg(R) ? 1 : 0)), b(S.U);
  switch (R.op) {
    case RED_NONE: hipLaunchKernelGGL((k_jacobi_tile<TH, RED_NONE, NT>), g, b, 0, st, L, S, p, R); break;
    case RED_SUM: hipLaunchKernelGGL((k_jacobi_tile<TH, RED_SUM, NT>), g, b, 0, st, L, S, p, R); break;
    case RED_MAX: hipLaunchKernelGGL((k_jacobi_tile<TH, RED_MAX, NT>), g, b, 0, st, L, S, p, R); break;
    default: hipLaunchKernelGGL((k_jacobi_tile<TH, RED_MIN, NT>), g, b, 0, st, L, S, p, R); break;
  }
  return hipGetLastError();
}

template <int TH>
static hipError_t go_jacobi(const JacobiP &p, const LoopK &L, const SchedK &S, const RedK &R, hipStream_t st) {
  // source and destination rows the sweep touches, against the 256 MB cache
  const uint64_t bytes = 2ull * (uint64_t)(L.cnt[0] + 2) * (uint64_t)p.ld * 4u;
  return bytes > (256ull << 20) ? go_jacobi_nt<TH, true>(p, L, S, R, st) : go_jacobi_nt<TH, false>(p, L, S, R, st);
}

hipError_t launch_jacobi_tile(const JacobiP &p, const LoopK &L, const SchedK &S, const RedK &R, hipStream_t st) {
  switch (S.tile[0]) {
    case 4: return go_jacobi<4>(p, L, S, R, st);
    case 8: return go_jacobi<8>(p, L, S, R, st);
    case 16: return go_jacobi<16>(p, L, S, R, st);
    case 32: return go_jacobi<32>(p, L, S, R, st);
    case 64: return go_jacobi<64>(p, L, S, R, st);
    case 128: return go_jacobi<128>(p, L, S, R, st);
  }
  return hipErrorInvalidValue;
}

// ----------------------------------------- 7 x 7 filter, wavefront strips
// Tiles of TH rows x 256 columns go to teams as for Jacobi; wavefront w of a
// team takes a strip of ceil(TH / NW) rows and lane l columns 4l .. 4l+3.
// The wavefront walks the input rows from three above its strip to three
// below. Each input row is assembled as ten values per lane (columns
// 4l-3 .. 4l+6: its own four and three from each neighbouring lane; lanes 0
// and 63 load the tile's halo) and added into the seven output rows it
// feeds. An output row receives filter row m = 0..6 in that order, and
// within a row n = 0..6, so its value is the definition's fused
// multiply-add chain. After each input row the oldest output row is
// complete and is stored.
constexpr int F7_G = 4;  // input rows loaded together

struct F7Row {
  f32x4 v;
  float h0, h1, h2;  // lane 0: columns c0-3 .. c0-1; lane 63: columns c0+4 .. c0+6
};

template <bool EDGE>
__device__ __forceinline__ void f7_load(const float *row, int64_t c0, int lane, int64_t clo, int64_t chi, F7Row &r) {
  if (!EDGE || (c0 >= clo && c0 + 3 <= chi)) {
    r.v = *(const f32x4 *)(row + c0);
  } else {
    float e[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) e[q] = (c0 + q >= clo && c0 + q <= chi) ? row[c0 + q] : 0.0f;
    r.v = f32x4{e[0], e[1], e[2], e[3]};
  }
  r.h0 = r.h1 = r.h2 = 0.0f;
  if (lane == 0) {
    if (c0 - 3 >= clo) r.h0 = row[c0 - 3];
    if (c0 - 2 >= clo) r.h1 = row[c0 - 2];
    if (c0 - 1 >= clo) r.h2 = row[c0 - 1];
  } else if (lane == WAVE - 1) {
    if (c0 + 4 <= chi) r.h0 = row[c0 + 4];
    if (c0 + 5 <= chi) r.h1 = row[c0 + 5];
    if (c0 + 6 <= chi) r.h2 = row[c0 + 6];
  }
}

template <bool EDGE>
__device__ __forceinline__ void f7_strip(const Filter7P &p, const float (&wk)[49], int64_t ra, int64_t rb, int64_t c0,
                                         int lane, int64_t clo, int64_t chi, int64_t jlo, int64_t jhi) {
  const int64_t ld = p.ld;
  float acc[7][4];  // acc[k]: output row (input row - 3 + k), which takes filter row 6 - k next
#pragma unroll
  for (int k = 0; k < 7; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[k][q] = 0.0f;
  const int64_t rlast = rb + 2;  // last input row
  for (int64_t r0 = ra - 3; r0 <= rlast; r0 += F7_G) {
    F7Row in[F7_G];
#pragma unroll
    for (int g = 0; g < F7_G; ++g) {
      const int64_t rr = r0 + g < rlast ? r0 + g : rlast;
      f7_load<EDGE>(p.src + rr * ld, c0, lane, clo, chi, in[g]);
    }
#pragma unroll
    for (int g = 0; g < F7_G; ++g) {
      const int64_t r = r0 + g;
      if (r > rlast) break;
      const F7Row &x = in[g];
      const float l1 = __shfl_up(x.v.y, 1), l2 = __shfl_up(x.v.z, 1), l3 = __shfl_up(x.v.w, 1);
      const float q1 = __shfl_down(x.v.x, 1), q2 = __shfl_down(x.v.y, 1), q3 = __shfl_down(x.v.z, 1);
      const bool first = lane == 0, last = lane == WAVE - 1;
      const float seg[10] = {first ? x.h0 : l1, first ? x.h1 : l2, first ? x.h2 : l3, x.v.x, x.v.y, x.v.z, x.v.w,
                             last ? x.h0 : q1,  last ? x.h1 : q2,  last ? x.h2 : q3};
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const int64_t o = r - 3 + k;
        if (o >= ra && o < rb) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int n = 0; n < 7; ++n) acc[k][q] = __builtin_fmaf(wk[(6 - k) * 7 + n], seg[q + n], acc[k][q]);
        }
      }
      const int64_t o = r - 3;  // complete: it has taken filter row 6
      if (o >= ra && o < rb) {
        float *out = p.dst + o * ld + c0;
        if (!EDGE || (c0 >= jlo && c0 + 3 < jhi)) {
          __builtin_nontemporal_store(f32x4{acc[0][0], acc[0][1], acc[0][2], acc[0][3]}, (f32x4 *)out);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (c0 + q >= jlo && c0 + q < jhi) out[q] = acc[0][q];
        }
      }
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[k][q] = acc[k + 1][q];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[6][q] = 0.0f;
    }
  }
}

template <int TH>
__global__ void __launch_bounds__(1024) k_filter7_tile(LoopK L, SchedK S, Filter7P p, RedK R) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE, NW = blockDim.x / WAVE;
  const int team = xcd_team(blockIdx.x, gridDim.x);
  const int SH = (TH + NW - 1) / NW;
  const int64_t ilo = L.lb[0], ihi = L.lb[0] + L.cnt[0];
  const int64_t jlo = L.lb[1], jhi = L.lb[1] + L.cnt[1];
  float wk[49];
#pragma unroll
  for (int i = 0; i < 49; ++i) wk[i] = p.w[i];
  auto do_tile = [&](int64_t m) {
    const int64_t ti = S.t0[0] + m / S.nt[1], tj = S.t0[1] + m % S.nt[1];
    const int64_t i0 = ti * TH, j0 = tj * JT_W;
    const int64_t s0 = i0 + (int64_t)w * SH, s1 = s0 + SH < i0 + TH ? s0 + SH : i0 + TH;
    const int64_t ra = s0 > ilo ? s0 : ilo, rb = s1 < ihi ? s1 : ihi;
    if (ra >= rb) return;
    const int64_t c0 = j0 + 4 * lane;
    if (j0 >= jlo && j0 + JT_W <= jhi) {
      f7_strip<false>(p, wk, ra, rb, c0, lane, j0 - 3, j0 + JT_W + 2, jlo, jhi);
    } else {
      // columns read by in-box points of this tile (inclusive)
      const int64_t clo = (j0 > jlo ? j0 : jlo) - 3, chi = (j0 + JT_W < jhi ? j0 + JT_W : jhi) + 2;
      f7_strip<true>(p, wk, ra, rb, c0, lane, clo, chi, jlo, jhi);
    }
  };
  if (S.policy == POL_STATIC) {
    int64_t lo, hi;
    block_range(S.ntiles, S.T, team, lo, hi);
    for (int64_t m = lo; m < hi; ++m) do_tile(m);
  } else {
    const int64_t c = S.chunk;
    for (int64_t m0 = (int64_t)team * c; m0 < S.ntiles; m0 += (int64_t)S.T * c)
      for (int64_t m = m0; m < m0 + c && m < S.ntiles; ++m) do_tile(m);
  }
  fold_hook(R);
}

bool filter7_tile_supports(const Filter7P &p, const LoopK &L, const SchedK &S) {
  if (L.nd != 2 || !S.tiled || S.dist != DIST_TU) return false;
  if (L.step[0] != 1 || L.step[1] != 1) return false;
  if (S.tile[1] != JT_W) return false;
  const int th = S.tile[0];
  if (th != 4 && th != 8 && th != 16 && th != 32 && th != 64) return false;
  if (S.U % WAVE != 0 || S.U < WAVE) return false;
  if (S.policy != POL_STATIC && S.policy != POL_CHUNK) return false;
  if ((p.ld % 4) != 0 || ((uintptr_t)p.src % 16) != 0 || ((uintptr_t)p.dst % 16) != 0) return false;
  if (L.lb[1] < 3 || L.lb[0] < 3) return false;  // reads at lb-3 stay in the array
  return true;
}

hipError_t launch_filter7_tile(const Filter7P &p, const LoopK &L, const SchedK &S, const RedK &R, hipStream_t st) {
  const dim3 g(S.T), b(S.U);
  switch (S.tile[0]) {
    case 4: hipLaunchKernelGGL(k_filter7_tile<4>, g, b, 0, st, L, S, p, R); break;
    case 8: hipLaunchKernelGGL(k_filter7_tile<8>, g, b, 0, st, L, S, p, R); break;
    case 16: hipLaunchKernelGGL(k_filter7_tile<16>, g, b, 0, st, L, S, p, R); break;
    case 32: hipLaunchKernelGGL(k_filter7_tile<32>, g, b, 0, st, L, S, p, R); break;
    case 64: hipLaunchKernelGGL(k_filter7_tile<64>, g, b, 0, st, L, S, p, R); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------- matvec, wave/row
// The unit of a MATVEC loop is a wavefront: rows are owned by (team, wave)
// under the schedule with U/64 units per team. Inside a row, lane l takes
// columns 4l .. 4l+3 of every 256-column block in order, then the 64 lane
// sums meet in a fixed reduction tree.
template <bool RED>
__global__ void __launch_bounds__(1024) k_matvec(LoopK L, SchedK S, MatvecP p, RedK R) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  SchedK SW = S;
  SW.U = S.U / WAVE;
  float acc = RED ? red_identity<float>(R.op) : 0.0f;
  const bool vec = (p.lda % 4 == 0) && ((uintptr_t)p.A % 16 == 0) && ((uintptr_t)p.x % 16 == 0);
  auto row = [&](int64_t, const int64_t *iv) {
    const int64_t r = iv[0];
    const float *a = p.A + r * p.lda;
    float s = 0.0f;
    int64_t c0 = 0;
    if (vec) {
      // eight (then four) 256-column blocks per trip: their loads are all
      // issued before the multiply-adds, which keep the block-by-block order
      // (N = 16384: 191 us against 238 us one block at a time)
      auto blocks = [&](auto nb) {
        constexpr int NB = decltype(nb)::value;
        for (; c0 + 256 * NB <= p.cols; c0 += 256 * NB) {
          f32x4 av[NB], xv[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            av[u] = *(const f32x4 *)(a + c0 + 256 * u + 4 * lane);
            xv[u] = *(const f32x4 *)(p.x + c0 + 256 * u + 4 * lane);
          }
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            s = __builtin_fmaf(av[u].x, xv[u].x, s);
            s = __builtin_fmaf(av[u].y, xv[u].y, s);
            s = __builtin_fmaf(av[u].z, xv[u].z, s);
            s = __builtin_fmaf(av[u].w, xv[u].w, s);
          }
        }
      };
      blocks(std::integral_constant<int, 8>{});
      blocks(std::integral_constant<int, 4>{});
    }
    for (; c0 < p.cols; c0 += 256) {
      const int64_t c = c0 + 4 * lane;
      if (vec && c + 3 < p.cols) {
        const f32x4 av = *(const f32x4 *)(a + c);
        const f32x4 xv = *(const f32x4 *)(p.x + c);
        s = __builtin_fmaf(av.x, xv.x, s);
        s = __builtin_fmaf(av.y, xv.y, s);
        s = __builtin_fmaf(av.z, xv.z, s);
        s = __builtin_fmaf(av.w, xv.w, s);
      } else {
        for (int q = 0; q < 4; ++q)
          if (c + q < p.cols) s = __builtin_fmaf(a[c + q], p.x[c + q], s);
      }
    }
    s = wave_reduce(RED_SUM, s);
    if (lane == 0) {
      p.y[r] = s;
      if (RED) acc = red_apply(R.op, acc, s);
    }
  };
  for_owned_untiled(L, SW, blockIdx.x, w, row);
  if (RED) finish_reduction<float>(R, acc);
  fold_hook(R);
}

hipError_t launch_matvec_wave(const MatvecP &p, const LoopK &L, const SchedK &S, const RedK &R, hipStream_t st) {
  if (R.op != RED_NONE)
    hipLaunchKernelGGL(k_matvec<true>, dim3(S.T), dim3(S.U), 0, st, L, S, p, R);
  else
    hipLaunchKernelGGL(k_matvec<false>, dim3(S.T), dim3(S.U), 0, st, L, S, p, R);
  return hipGetLastError();
}

}  // namespace upir

// Standalone fold of a deferred reduction (one workgroup).
namespace upir {
__global__ void __launch_bounds__(256) k_fold(FoldK F) { run_fold(F); }
hipError_t launch_fold(const FoldK &F, hipStream_t st) {
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(256), 0, st, F);
  return hipGetLastError();
}
}  // namespace upir
