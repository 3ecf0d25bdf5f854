// Dense matmul loop C = A B (gfx950): bfloat16 split pre-pass and MFMA tiles.
//
// Paper: sec. 6.2 names a matrix multiplication kernel among its four
// offloaded loops; its source and precision are not given. The loop here is
// collapse(2) over C with the k reduction in the body. Precision variants
// (not in the paper): float32; A, B rounded to bfloat16 (round to nearest
// even) with float32 accumulation; and the three-pass split
// A_lo B_hi + A_hi B_lo + A_hi B_hi that recovers float32 accuracy.
#include "upir.h"
#include "upir_launch.h"

namespace upir {

__device__ inline uint16_t to_bf16_rne(float x) {
  __bf16 h = (__bf16)x;  // IEEE conversion: round to nearest, ties to even
  return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf16f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// A (M x K, lda) -> ah / al (M x K, dense). Row-major, coalesced.
__global__ void __launch_bounds__(256) k_split_rows(const float *__restrict__ A, int64_t M, int64_t K, int64_t lda,
                                                    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  const int64_t total = M * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / K, k = e - i * K;
    const float x = A[i * lda + k];
    const uint16_t h = to_bf16_rne(x);
    hi[e] = h;
    if (lo) lo[e] = to_bf16_rne(x - bf16f(h));
  }
}

// B (K x N, ldb) -> bh / bl transposed (N x K, dense) through a 64 x 64 LDS tile.
__global__ void __launch_bounds__(256) k_split_cols(const float *__restrict__ B, int64_t K, int64_t N, int64_t ldb,
                                                    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  __shared__ float t[64][65];
  const int64_t k0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;  // 64 x 4
  for (int r = ty; r < 64; r += 4) {
    const int64_t k = k0 + r, n = n0 + tx;
    t[r][tx] = (k < K && n < N) ? B[k * ldb + n] : 0.0f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t n = n0 + r, k = k0 + tx;
    if (n < N && k < K) {
      const float x = t[tx][r];
      const uint16_t h = to_bf16_rne(x);
      hi[n * K + k] = h;
      if (lo) lo[n * K + k] = to_bf16_rne(x - bf16f(h));
    }
  }
}

// Vector forms (K % 8 == 0, 16-byte aligned rows): eight consecutive k per
// thread, two 16-byte loads and one 16-byte store of eight bfloat16 per
// output array.
typedef float f32x4s __attribute__((ext_vector_type(4)));
typedef unsigned u32x4s __attribute__((ext_vector_type(4)));
__device__ inline unsigned pack2(uint16_t a, uint16_t b) { return (unsigned)a | ((unsigned)b << 16); }

__global__ void __launch_bounds__(256) k_split_rows8(const float *__restrict__ A, int64_t M, int64_t K, int64_t lda,
                                                     uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  const int64_t chunks = M * (K / 8);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < chunks; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = 8 * c, i = e / K, k = e - i * K;
    const f32x4s v0 = *(const f32x4s *)(A + i * lda + k), v1 = *(const f32x4s *)(A + i * lda + k + 4);
    const float x[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    uint16_t h[8], l[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      h[q] = to_bf16_rne(x[q]);
      l[q] = to_bf16_rne(x[q] - bf16f(h[q]));
    }
    *(u32x4s *)(hi + e) = u32x4s{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
    if (lo) *(u32x4s *)(lo + e) = u32x4s{pack2(l[0], l[1]), pack2(l[2], l[3]), pack2(l[4], l[5]), pack2(l[6], l[7])};
  }
}

// B (K x N) -> N x K through a 64 (k) x 64 (n) LDS tile: rows of B are read
// as float4, each output row n gets its 64 k as eight 16-byte stores.
__global__ void __launch_bounds__(256) k_split_cols8(const float *__restrict__ B, int64_t K, int64_t N, int64_t ldb,
                                                     uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  __shared__ float t[64][65];
  const int64_t k0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  for (int q = threadIdx.x; q < 64 * 16; q += 256) {  // 64 rows x 16 float4
    const int r = q / 16, c4 = 4 * (q % 16);
    const int64_t k = k0 + r, n = n0 + c4;
    f32x4s v = {0.0f, 0.0f, 0.0f, 0.0f};
    if (k < K && n + 3 < N) {
      v = *(const f32x4s *)(B + k * ldb + n);
    } else if (k < K) {
      float e[4];
      for (int j = 0; j < 4; ++j) e[j] = n + j < N ? B[k * ldb + n + j] : 0.0f;
      v = f32x4s{e[0], e[1], e[2], e[3]};
    }
    t[r][c4] = v.x;
    t[r][c4 + 1] = v.y;
    t[r][c4 + 2] = v.z;
    t[r][c4 + 3] = v.w;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * 8; q += 256) {  // 64 output rows x 8 chunks of 8 k
    const int r = q / 8, kc = 8 * (q % 8);
    const int64_t n = n0 + r, k = k0 + kc;
    if (n >= N || k >= K) continue;  // K % 8 == 0: a chunk is all in or all out
    uint16_t h[8], l[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float x = t[kc + j][r];
      h[j] = to_bf16_rne(x);
      l[j] = to_bf16_rne(x - bf16f(h[j]));
    }
    *(u32x4s *)(hi + n * K + k) = u32x4s{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
    if (lo) *(u32x4s *)(lo + n * K + k) = u32x4s{pack2(l[0], l[1]), pack2(l[2], l[3]), pack2(l[4], l[5]), pack2(l[6], l[7])};
  }
}

hipError_t launch_bf16_split(const MatmulP &p, bool need_lo, hipStream_t st) {
  // vector forms: K % 8 == 0, 16-byte aligned operands and rows, aligned workspace
  const bool ws_ok = (uintptr_t)p.ah % 16 == 0 && (uintptr_t)p.bh % 16 == 0 &&
                     (!need_lo || ((uintptr_t)p.al % 16 == 0 && (uintptr_t)p.bl % 16 == 0));
  const bool vec = p.K % 8 == 0 && ws_ok;
  const bool vec_a = vec && p.lda % 4 == 0 && (uintptr_t)p.A % 16 == 0;
  const bool vec_b = vec && p.ldb % 4 == 0 && (uintptr_t)p.B % 16 == 0;
  if (p.M > 0 && p.K > 0) {
    if (vec_a) {
      const int64_t chunks = p.M * (p.K / 8);
      const int g = (int)std::min<int64_t>((chunks + 255) / 256, 16384);
      hipLaunchKernelGGL(k_split_rows8, dim3(g), dim3(256), 0, st, p.A, p.M, p.K, p.lda, p.ah,
                         need_lo ? p.al : nullptr);
    } else {
      const int64_t tot = p.M * p.K;
      const int g = (int)std::min<int64_t>((tot + 255) / 256, 8192);
      hipLaunchKernelGGL(k_split_rows, dim3(g), dim3(256), 0, st, p.A, p.M, p.K, p.lda, p.ah,
                         need_lo ? p.al : nullptr);
    }
  }
  if (p.N > 0 && p.K > 0) {
    dim3 g((unsigned)((p.N + 63) / 64), (unsigned)((p.K + 63) / 64));
    if (vec_b)
      hipLaunchKernelGGL(k_split_cols8, g, dim3(256), 0, st, p.B, p.K, p.N, p.ldb, p.bh, need_lo ? p.bl : nullptr);
    else
      hipLaunchKernelGGL(k_split_cols, g, dim3(256), 0, st, p.B, p.K, p.N, p.ldb, p.bh, need_lo ? p.bl : nullptr);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ MFMA tiles
// A team computes whole BM x BN tiles of C; tiles are numbered row-major
// over C and handed to teams by the tiled schedule (static blocks or
// chunks). Team ids are laid out so consecutive tiles share an XCD (and its
// L2). Inside a tile the points are computed by MFMA fragments, so the
// within-tile assignment of points to units is fixed by the matrix cores.
//
// Waves form a WM x WN grid; each wave owns (BM/WM) x (BN/WN) of the tile as
// 32 x 32 MFMA blocks. K advances in steps of BK: the next step's operands
// are fetched from global memory into registers while the current step's
// operands, staged in LDS with padded rows (no bank conflicts on the 16-byte
// fragment reads), feed the matrix cores.
//
// bfloat16 variants use v_mfma_f32_32x32x16_bf16 (lane l supplies row l%32
// and 8 consecutive k of group l/32); both hi/lo operands come from the
// pre-pass workspace (A as M x K, B transposed as N x K). The split variant
// accumulates lo_A hi_B, hi_A lo_B and hi_A hi_B into one float32 sum.
// float32 uses v_mfma_f32_32x32x2f32 over A (M x K) and B (K x N) directly.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int WM, int WN>
__device__ inline void store_c(const MatmulP &p, int64_t row0, int64_t col0, const f32x16 (&acc)[BM / WM / 32][BN / WN / 32]) {
  constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = col0 + wn * (BN / WN) + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = row0 + wm * (BM / WM) + i * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        if (row < p.M && col < p.N) p.C[row * p.ldc + col] = acc[i][j][r];
      }
    }
}

// Tiles owned by this team under the tiled schedule.
template <class F>
__device__ inline void for_team_tiles(const SchedK &S, F &&f) {
  const int team = xcd_team(blockIdx.x, gridDim.x);
  if (S.policy == POL_STATIC) {
    int64_t lo, hi;
    block_range(S.ntiles, S.T, team, lo, hi);
    for (int64_t m = lo; m < hi; ++m) f(m);
  } else {
    const int64_t c = S.chunk;
    for (int64_t m0 = (int64_t)team * c; m0 < S.ntiles; m0 += (int64_t)S.T * c)
      for (int64_t m = m0; m < m0 + c && m < S.ntiles; ++m) f(m);
  }
}

template <int NPROD, int BM, int BN, int WM, int WN, int BK, int STAGES>
__global__ void __launch_bounds__(WM * WN * 64) k_mm_bf16(MatmulP p, SchedK S) {
  constexpr int NTH = WM * WN * 64;
  constexpr int PITCH = BK + 8;  // halfwords per LDS row (16-byte multiple)
  constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
  constexpr int CPR = BK / 8;                    // 16-byte chunks per row
  constexpr int CA = BM * CPR / NTH, CB = BN * CPR / NTH;
  constexpr int STAGE = (NPROD == 3 ? 2 : 1) * (BM + BN) * PITCH;  // halfwords per LDS stage
  static_assert(BM * CPR % NTH == 0 && BN * CPR % NTH == 0, "chunk split");
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t K = p.K;

  for_team_tiles(S, [&](int64_t m) {
    const int64_t row0 = (S.t0[0] + m / S.nt[1]) * BM, col0 = (S.t0[1] + m % S.nt[1]) * BN;
    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};
    u32x4 ra[CA], rb[CB], ral[NPROD == 3 ? CA : 1], rbl[NPROD == 3 ? CB : 1];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int q = 0; q < CA; ++q) {
        const int c = tid + q * NTH, r = c / CPR, kc = c % CPR;
        const int64_t gr = row0 + r, gk = k0 + kc * 8;
        const bool in = gr < p.M && gk < K;
        ra[q] = in ? *(const u32x4 *)(p.ah + gr * K + gk) : u32x4{};
        if (NPROD == 3) ral[q] = in ? *(const u32x4 *)(p.al + gr * K + gk) : u32x4{};
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        const int c = tid + q * NTH, r = c / CPR, kc = c % CPR;
        const int64_t gc = col0 + r, gk = k0 + kc * 8;
        const bool in = gc < p.N && gk < K;
        rb[q] = in ? *(const u32x4 *)(p.bh + gc * K + gk) : u32x4{};
        if (NPROD == 3) rbl[q] = in ? *(const u32x4 *)(p.bl + gc * K + gk) : u32x4{};
      }
    };
    // LDS stage layout: A_hi (BM rows), B_hi (BN rows), then A_lo, B_lo
    auto stage = [&](int buf) {
      uint16_t *sAh = lds + buf * STAGE, *sBh = sAh + BM * PITCH;
      uint16_t *sAl = sBh + BN * PITCH, *sBl = sAl + BM * PITCH;
#pragma unroll
      for (int q = 0; q < CA; ++q) {
        const int c = tid + q * NTH, r = c / CPR, kc = c % CPR;
        *(u32x4 *)(sAh + r * PITCH + kc * 8) = ra[q];
        if (NPROD == 3) *(u32x4 *)(sAl + r * PITCH + kc * 8) = ral[q];
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        const int c = tid + q * NTH, r = c / CPR, kc = c % CPR;
        *(u32x4 *)(sBh + r * PITCH + kc * 8) = rb[q];
        if (NPROD == 3) *(u32x4 *)(sBl + r * PITCH + kc * 8) = rbl[q];
      }
    };
    __syncthreads();  // previous tile's readers are done with LDS
    fetch(0);
    stage(0);
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
      const bool more = k0 + BK < K;
      if (more) fetch(k0 + BK);
      const uint16_t *sAh = lds + cur * STAGE, *sBh = sAh + BM * PITCH;
      const uint16_t *sAl = sBh + BN * PITCH, *sBl = sAl + BM * PITCH;
#pragma unroll
      for (int ks = 0; ks < BK; ks += 16) {
        const int koff = ks + 8 * (lane >> 5);
        bf16x8 a[FM], b[FN], al[NPROD == 3 ? FM : 1], bl[NPROD == 3 ? FN : 1];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const int r = wm * (BM / WM) + i * 32 + (lane & 31);
          a[i] = *(const bf16x8 *)(sAh + r * PITCH + koff);
          if (NPROD == 3) al[i] = *(const bf16x8 *)(sAl + r * PITCH + koff);
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int r = wn * (BN / WN) + j * 32 + (lane & 31);
          b[j] = *(const bf16x8 *)(sBh + r * PITCH + koff);
          if (NPROD == 3) bl[j] = *(const bf16x8 *)(sBl + r * PITCH + koff);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if (NPROD == 3) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], b[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bl[j], acc[i][j], 0, 0, 0);
            }
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
          }
      }
      if (STAGES == 2) {
        // the other buffer was last read before the previous barrier
        if (more) stage(cur ^ 1);
        __syncthreads();
        cur ^= 1;
      } else if (more) {
        __syncthreads();
        stage(0);
        __syncthreads();
      }
    }
    store_c<BM, BN, WM, WN>(p, row0, col0, acc);
  });
}

template <int BM, int BN, int WM, int WN, int BK>
__global__ void __launch_bounds__(WM * WN * 64) k_mm_f32(MatmulP p, SchedK S) {
  constexpr int NTH = WM * WN * 64;
  constexpr int PA = BK + 4;   // floats per A row in LDS
  constexpr int PB = BN + 8;   // floats per B row (k) in LDS
  constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
  constexpr int CA = BM * (BK / 4) / NTH, CB = BK * (BN / 4) / NTH;
  static_assert(BM * (BK / 4) % NTH == 0 && BK * (BN / 4) % NTH == 0, "chunk split");
  extern __shared__ __attribute__((aligned(16))) float ldsf[];
  float *sA = ldsf, *sB = ldsf + BM * PA;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t K = p.K;

  for_team_tiles(S, [&](int64_t m) {
    const int64_t row0 = (S.t0[0] + m / S.nt[1]) * BM, col0 = (S.t0[1] + m % S.nt[1]) * BN;
    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};
    f32x4v ra[CA], rb[CB];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int q = 0; q < CA; ++q) {
        const int c = tid + q * NTH, r = c / (BK / 4), kc = c % (BK / 4);
        const int64_t gr = row0 + r, gk = k0 + kc * 4;
        ra[q] = (gr < p.M && gk < K) ? *(const f32x4v *)(p.A + gr * p.lda + gk) : f32x4v{};
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        const int c = tid + q * NTH, r = c / (BN / 4), nc = c % (BN / 4);
        const int64_t gk = k0 + r, gc = col0 + nc * 4;
        rb[q] = (gk < K && gc < p.N) ? *(const f32x4v *)(p.B + gk * p.ldb + gc) : f32x4v{};
      }
    };
    auto stage = [&]() {
#pragma unroll
      for (int q = 0; q < CA; ++q) {
        const int c = tid + q * NTH, r = c / (BK / 4), kc = c % (BK / 4);
        *(f32x4v *)(sA + r * PA + kc * 4) = ra[q];
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        const int c = tid + q * NTH, r = c / (BN / 4), nc = c % (BN / 4);
        *(f32x4v *)(sB + r * PB + nc * 4) = rb[q];
      }
    };
    __syncthreads();
    fetch(0);
    stage();
    __syncthreads();
    const int g = lane >> 5;
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
      const bool more = k0 + BK < K;
      if (more) fetch(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 8) {
        // group g takes k = kk + 4g + s at MFMA step s (same for A and B)
        f32x4v a[FM];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          a[i] = *(const f32x4v *)(sA + (wm * (BM / WM) + i * 32 + (lane & 31)) * PA + kk + 4 * g);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          float b[FN];
#pragma unroll
          for (int j = 0; j < FN; ++j) b[j] = sB[(kk + 4 * g + s) * PB + wn * (BN / WN) + j * 32 + (lane & 31)];
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s], b[j], acc[i][j], 0, 0, 0);
        }
      }
      if (more) {
        __syncthreads();
        stage();
        __syncthreads();
      }
    }
    store_c<BM, BN, WM, WN>(p, row0, col0, acc);
  });
}

// Kernel configurations: (kind, tile) -> block size.
struct MMConf { int kind, bm, bn, threads; };
static const MMConf kMM[] = {
    {UPIR_BODY_MATMUL_BF16, 256, 256, 512}, {UPIR_BODY_MATMUL_BF16, 128, 128, 256},
    {UPIR_BODY_MATMUL_SPLIT3, 256, 256, 512}, {UPIR_BODY_MATMUL_SPLIT3, 128, 128, 256},
    {UPIR_BODY_MATMUL_F32, 128, 128, 256}, {UPIR_BODY_MATMUL_F32, 256, 128, 512},
};

bool matmul_mfma_supports(const MatmulP &p, const LoopK &L, const SchedK &S) {
  if (L.nd != 2 || !S.tiled || S.dist != DIST_TU) return false;
  if (S.policy != POL_STATIC && S.policy != POL_CHUNK) return false;
  if (L.lb[0] != 0 || L.lb[1] != 0) return false;
  bool conf = false;
  for (const MMConf &c : kMM)
    if (c.kind == p.kind && c.bm == S.tile[0] && c.bn == S.tile[1] && c.threads == S.U) conf = true;
  if (!conf) return false;
  if (p.kind == UPIR_BODY_MATMUL_F32) {
    if (p.K % 4 || p.lda % 4 || p.ldb % 4 || p.N % 4) return false;
    if ((uintptr_t)p.A % 16 || (uintptr_t)p.B % 16) return false;
  } else {
    if (p.K % 8) return false;
    if ((uintptr_t)p.ah % 16 || (uintptr_t)p.bh % 16) return false;
    if (p.kind == UPIR_BODY_MATMUL_SPLIT3 && ((uintptr_t)p.al % 16 || (uintptr_t)p.bl % 16)) return false;
  }
  return true;
}

template <class Kern>
static hipError_t go_mm(Kern k, const MatmulP &p, const SchedK &S, size_t lds, hipStream_t st) {
  static bool attr_set = false;  // raise the dynamic LDS limit once per kernel
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k, dim3(S.T), dim3(S.U), lds, st, p, S);
  return hipGetLastError();
}

hipError_t launch_matmul_mfma(const MatmulP &p, const LoopK &, const SchedK &S, hipStream_t st) {
  const int bm = S.tile[0], bn = S.tile[1];
  // LDS bytes = stages x (BM + BN) rows x pitch x 2 bytes (x 2 for the lo halves)
  if (p.kind == UPIR_BODY_MATMUL_BF16) {
    if (bm == 256) return go_mm(k_mm_bf16<1, 256, 256, 2, 4, 64, 2>, p, S, 2 * (256 + 256) * 72 * 2, st);
    return go_mm(k_mm_bf16<1, 128, 128, 2, 2, 64, 2>, p, S, 2 * (128 + 128) * 72 * 2, st);
  }
  if (p.kind == UPIR_BODY_MATMUL_SPLIT3) {
    if (bm == 256) return go_mm(k_mm_bf16<3, 256, 256, 2, 4, 32, 1>, p, S, 2 * (256 + 256) * 40 * 2, st);
    return go_mm(k_mm_bf16<3, 128, 128, 2, 2, 32, 2>, p, S, 2 * 2 * (128 + 128) * 40 * 2, st);
  }
  if (bm == 256 && bn == 128) return go_mm(k_mm_f32<256, 128, 4, 2, 32>, p, S, (256 * 36 + 32 * 136) * 4, st);
  return go_mm(k_mm_f32<128, 128, 2, 2, 32>, p, S, (128 * 36 + 32 * 136) * 4, st);
}

}  // namespace upir
