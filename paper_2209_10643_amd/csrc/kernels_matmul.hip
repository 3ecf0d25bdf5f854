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

// Workspace element (row, k) of an operand with `rows` rows: rows of K
// (layout 0), or k-panels of 32 (layout 1): panel k / 32 holds 32 k of every
// row, row after row, so the rows x 32 block one k step reads is contiguous.
__device__ inline int64_t ws_index(int panel, int64_t row, int64_t k, int64_t rows, int64_t K) {
  return panel ? (((k >> 5) * rows + row) << 5) + (k & 31) : row * K + k;
}

// A (M x K, lda) -> ah / al (M x K, dense). Row-major, coalesced.
__global__ void __launch_bounds__(256) k_split_rows(const float *__restrict__ A, int64_t M, int64_t K, int64_t lda,
                                                    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int panel) {
  const int64_t total = M * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / K, k = e - i * K, d = ws_index(panel, i, k, M, K);
    const float x = A[i * lda + k];
    const uint16_t h = to_bf16_rne(x);
    hi[d] = h;
    if (lo) lo[d] = to_bf16_rne(x - bf16f(h));
  }
}

// B (K x N, ldb) -> bh / bl transposed (N x K, dense) through a 64 x 64 LDS tile.
__global__ void __launch_bounds__(256) k_split_cols(const float *__restrict__ B, int64_t K, int64_t N, int64_t ldb,
                                                    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int panel) {
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
      const int64_t d = ws_index(panel, n, k, N, K);
      hi[d] = h;
      if (lo) lo[d] = to_bf16_rne(x - bf16f(h));
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
                                                     uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int panel) {
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
    const int64_t d = ws_index(panel, i, k, M, K);  // 8 | k: the eight stay in one panel
    *(u32x4s *)(hi + d) = u32x4s{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
    if (lo) *(u32x4s *)(lo + d) = u32x4s{pack2(l[0], l[1]), pack2(l[2], l[3]), pack2(l[4], l[5]), pack2(l[6], l[7])};
  }
}

// B (K x N) -> N x K through a 64 (k) x 64 (n) LDS tile: rows of B are read
// as float4, each output row n gets its 64 k as eight 16-byte stores.
__global__ void __launch_bounds__(256) k_split_cols8(const float *__restrict__ B, int64_t K, int64_t N, int64_t ldb,
                                                     uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int panel) {
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
    const int64_t d = ws_index(panel, n, k, N, K);
    *(u32x4s *)(hi + d) = u32x4s{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
    if (lo) *(u32x4s *)(lo + d) = u32x4s{pack2(l[0], l[1]), pack2(l[2], l[3]), pack2(l[4], l[5]), pack2(l[6], l[7])};
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
                         need_lo ? p.al : nullptr, p.panel);
    } else {
      const int64_t tot = p.M * p.K;
      const int g = (int)std::min<int64_t>((tot + 255) / 256, 8192);
      hipLaunchKernelGGL(k_split_rows, dim3(g), dim3(256), 0, st, p.A, p.M, p.K, p.lda, p.ah,
                         need_lo ? p.al : nullptr, p.panel);
    }
  }
  if (p.N > 0 && p.K > 0) {
    dim3 g((unsigned)((p.N + 63) / 64), (unsigned)((p.K + 63) / 64));
    if (vec_b)
      hipLaunchKernelGGL(k_split_cols8, g, dim3(256), 0, st, p.B, p.K, p.N, p.ldb, p.bh, need_lo ? p.bl : nullptr,
                         p.panel);
    else
      hipLaunchKernelGGL(k_split_cols, g, dim3(256), 0, st, p.B, p.K, p.N, p.ldb, p.bh, need_lo ? p.bl : nullptr,
                         p.panel);
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
// 32 x 32 MFMA blocks. K advances in steps of BK. In the tiles below
// (k_mm_bf16, k_mm_f32) the next step's operands are fetched from global
// memory into registers while the current step's operands, staged in LDS
// (padded or swizzled rows: no bank conflicts on the fragment reads), feed
// the matrix cores; the four-wave 256 x 256 tile further down
// (k_mm_bf16_wide) loads straight into a ring of LDS stages instead.
//
// bfloat16 variants use v_mfma_f32_32x32x16_bf16 (lane l supplies row l%32
// and 8 consecutive k of group l/32); both hi/lo operands come from the
// pre-pass workspace (A as M x K, B transposed as N x K, or k-panels of 32
// for the wide tile). The split variant accumulates lo_A hi_B, hi_A lo_B and
// hi_A hi_B into one float32 sum. float32 uses v_mfma_f32_32x32x2f32 over A
// (M x K) and B (K x N) directly.
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

// The same stores with the non-temporal hint (C is written once and not read
// again here); the row and column tests are hoisted out of the element loop,
// and left out for tiles known to be whole (CHECK false: each test became a
// branch around its store).
// (A form through a buffer resource with __builtin_amdgcn_raw_buffer_store_b32
// was compiled to stores that all took the same accumulator register.)
template <int BM, int BN, int WM, int WN, bool CHECK = true>
__device__ inline void store_c_nt(const MatmulP &p, int64_t row0, int64_t col0, const f32x16 (&acc)[BM / WM / 32][BN / WN / 32]) {
  constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = col0 + wn * (BN / WN) + j * 32 + (lane & 31);
      const int64_t rb = row0 + wm * (BM / WM) + i * 32 + 4 * (lane >> 5);
      float *cp = p.C + rb * p.ldc + col;
      const bool cin = col < p.N;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ro = 8 * (r / 4) + (r % 4);
        if (!CHECK || (cin && rb + ro < p.M)) __builtin_nontemporal_store(acc[i][j][r], cp + ro * p.ldc);
      }
    }
}

// Chunk swizzle of LDS rows of 64 bytes (four 16-byte chunks): chunk c of
// row r is stored at chunk c ^ swz(r), swz(r) = r2 | (r1 ^ r3) << 1 over the
// bits of r. The sixteen consecutive rows a 16-lane phase of a 16-byte read
// touches (4 rows per 256 bytes of banks) then fall on distinct banks, and so
// do the eight rows of an 8-lane phase (2 rows per 128 bytes); a phase that
// writes four whole rows covers the banks once whatever the swizzle.
__device__ inline int mmw_swz(int r) { return ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1); }

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
  // LDS rows: 64 k with 8 halfwords of padding (no conflicts), or 32 k with
  // the chunk swizzle (padded 80-byte rows had conflicting staging writes)
  constexpr bool SWZ = BK == 32;
  constexpr int PITCH = SWZ ? BK : BK + 8;  // halfwords per LDS row (16-byte multiple)
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
        const int c = tid + q * NTH, r = c / CPR, kc = SWZ ? (c % CPR) ^ mmw_swz(c / CPR) : c % CPR;
        *(u32x4 *)(sAh + r * PITCH + kc * 8) = ra[q];
        if (NPROD == 3) *(u32x4 *)(sAl + r * PITCH + kc * 8) = ral[q];
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        const int c = tid + q * NTH, r = c / CPR, kc = SWZ ? (c % CPR) ^ mmw_swz(c / CPR) : c % CPR;
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
        // rows read here are = lane mod 32 (mod 32): the swizzle of the row is that of lane mod 32
        const int koff = SWZ ? (((ks >> 3) + (lane >> 5)) ^ mmw_swz(lane & 31)) * 8 : ks + 8 * (lane >> 5);
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

// 256 x 256 tiles on four waves (2 x 2), each wave 128 x 128 of C as 4 x 4
// blocks of v_mfma_f32_32x32x16_bf16: twice the flops per fragment read from
// LDS of the eight-wave tile above, whose fragment reads and staging writes
// together kept the LDS close to saturation.
//
// Operands go from the workspace straight into LDS (buffer_load ... lds, no
// staging registers; offsets past the operand read as zero, which also pads
// the k tail) through a ring of five stages of BK = 32. The pre-pass writes
// the workspace in k-panels of 32 (ws_index layout 1), so the 256 rows x 32 k
// one step needs are 16 KB of contiguous memory: with rows of K, each row's
// 64 bytes were half of a cache line whose other half the next step fetched
// again (measured on the load path alone: 48 us against 78 us for 4096^3).
// A lane's offset inside a panel is fixed; the panel's offset is the scalar
// offset of the load.
//
// LDS rows hold 32 k (64 bytes, four 16-byte chunks) of one row of A or B;
// chunk c of row r is stored at chunk c ^ swz(r), swz(r) = r2 | (r1 ^ r3) << 1
// over the bits of r: the sixteen consecutive rows a 16-lane phase of a
// 16-byte read touches (4 rows per 256 bytes of banks) then fall on distinct
// banks, and so do the eight rows of an 8-lane phase.
//
// Software pipeline over k steps, one phase per step u: wait until step u's
// loads have landed (each wave's own count, then a barrier for everyone's),
// issue four matrix instructions of step u - 1, then read step u's sixteen
// fragments into the second register set spread over the next sixteen
// matrix instructions, with the eight loads of step u + 4 (into the slot
// step u - 1 used) issued after every second read, and finish step u - 1's
// 32. The matrix cores are thus never left waiting on LDS reads (reading all
// fragments before the MFMAs left them idle a third of the time), and the
// loads run four steps ahead; spreading the loads over the phase instead of
// issuing them together cut a 4096^3 product from 119 to 110 us in a
// standalone copy of the tile on random data. Each wave's
// reads of step u - 1 are complete before the barrier of phase u, so that
// slot is free for reuse by then. Steps past the last one load panel 0 again
// into a slot nobody reads, which keeps the wait counts the same in every
// phase; the last wait of a tile drains them before LDS is reused.
//
// Tiles are visited in groups of four tile rows, column by column inside a
// group, so the 32 consecutive tiles one XCD runs at a time share four A
// panels and eight B panels in that XCD's L2 (rather than two and sixteen).
//
// NSEG = 3 runs the split product as one bfloat16 GEMM over K' = 3K: the
// k steps walk (A_lo, B_hi), then (A_hi, B_lo), then (A_hi, B_hi), so the
// small terms are summed first, all in the float32 accumulators.
// EVEN: the step count (NSEG x ceil(K / 32)) is even, which fixes which of
// the two fragment register sets holds the last step.
constexpr int MMW_BK = 32, MMW_ROWB = 64, MMW_STAGES = 5, MMW_STAGE = 512 * MMW_ROWB;

// s_waitcnt with only the vector-memory counter limited to n (other counters at their maximum)
template <int N>
__device__ inline void wait_vm() {
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// s_waitcnt lgkmcnt(0) (LDS reads of this wave complete), other counters at their maximum
__device__ inline void wait_lds() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }

// The operands of one k step of the wide tile: buffer resources of the A
// and B arrays it reads, their k-panel byte offsets (the loads' scalar
// offsets), whether this lane's k chunk lies below K, and the LDS stage.
struct MmwStep {
  __amdgpu_buffer_rsrc_t ra, rb;
  uint32_t sa, sb;
  bool kin;
  unsigned char *dst;
};

bool matmul_wide(const MatmulP &p, const SchedK &S) {
  return p.kind != UPIR_BODY_MATMUL_F32 && S.tile[0] == 256 && S.tile[1] == 256 && S.U == 256;
}

template <int NSEG, bool ALIGNED, bool EVEN>
__global__ void __launch_bounds__(256) k_mm_bf16_wide(MatmulP p, SchedK S) {
  constexpr int BM = 256, ROWB = MMW_ROWB, STAGE = MMW_STAGE, NST = MMW_STAGES;
  constexpr int AHEAD = NST - 1;   // phase u issues the loads of step u + AHEAD
  constexpr int LOADS = 8;         // load instructions per wave per step (4 of A, 4 of B: 16 rows each)
  constexpr int PRE = 4, SPAN = 16;  // MFMAs before the first fragment read; MFMAs the reads spread over
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_w[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int64_t K = p.K, KP = mm_kpad(K);
  // the host admits this kernel only with every operand under 2 GiB, so steps fit in int
  const int seg_steps = (int)((K + MMW_BK - 1) / MMW_BK), steps = NSEG * seg_steps;
  const __amdgpu_buffer_rsrc_t rah = __builtin_amdgcn_make_buffer_rsrc((void *)p.ah, (short)0, (int)(p.M * KP * 2), 0x00020000);
  const __amdgpu_buffer_rsrc_t rbh = __builtin_amdgcn_make_buffer_rsrc((void *)p.bh, (short)0, (int)(p.N * KP * 2), 0x00020000);
  const __amdgpu_buffer_rsrc_t ral = NSEG == 3 ? __builtin_amdgcn_make_buffer_rsrc((void *)p.al, (short)0, (int)(p.M * KP * 2), 0x00020000) : rah;
  const __amdgpu_buffer_rsrc_t rbl = NSEG == 3 ? __builtin_amdgcn_make_buffer_rsrc((void *)p.bl, (short)0, (int)(p.N * KP * 2), 0x00020000) : rbh;
  // this lane's place in every 16-row load group: row rr of the group,
  // physical chunk lane % 4, which holds logical chunk lc
  const int rr = lane >> 2, lc = (lane & 3) ^ mmw_swz(rr);
  // fragment reads: row (lane mod 32) of a 32-row block, k group lane / 32;
  // byte offsets inside a stage for k half 0 / 1 of A and of B
  const int fr = lane & 31, fsw = mmw_swz(fr), hg = lane >> 5;
  const int fa0 = (wm * 128 + fr) * ROWB + ((hg ^ fsw) << 4), fa1 = (wm * 128 + fr) * ROWB + (((2 + hg) ^ fsw) << 4);
  const int fb0 = BM * ROWB + (wn * 128 + fr) * ROWB + ((hg ^ fsw) << 4);
  const int fb1 = BM * ROWB + (wn * 128 + fr) * ROWB + (((2 + hg) ^ fsw) << 4);
  const uint32_t pa = (uint32_t)(p.M * 64), pb = (uint32_t)(p.N * 64);  // bytes per k-panel

  for_team_tiles(S, [&](int64_t m) {
    // grouped tile order: groups of G tile rows, column-major inside a group
    const int64_t nt0 = S.nt[0], nt1 = S.nt[1], G = 4;
    const int64_t grp = m / (G * nt1), in = m - grp * G * nt1;
    const int64_t gsz = std::min<int64_t>(G, nt0 - grp * G);
    const int64_t trow = grp * G + in % gsz, tcol = in / gsz;
    const int64_t row0 = (S.t0[0] + trow) * BM, col0 = (S.t0[1] + tcol) * BM;
    f32x16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x16{};
    // this lane's byte offsets in k-panel 0 for its four row groups (32-bit:
    // every operand is under 2 GiB), and whether its rows exist
    uint32_t oa0[4], ob0[4];
    bool va[4], vb[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int r = wave * 64 + g * 16 + rr;
      oa0[g] = (uint32_t)(((row0 + r) * 32 + lc * 8) * 2);
      ob0[g] = (uint32_t)(((col0 + r) * 32 + lc * 8) * 2);
      va[g] = ALIGNED || row0 + r < p.M;
      vb[g] = ALIGNED || col0 + r < p.N;
    }
    // the next step to load: its index, segment and k-panel (scalars)
    int lt = 0, lseg = 0, lkt = 0;
    // the operands of step lt (segment for NSEG = 3, k-panel; steps past the
    // end load panel 0) and the LDS stage that receives them
    auto step_ops = [&](int slot) {
      const bool live = lt < steps;
      const int kt = live ? lkt : 0, seg = NSEG == 3 && live ? lseg : 0;
      MmwStep o;
      o.ra = seg == 0 ? ral : rah;
      o.rb = seg == 1 ? rbl : rbh;
      o.sa = (uint32_t)kt * pa;
      o.sb = (uint32_t)kt * pb;
      o.kin = ALIGNED || (int64_t)kt * MMW_BK + lc * 8 < K;
      o.dst = lds_w + slot * STAGE + wv * 64 * ROWB;
      return o;
    };
    // load instruction idx (0..7: row group idx / 2, A if even, B if odd)
    auto load_one = [&](const MmwStep &o, int idx) {
      const bool isb = idx & 1;
      const int g = idx >> 1;
      // ragged shapes: rows past M or N and k past K read as zero
      const uint32_t vo = ALIGNED || ((isb ? vb[g] : va[g]) && o.kin) ? (isb ? ob0[g] : oa0[g]) : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(isb ? o.rb : o.ra,
                                               (__attribute__((address_space(3))) void *)(o.dst + (isb ? BM * ROWB : 0) + g * 16 * ROWB),
                                               16, vo, isb ? o.sb : o.sa, 0, 0);
    };
    auto advance = [&] {
      ++lt;
      if (++lkt == seg_steps) {
        lkt = 0;
        ++lseg;
      }
    };
    auto load_next = [&](int slot) {
      const MmwStep o = step_ops(slot);
#pragma unroll
      for (int idx = 0; idx < LOADS; ++idx) load_one(o, idx);
      advance();
    };
    // fragment q of a step (k half q / 8; 0-3: A blocks, 4-7: B blocks) from the stage at byte sbase
    auto read_one = [&](int sbase, bf16x8 (&Y)[2][8], int q) {
      const int ks = q >> 3, x = q & 7;
      const int off = x < 4 ? (ks ? fa1 : fa0) + x * 32 * ROWB : (ks ? fb1 : fb0) + (x - 4) * 32 * ROWB;
      Y[ks][x] = *(const bf16x8 *)(lds_w + sbase + off);
    };
    // matrix instructions lo..hi-1 of a step: k half q / 16, block (q / 4 mod 4, q mod 4)
    auto mfmas = [&](bf16x8 (&X)[2][8], int lo, int hi) {
#pragma unroll
      for (int q = lo; q < hi; ++q) {
        const int ks = q >> 4, i = (q >> 2) & 3, j = q & 3;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X[ks][i], X[ks][4 + j], acc[i][j], 0, 0, 0);
      }
    };
    auto bar = [] {
      // a bare barrier: __syncthreads() adds a workgroup release fence, which
      // waits for every load in flight (the loads into LDS count as
      // vector-memory operations) and would drain the ring at every step
      __asm__ volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      __asm__ volatile("" ::: "memory");
    };
    int rslot = 0, lslot = AHEAD;  // stage of step u, stage that receives step u + AHEAD
    // phase u: X holds step u - 1's fragments, Y receives step u's
    auto phase = [&](bf16x8 (&X)[2][8], bf16x8 (&Y)[2][8]) {
      rslot = rslot + 1 == NST ? 0 : rslot + 1;
      lslot = lslot + 1 == NST ? 0 : lslot + 1;
      wait_vm<(AHEAD - 1) * LOADS>();  // step u's loads (AHEAD - 1 later steps may be pending)
      wait_lds();                      // this wave's reads of step u - 1 (slot lslot) are done
      bar();
      __builtin_amdgcn_sched_barrier(0);
      mfmas(X, 0, PRE);
      const int sbase = rslot * STAGE;
      const MmwStep o = step_ops(lslot);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        __builtin_amdgcn_sched_barrier(0);
        read_one(sbase, Y, q);
        if (q & 1) load_one(o, q >> 1);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(X, PRE + (q * SPAN) / 16, PRE + ((q + 1) * SPAN) / 16);
      }
      advance();
      __builtin_amdgcn_sched_barrier(0);
      mfmas(X, PRE + SPAN, 32);
      __builtin_amdgcn_sched_barrier(0);
    };
    __syncthreads();  // the previous tile's readers are done with LDS
    if (steps > 0) {
      bf16x8 F[2][8], Gr[2][8];
#pragma unroll
      for (int q = 0; q < AHEAD; ++q) load_next(q);
      wait_vm<(AHEAD - 1) * LOADS>();
      bar();
      load_next(AHEAD);
#pragma unroll
      for (int q = 0; q < 16; ++q) read_one(0, F, q);
      // phases 1 .. steps - 1, two per trip so the register sets swap roles without copies
      for (int u = 1; u + 1 < steps; u += 2) {
        phase(F, Gr);
        phase(Gr, F);
      }
      if (EVEN) {
        phase(F, Gr);
        mfmas(Gr, 0, 32);
      } else {
        mfmas(F, 0, 32);
      }
      wait_vm<0>();  // the loads past the last step have landed before LDS is reused
    }
    store_c_nt<256, 256, 2, 2, !ALIGNED>(p, row0, col0, acc);
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
  constexpr int STAGEF = BM * PA + BK * PB;  // floats per LDS stage (two stages)
  extern __shared__ __attribute__((aligned(16))) float ldsf[];
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
    auto stage = [&](int buf) {
      float *sA = ldsf + buf * STAGEF, *sB = sA + BM * PA;
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
    __syncthreads();  // the previous tile's readers are done with both stages
    fetch(0);
    stage(0);
    __syncthreads();
    const int g = lane >> 5;
    int cur = 0;
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
      const bool more = k0 + BK < K;
      if (more) fetch(k0 + BK);
      const float *sA = ldsf + cur * STAGEF, *sB = sA + BM * PA;
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
      // the next step goes into the other stage; one barrier then both makes
      // it visible and keeps this stage from being overwritten (two steps on)
      // before every wave has read it
      if (more) stage(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
    store_c<BM, BN, WM, WN>(p, row0, col0, acc);
  });
}

// Kernel configurations: (kind, tile) -> block size.
struct MMConf { int kind, bm, bn, threads; };
static const MMConf kMM[] = {
    {UPIR_BODY_MATMUL_BF16, 256, 256, 256}, {UPIR_BODY_MATMUL_SPLIT3, 256, 256, 256},
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
    // the wide tile addresses each operand with 32-bit buffer offsets
    if (matmul_wide(p, S) && (p.M * mm_kpad(p.K) * 2 >= (1LL << 31) || p.N * mm_kpad(p.K) * 2 >= (1LL << 31)))
      return false;
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
  if (matmul_wide(p, S)) {
    // whole tiles and whole k-panels: no bounds tests in the load loop
    const bool al = p.M % 256 == 0 && p.N % 256 == 0 && p.K % MMW_BK == 0;
    const size_t lds = MMW_STAGES * MMW_STAGE;
    const bool even = (p.K + MMW_BK - 1) / MMW_BK % 2 == 0;  // NSEG x steps is even iff steps is
    if (p.kind == UPIR_BODY_MATMUL_BF16) {
      if (al) return even ? go_mm(k_mm_bf16_wide<1, true, true>, p, S, lds, st) : go_mm(k_mm_bf16_wide<1, true, false>, p, S, lds, st);
      return even ? go_mm(k_mm_bf16_wide<1, false, true>, p, S, lds, st) : go_mm(k_mm_bf16_wide<1, false, false>, p, S, lds, st);
    }
    if (al) return even ? go_mm(k_mm_bf16_wide<3, true, true>, p, S, lds, st) : go_mm(k_mm_bf16_wide<3, true, false>, p, S, lds, st);
    return even ? go_mm(k_mm_bf16_wide<3, false, true>, p, S, lds, st) : go_mm(k_mm_bf16_wide<3, false, false>, p, S, lds, st);
  }
  if (p.kind == UPIR_BODY_MATMUL_BF16) {
    if (bm == 256) return go_mm(k_mm_bf16<1, 256, 256, 2, 4, 64, 2>, p, S, 2 * (256 + 256) * 72 * 2, st);
    return go_mm(k_mm_bf16<1, 128, 128, 2, 2, 64, 2>, p, S, 2 * (128 + 128) * 72 * 2, st);
  }
  if (p.kind == UPIR_BODY_MATMUL_SPLIT3) {
    // two stages of (A_hi, B_hi, A_lo, B_lo) x rows x 64 bytes (swizzled, unpadded)
    if (bm == 256) return go_mm(k_mm_bf16<3, 256, 256, 2, 4, 32, 2>, p, S, 2 * 2 * (256 + 256) * 32 * 2, st);
    return go_mm(k_mm_bf16<3, 128, 128, 2, 2, 32, 2>, p, S, 2 * 2 * (128 + 128) * 32 * 2, st);
  }
  // two LDS stages of (BM x (BK + 4) + BK x (BN + 8)) floats
  if (bm == 256 && bn == 128) return go_mm(k_mm_f32<256, 128, 4, 2, 32>, p, S, 2 * (256 * 36 + 32 * 136) * 4, st);
  return go_mm(k_mm_f32<128, 128, 2, 2, 32>, p, S, 2 * (128 * 36 + 32 * 136) * 4, st);
}

}  // namespace upir
