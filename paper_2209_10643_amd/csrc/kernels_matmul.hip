// Dense matmul loop C = A B (gfx950): bfloat16 split pre-pass and MFMA tiles.
//
// Paper: sec. 6.2 names a matrix multiplication kernel among its four
// offloaded loops; its source and precision are not given. The loop here is
// collapse(2) over C with the k reduction in the body. Precision variants
// (not in the paper): float32; A, B rounded to bfloat16 (round to nearest
// even) with float32 accumulation; and the three-pass split
// A_lo B_hi + A_hi B_lo + A_hi B_hi that recovers float32 accuracy.
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

hipError_t launch_bf16_split(const MatmulP &p, bool need_lo, hipStream_t st) {
  if (p.M > 0 && p.K > 0) {
    const int64_t tot = p.M * p.K;
    const int g = (int)std::min<int64_t>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(k_split_rows, dim3(g), dim3(256), 0, st, p.A, p.M, p.K, p.lda, p.ah, need_lo ? p.al : nullptr);
  }
  if (p.N > 0 && p.K > 0) {
    dim3 g((unsigned)((p.N + 63) / 64), (unsigned)((p.K + 63) / 64));
    hipLaunchKernelGGL(k_split_cols, g, dim3(256), 0, st, p.B, p.K, p.N, p.ldb, p.bh, need_lo ? p.bl : nullptr);
  }
  return hipGetLastError();
}

bool matmul_mfma_supports(const MatmulP &, const LoopK &, const SchedK &) { return false; }

hipError_t launch_matmul_mfma(const MatmulP &, const LoopK &, const SchedK &, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace upir
