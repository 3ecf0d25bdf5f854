// Host-side launchers of the HIP kernels (internal to libupir).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "upir_kern.h"

namespace upir {

// Kernel variants a loop can run with (reported by upir_loop_resolve).
enum Variant : int32_t {
  V_GENERIC = 0,      // schedule-exact generic worksharing kernel
  V_STREAM4 = 1,      // 1-D, static chunk 4, vectorised (AXPY, SUM f32, COVER)
  V_JACOBI_TILE = 2,  // tiled Jacobi, wavefront strips
  V_MATVEC_WAVE = 3,  // one wavefront per row
  V_MATMUL_MFMA = 4,  // MFMA tiles over C
  V_DYNAMIC = 5,      // dynamic / guided claim loop (generic bodies)
  V_FILTER7_TILE = 6, // tiled 7 x 7 filter, wavefront strips
};

// Body payloads with device pointers already resolved.
struct AxpyP { float a; const float *x; float *y; };
struct SumP { const void *x; int32_t dtype; };
struct JacobiP { const float *src; float *dst; int64_t ld; };
struct MatmulP {
  const float *A, *B; float *C; int64_t M, N, K, lda, ldb, ldc;
  uint16_t *ah, *al, *bh, *bl;  // bfloat16 workspace (bh/bl stored transposed: N x K)
  int32_t kind;                 // 4 = f32, 5 = bf16, 6 = split3
  int32_t panel;                // workspace layout: 0 rows of K; 1 k-panels of 32 (see kernels_matmul.hip)
};
// Workspace k extent: K rounded up to the 32-wide k-panels.
__host__ __device__ inline int64_t mm_kpad(int64_t K) { return (K + 31) / 32 * 32; }
struct MatvecP { const float *A; const float *x; float *y; int64_t cols, lda; };
struct OwnerP { int32_t *out; };
struct CoverP { int32_t *count; };
struct Filter7P { const float *src; float *dst; const float *w; int64_t ld; };

hipError_t launch_generic(int32_t body, const void *payload, const LoopK &L, const SchedK &S,
                          const RedK &R, hipStream_t st);
hipError_t launch_stream4(int32_t body, const void *payload, const LoopK &L, const SchedK &S,
                          const RedK &R, hipStream_t st);
hipError_t launch_fold(const FoldK &F, hipStream_t st);
hipError_t launch_jacobi_tile(const JacobiP &p, const LoopK &L, const SchedK &S, const RedK &R,
                              hipStream_t st);
hipError_t launch_filter7_tile(const Filter7P &p, const LoopK &L, const SchedK &S, const RedK &R,
                               hipStream_t st);
hipError_t launch_matvec_wave(const MatvecP &p, const LoopK &L, const SchedK &S, const RedK &R,
                              hipStream_t st);
// MFMA matmul over tiles of C (tile[0] x tile[1]); S gives the team schedule over tiles.
hipError_t launch_matmul_mfma(const MatmulP &p, const LoopK &L, const SchedK &S, hipStream_t st);
bool matmul_mfma_supports(const MatmulP &p, const LoopK &L, const SchedK &S);
// BF16 pre-pass: A (M x K) -> ah, al; B (K x N) -> bh, bl transposed (N x K).
hipError_t launch_bf16_split(const MatmulP &p, bool need_lo, hipStream_t st);
// The 256 x 256 four-wavefront bfloat16 tile (it reads the k-panel workspace layout).
bool matmul_wide(const MatmulP &p, const SchedK &S);

// Jacobi tiled kernel constraints.
bool jacobi_tile_supports(const JacobiP &p, const LoopK &L, const SchedK &S);
bool filter7_tile_supports(const Filter7P &p, const LoopK &L, const SchedK &S);

}  // namespace upir
