// Batched FP32 MFMA complex GEMM (64 x 64 tiles, 4 waves of 32 x 32), shared by the
// general-spin nucleon path and the two-meson path.
#pragma once

#include <hip/hip_runtime.h>

namespace nuc {
namespace spin {

// C[b] = A[b] B[b] for b < batch, row-major complex FP32: A [M][K] (lda), B [K][N] (ldb),
// C [M][N] (ldc); batch b reads A + ((b / dA) % mA) sA and B + ((b / dB) % mB) sB and
// writes C + b sC. The defaults give plain uniform strides.
hipError_t gemm(const float2* A, const float2* B, float2* C, int M, int N, int K, int lda, int ldb, int ldc,
                long long sA, long long sB, long long sC, int batch, hipStream_t s, int dA = 1, int mA = 1 << 30,
                int dB = 1, int mB = 1 << 30);

}  // namespace spin
}  // namespace nuc
