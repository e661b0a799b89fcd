// Internal declarations of the warm-start network's kernels (k_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// epilogues of the matrix-core product
enum GemmEpilogue { EP_STORE = 0, EP_BIAS_GELU = 1, EP_BIAS = 2, EP_GELU_GRAD = 3 };

// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak] (FP32),
// B(k, n) = B[k sbk + n sbn] (FP32 or BF16 bits); operands rounded to BF16,
// FP32 accumulation; epilogue as GemmEpilogue (bias, Z: see k_mlp.hip).
hipError_t launch_gemm_f32(int ep, const float* A, int64_t sam, int64_t sak, const float* B,
                           int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias,
                           float* Z, int M, int N, int K, hipStream_t s);
hipError_t launch_gemm_bf16(int ep, const float* A, int64_t sam, int64_t sak, const uint16_t* B,
                            int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias,
                            float* Z, int M, int N, int K, hipStream_t s);
hipError_t launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s);
hipError_t launch_mse(const float* Y, const float* T, int64_t count, float* dY, float* loss,
                      hipStream_t s);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, float bc1, float bc2, hipStream_t s);
hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s);

}  // namespace pic
