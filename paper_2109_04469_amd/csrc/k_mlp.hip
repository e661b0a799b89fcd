// Kernels of the warm-start network: a plain MLP (GELU hidden layers, linear
// output) with BF16 weights and FP32 accumulation, trained with Adam.
//
// The dense products run on the matrix cores: v_mfma_f32_32x32x16_bf16
// (gfx950) takes a 32x16 block of A and a 16x32 block of B, both rounded to
// BF16, and accumulates the 32x32 product in FP32. A workgroup of four waves
// computes a 64x64 tile of C, one 32x32 quarter per wave. K advances in
// chunks of 32: the workgroup loads the chunk's 64x32 block of A and 32x64
// block of B from global memory with consecutive threads on consecutive
// addresses (along k or along m / n, whichever is contiguous), rounds them
// to BF16 into LDS (rows of m or n, k contiguous), and each wave then reads
// its fragments from LDS, 16 bytes per lane. Bounds are checked on the
// loads, so any M, N, K and strides work.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"

namespace pic {

typedef short short8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

template <typename T>
__device__ __forceinline__ float load_elem(const T* p, int64_t i);
template <>
__device__ __forceinline__ float load_elem<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_elem<uint16_t>(const uint16_t* p, int64_t i) {
  return from_bf16(p[i]);
}

constexpr int kGemmKC = 32;              // k per chunk
constexpr int kGemmLd = kGemmKC + 8;      // LDS row length in BF16 (16-byte rows, padded)

// One 64 x kGemmKC block of a matrix X(r, k) = X[r sr + k sk] into LDS rows
// (r, k contiguous) as BF16, zero outside [0, R) x [0, K). 256 threads, 8
// elements each; consecutive threads walk the contiguous dimension.
template <typename T>
__device__ __forceinline__ void stage_block(const T* __restrict__ X, int64_t sr, int64_t sk, int r0,
                                            int k0, int R, int K, uint16_t* sX) {
  const int tid = threadIdx.x;
  if (sk == 1) {
    // k contiguous: thread t takes row t / 4, k (t % 4) * 8 .. + 7
    const int rr = tid >> 2, kk = (tid & 3) * 8;
    const int r = r0 + rr;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + kk + q;
      const float v = (r < R && k < K) ? load_elem<T>(X, (int64_t)r * sr + k) : 0.0f;
      sX[rr * kGemmLd + kk + q] = to_bf16(v);
    }
  } else {
    // r contiguous (or neither): thread t takes k t / 8, rows (t % 8) * 8 .. + 7
    const int kk = tid >> 3, rb = (tid & 7) * 8;
    const int k = k0 + kk;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = r0 + rb + q;
      const float v = (r < R && k < K) ? load_elem<T>(X, (int64_t)r * sr + (int64_t)k * sk) : 0.0f;
      sX[(rb + q) * kGemmLd + kk] = to_bf16(v);
    }
  }
}

// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] (FP32) and
// B(k, n) = B[k sbk + n sbn] (FP32 or BF16), both rounded to BF16 for the
// product. Epilogue (ep):
//   EP_STORE      C[m][n] = acc
//   EP_BIAS_GELU  Z[m][n] = acc + bias[n], C[m][n] = gelu(Z)   (hidden layer)
//   EP_BIAS       C[m][n] = acc + bias[n]                       (output layer)
//   EP_GELU_GRAD  C[m][n] = acc * gelu'(Z[m][n])                (back through a hidden layer)
template <typename TB, int EP>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int64_t sam, int64_t sak,
                                              const TB* __restrict__ B, int64_t sbk, int64_t sbn,
                                              float* __restrict__ C, int64_t ldc,
                                              const float* __restrict__ bias, float* Z, int M, int N,
                                              int K) {
  __shared__ __align__(16) uint16_t sA[64 * kGemmLd];  // rows m, k contiguous
  __shared__ __align__(16) uint16_t sB[64 * kGemmLd];  // rows n, k contiguous
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int r = lane & 31;        // row of A / column of B this lane feeds
  const int kh = (lane >> 5) * 8;  // which eight k of a 16-k step
  f32x16 acc = {};
  for (int k0 = 0; k0 < K; k0 += kGemmKC) {
    stage_block<float>(A, sam, sak, bm, k0, M, K, sA);
    // B(k, n) as rows of n: X(n, k) = B[n sbn + k sbk]
    stage_block<TB>(B, sbn, sbk, bn, k0, N, K, sB);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGemmKC; ks += 16) {
      const short8 a = *reinterpret_cast<const short8*>(&sA[(wm + r) * kGemmLd + ks + kh]);
      const short8 b = *reinterpret_cast<const short8*>(&sB[(wn + r) * kGemmLd + ks + kh]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j]: lane j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8)
  const int n = bn + wn + (lane & 31);
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    const int m = bm + wm + 8 * (g >> 2) + 4 * (lane >> 5) + (g & 3);
    if (m >= M || n >= N) continue;
    const int64_t o = (int64_t)m * ldc + n;
    float v = acc[g];
    if (EP == EP_BIAS_GELU) {
      v += bias[n];
      Z[o] = v;
      v = gelu(v);
    } else if (EP == EP_BIAS) {
      v += bias[n];
    } else if (EP == EP_GELU_GRAD) {
      v *= gelu_grad(Z[o]);
    }
    C[o] = v;
  }
}

// db[n] = sum_m dZ[m][n] (one thread per column, fixed order)
__global__ void k_colsum(const float* __restrict__ dZ, int M, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int m = 0; m < M; ++m) s += dZ[(int64_t)m * N + n];
  db[n] = s;
}

// Mean squared error over M x N and its gradient dY = 2 (Y - T) / (M N).
// One workgroup of 1024 threads, fixed reduction order.
__global__ __launch_bounds__(1024) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                              int64_t count, float* __restrict__ dY,
                                              float* __restrict__ loss) {
  __shared__ float s_part[1024 / 64];
  const float scale = 2.0f / (float)count;
  float s = 0.0f;
  for (int64_t i = threadIdx.x; i < count; i += 1024) {
    const float d = Y[i] - T[i];
    dY[i] = scale * d;
    s += d * d;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < 1024 / 64; ++w) t += s_part[w];
    *loss = t / (float)count;
  }
}

// AdamW on the FP32 master copy, then the BF16 working copy of the weight
// matrices. bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                       float eps, float wd, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1;
  const float vh = vi / bc2;
  w[i] = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
}

__global__ void k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = to_bf16(src[i]);
}

// ---------------------------------------------------------------------------
// host launchers

static dim3 gemm_grid(int M, int N) { return dim3((N + 63) / 64, (M + 63) / 64); }

hipError_t launch_gemm_f32(int ep, const float* A, int64_t sam, int64_t sak, const float* B,
                           int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias,
                           float* Z, int M, int N, int K, hipStream_t s) {
  if (M < 1 || N < 1 || K < 1) return hipErrorInvalidValue;
  const dim3 g = gemm_grid(M, N);
  switch (ep) {
    case EP_STORE:
      hipLaunchKernelGGL((k_gemm<float, EP_STORE>), g, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C,
                         ldc, bias, Z, M, N, K);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(int ep, const float* A, int64_t sam, int64_t sak, const uint16_t* B,
                            int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias,
                            float* Z, int M, int N, int K, hipStream_t s) {
  if (M < 1 || N < 1 || K < 1) return hipErrorInvalidValue;
  const dim3 g = gemm_grid(M, N);
  switch (ep) {
    case EP_STORE:
      hipLaunchKernelGGL((k_gemm<uint16_t, EP_STORE>), g, dim3(256), 0, s, A, sam, sak, B, sbk, sbn,
                         C, ldc, bias, Z, M, N, K);
      break;
    case EP_BIAS_GELU:
      hipLaunchKernelGGL((k_gemm<uint16_t, EP_BIAS_GELU>), g, dim3(256), 0, s, A, sam, sak, B, sbk,
                         sbn, C, ldc, bias, Z, M, N, K);
      break;
    case EP_BIAS:
      hipLaunchKernelGGL((k_gemm<uint16_t, EP_BIAS>), g, dim3(256), 0, s, A, sam, sak, B, sbk, sbn,
                         C, ldc, bias, Z, M, N, K);
      break;
    case EP_GELU_GRAD:
      hipLaunchKernelGGL((k_gemm<uint16_t, EP_GELU_GRAD>), g, dim3(256), 0, s, A, sam, sak, B, sbk,
                         sbn, C, ldc, bias, Z, M, N, K);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, dZ, M, N, db);
  return hipGetLastError();
}

hipError_t launch_mse(const float* Y, const float* T, int64_t count, float* dY, float* loss,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, Y, T, count, dY, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, n, lr,
                     b1, b2, eps, wd, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace pic
