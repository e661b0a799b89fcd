// Small kernels: the deposit of a freshly loaded species (pic_set_state) and
// the device self-checks of the generator and of FP64 sqrt.
#include "pic_internal.h"

namespace pic {

__global__ __launch_bounds__(256) void k_deposit(const double* x, const int64_t* count,
                                                 double inv_dx, int nx, unsigned long long* dep) {
  const int64_t n = *count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int j;
    double f;
    int64_t w1;
    cell_of(x[i], inv_dx, nx, j, f, w1);
    atomicAdd(&dep[j], (unsigned long long)(kOne32 - w1));
    atomicAdd(&dep[j + 1], (unsigned long long)w1);
  }
}

hipError_t launch_deposit(const double* x, const int64_t* count, double inv_dx, int nx,
                          unsigned long long* dep, hipStream_t s) {
  hipLaunchKernelGGL(k_deposit, dim3(1024), dim3(256), 0, s, x, count, inv_dx, nx, dep);
  return hipGetLastError();
}

__global__ void k_selftest_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 r = philox(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]),
                         k0, k1);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

__global__ void k_selftest_sqrt(const double* in, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt(in[i]);
}

__global__ __launch_bounds__(256) void k_iota(uint32_t* id, const int64_t* count) {
  const int64_t n = *count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    id[i] = (uint32_t)i;
}

hipError_t launch_iota(uint32_t* id, const int64_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(1024), dim3(256), 0, s, id, count);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather(const uint32_t* id, const double* vy,
                                                const double* vz, double* out_y, double* out_z,
                                                int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = id[i];
    out_y[i] = vy[k];
    out_z[i] = vz[k];
  }
}

hipError_t launch_gather(const uint32_t* id, const double* vy, const double* vz, double* out_y,
                         double* out_z, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gather, dim3(1024), dim3(256), 0, s, id, vy, vz, out_y, out_z, n);
  return hipGetLastError();
}

// Plain streaming copy, 16 bytes per lane per iteration: the reference
// kernel for achievable HBM bandwidth and for scaling traffic counters.
__global__ __launch_bounds__(256) void k_selftest_copy(const double2* __restrict__ in,
                                                        double2* __restrict__ out, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
    out[i] = in[i];
}

hipError_t launch_selftest_copy(const double* in, double* out, int64_t n, hipStream_t s) {
  const int64_t n2 = n / 2;
  int64_t g = (n2 + 255) / 256;
  if (g > 65536) g = 65536;
  if (g > 0)
    hipLaunchKernelGGL(k_selftest_copy, dim3((unsigned)g), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out), n2);
  return hipGetLastError();
}

hipError_t launch_selftest_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                                  int64_t n, hipStream_t s) {
  const int64_t g = (n + 255) / 256;
  if (g > 0) hipLaunchKernelGGL(k_selftest_philox, dim3((unsigned)g), dim3(256), 0, s, ctr, k0, k1, out, n);
  return hipGetLastError();
}

hipError_t launch_selftest_sqrt(const double* in, double* out, int64_t n, hipStream_t s) {
  const int64_t g = (n + 255) / 256;
  if (g > 0) hipLaunchKernelGGL(k_selftest_sqrt, dim3((unsigned)g), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace pic
