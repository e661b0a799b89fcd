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

// Particles loaded from a density and a temperature profile given at npts
// equally spaced points on [0, L], both linear in between. Slot i takes the
// position whose cumulative density is u * (total) for its position uniform
// u (inverse of the piecewise-quadratic cumulative function, solved in
// closed form within the interval), and normal velocity components of
// variance e T(x) / m. Every workgroup builds the cumulative masses of the
// intervals in LDS in one fixed order.
__global__ __launch_bounds__(256) void k_load_profile(LoadArgs a) {
  extern __shared__ double sC[];  // sC[k]: mass of the intervals below point k
  const int np = a.npts;
  if (threadIdx.x == 0) {
    double c = 0.0;
    sC[0] = 0.0;
    for (int k = 0; k + 1 < np; ++k) {
      c = c + (fmax(a.dens[k], 0.0) + fmax(a.dens[k + 1], 0.0)) * a.hh;
      sC[k + 1] = c;
    }
  }
  __syncthreads();
  const double total = sC[np - 1];
  const double h = a.h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint4 r0 = philox(make_uint4(kLoadStep, (uint32_t)i, 16u * a.species, 0u), a.seed, a.run);
    const double r = u01(r0.x) * total;
    // the last interval whose cumulative mass starts at or below r
    int lo = 0, hi = np - 2;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sC[mid] <= r) lo = mid;
      else hi = mid - 1;
    }
    const double rp = r - sC[lo];
    const double da = fmax(a.dens[lo], 0.0), db = fmax(a.dens[lo + 1], 0.0);
    const double den = da + sqrt(fmax(da * da + 2.0 * (db - da) * rp / h, 0.0));
    double t = den > 0.0 ? 2.0 * rp / den : 0.0;
    t = fmin(fmax(t, 0.0), h);
    const double x = fmin((double)lo * h + t, a.L);
    const double ta = a.temp[lo], tb = a.temp[lo + 1];
    const double T = fmax(ta + (tb - ta) * (t / h), 0.0);
    const double sig = sqrt(T * a.vfac);
    const uint4 r1 = philox(make_uint4(kLoadStep, (uint32_t)i, 16u * a.species + 1u, 0u), a.seed,
                            a.run);
    double n1, n2, n3, n4;
    box_muller(u01(r1.x), u01(r1.y), n1, n2);
    box_muller(u01(r1.z), u01(r1.w), n3, n4);
    a.x[i] = x;
    a.vx[i] = sig * n1;
    a.vy[i] = sig * n2;
    a.vz[i] = sig * n3;
  }
}

hipError_t launch_load_profile(const LoadArgs& a, hipStream_t s) {
  if (a.npts < 2 || a.npts > kMaxLoadPoints) return hipErrorInvalidValue;
  int64_t g = (a.n + 255) / 256;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_load_profile, dim3((unsigned)g), dim3(256), (size_t)a.npts * 8, s, a);
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
