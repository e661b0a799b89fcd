// Periodic cell sort: a stable counting sort of one species by cell index
// j = clamp(floor(x / dx), 0, N_x - 2), which keeps the particles of a tile in
// a few neighbouring cells so the particle kernel's deposit flush and its
// field gathers stay local. Stable, so the result is a pure function of the
// input order. Three kernels:
//   count   per-chunk key histograms (LDS), written key-major
//   scan    exclusive scan over (key, chunk) -> output offsets (three
//           parallel kernels)
//   scatter each chunk walks its particles in order; lanes with equal keys
//           are ranked with wave ballots and the waves of a workgroup take
//           their offsets in turn, which preserves the input order.
#include "pic_internal.h"

namespace pic {

constexpr int kSortThreads = 256;

__device__ __forceinline__ void chunk_range(int64_t n, int nblocks, int b, int64_t& lo,
                                            int64_t& hi) {
  const int64_t chunk = (n + nblocks - 1) / nblocks;
  lo = (int64_t)b * chunk;
  hi = lo + chunk;
  if (hi > n) hi = n;
  if (lo > n) lo = n;
}

// Chunk b of a's input: per-key counts, written key-major.
__device__ __forceinline__ void sort_count_block(const SortArgs& a, int b, uint32_t* sh) {
  const int nkeys = a.nx - 1;
  for (int k = threadIdx.x; k < nkeys; k += kSortThreads) sh[k] = 0u;
  __syncthreads();
  int64_t lo, hi;
  chunk_range(min(*a.count, a.cap), a.nblocks, b, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kSortThreads)
    atomicAdd(&sh[cell_key(a.sx[i], a.inv_dx, a.nx)], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < nkeys; k += kSortThreads)
    a.cnt[(size_t)k * a.nblocks + b] = sh[k];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_count(SortArgs a) {
  extern __shared__ uint32_t sh[];
  sort_count_block(a, blockIdx.x, sh);
}

// Exclusive scan of the nkeys * nblocks counters in place, in three
// parallel kernels: per-segment sums, a scan of the segment sums, and the
// per-segment rescan with its base.
constexpr int kScanSegs = 256;

__device__ __forceinline__ void seg_range(int64_t total, int seg, int64_t& lo, int64_t& hi) {
  const int64_t len = (total + kScanSegs - 1) / kScanSegs;
  lo = (int64_t)seg * len;
  hi = lo + len;
  if (hi > total) hi = total;
  if (lo > total) lo = total;
}

__device__ __forceinline__ void scan_reduce_seg(const SortArgs& a, int seg, uint32_t* s_w) {
  const int64_t total = (int64_t)(a.nx - 1) * a.nblocks;
  int64_t lo, hi;
  seg_range(total, seg, lo, hi);
  uint32_t sum = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kSortThreads) sum += a.cnt[i];
  sum = wave_sum<unsigned int>(sum);
  if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kSortThreads / kWave; ++w) t += s_w[w];
    a.seg[seg] = t;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_scan_reduce(SortArgs a) {
  __shared__ uint32_t s_w[kSortThreads / kWave];
  scan_reduce_seg(a, blockIdx.x, s_w);
}

__device__ __forceinline__ void scan_top_all(const SortArgs& a, uint32_t* s_w) {
  const uint32_t v = a.seg[threadIdx.x];
  const uint32_t inc = wave_incl_scan<unsigned int>(v);
  if ((threadIdx.x & (kWave - 1)) == kWave - 1) s_w[threadIdx.x / kWave] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) base += s_w[w];
  a.seg[threadIdx.x] = base + inc - v;
}

__global__ __launch_bounds__(kScanSegs) void k_scan_top(SortArgs a) {
  __shared__ uint32_t s_w[kScanSegs / kWave];
  scan_top_all(a, s_w);
}

__device__ __forceinline__ void scan_down_seg(const SortArgs& a, int seg, uint32_t* s_w) {
  const int64_t total = (int64_t)(a.nx - 1) * a.nblocks;
  int64_t lo, hi;
  seg_range(total, seg, lo, hi);
  lo = uniform64(lo);
  hi = uniform64(hi);
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t run = a.seg[seg];
  for (int64_t b0 = lo; b0 < hi; b0 += kSortThreads) {
    const int64_t i = b0 + threadIdx.x;
    const uint32_t v = i < hi ? a.cnt[i] : 0u;
    const uint32_t inc = wave_incl_scan<unsigned int>(v);
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < kSortThreads / kWave; ++w) {
      if (w < wave) wbase += s_w[w];
      tot += s_w[w];
    }
    if (i < hi) a.cnt[i] = run + wbase + inc - v;
    run += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortThreads) void k_scan_down(SortArgs a) {
  __shared__ uint32_t s_w[kSortThreads / kWave];
  scan_down_seg(a, blockIdx.x, s_w);
}

__device__ __forceinline__ void sort_scatter_block(const SortArgs& a, int b, uint32_t* off,
                                                   uint32_t (*s_base)[kWave]) {
  const int nkeys = a.nx - 1;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  for (int k = threadIdx.x; k < nkeys; k += kSortThreads)
    off[k] = a.cnt[(size_t)k * a.nblocks + b];
  __syncthreads();
  int64_t lo, hi;
  const int64_t n = min(uniform64(*a.count), a.cap);
  // the rebuilt pool holds exactly the n sorted slots
  if (b == 0 && threadIdx.x == 0) *a.pool_n = n;
  chunk_range(n, a.nblocks, b, lo, hi);
  lo = uniform64(lo);
  hi = uniform64(hi);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int64_t b0 = lo; b0 < hi; b0 += kSortThreads) {
    const int64_t i = b0 + threadIdx.x;
    const bool valid = i < hi;
    double x = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
    int key = 0;
    if (valid) {
      x = a.sx[i];
      vx = a.svx[i];
      const uint32_t id = a.sid[i];
      vy = a.spvy[id];
      vz = a.spvz[id];
      key = cell_key(x, a.inv_dx, a.nx);
    }
    // lanes of this wave holding the same key
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 13; ++bit) {
      const bool on = (key >> bit) & 1;
      const uint64_t bm = __ballot(valid && on);
      mask &= on ? bm : ~bm;
    }
    const int rank = __popcll(mask & lt);
    const int leader = __ffsll((long long)mask) - 1;
    for (int w = 0; w < kSortThreads / kWave; ++w) {
      if (wave == w && valid && lane == leader) {
        const uint32_t bse = off[key];
        off[key] = bse + (uint32_t)__popcll(mask);
        s_base[w][lane] = bse;
      }
      __syncthreads();
    }
    if (valid) {
      // the sorted slot's pool entry is the slot itself
      const uint32_t dest = s_base[wave][leader] + (uint32_t)rank;
      a.dx[dest] = x;
      a.dvx[dest] = vx;
      a.did[dest] = dest;
      a.dpvy[dest] = vy;
      a.dpvz[dest] = vz;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortArgs a) {
  extern __shared__ uint32_t off[];
  __shared__ uint32_t s_base[kSortThreads / kWave][kWave];
  sort_scatter_block(a, blockIdx.x, off, s_base);
}

// ---------------------------------------------------------------------------
// Batched sorts: n independent jobs (one species of one discharge each, with
// their own counters) in one launch per kernel. Count and scatter lay the
// jobs' chunk blocks end to end; the scan kernels take kScanSegs blocks
// (or one) per job.

// The job of this workgroup among jobs whose block counts are nb(j), and
// the workgroup's block within it.
__device__ __forceinline__ void job_block(const SortArgs* __restrict__ args, int n, int& job,
                                          int& b) {
  __shared__ int64_t s_bs[kMaxBatch + 1];
  __shared__ int64_t s_w[kSortThreads / kWave];
  block_exclusive<kSortThreads>(threadIdx.x < (unsigned)n ? args[threadIdx.x].nblocks : 0, n, s_bs,
                                s_w);
  const int64_t g = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_bs[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  job = uniform32(lo);
  b = uniform32((int)(g - s_bs[lo]));
}

__global__ __launch_bounds__(kSortThreads) void k_sort_count_b(const SortArgs* __restrict__ args,
                                                                int n) {
  extern __shared__ uint32_t sh[];
  int job, b;
  job_block(args, n, job, b);
  sort_count_block(args[job], b, sh);
}

__global__ __launch_bounds__(kSortThreads) void k_scan_reduce_b(const SortArgs* __restrict__ args) {
  __shared__ uint32_t s_w[kSortThreads / kWave];
  const int job = blockIdx.x / kScanSegs;
  scan_reduce_seg(args[job], blockIdx.x % kScanSegs, s_w);
}

__global__ __launch_bounds__(kScanSegs) void k_scan_top_b(const SortArgs* __restrict__ args) {
  __shared__ uint32_t s_w[kScanSegs / kWave];
  scan_top_all(args[blockIdx.x], s_w);
}

__global__ __launch_bounds__(kSortThreads) void k_scan_down_b(const SortArgs* __restrict__ args) {
  __shared__ uint32_t s_w[kSortThreads / kWave];
  const int job = blockIdx.x / kScanSegs;
  scan_down_seg(args[job], blockIdx.x % kScanSegs, s_w);
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter_b(const SortArgs* __restrict__ args,
                                                                  int n) {
  extern __shared__ uint32_t off[];
  __shared__ uint32_t s_base[kSortThreads / kWave][kWave];
  int job, b;
  job_block(args, n, job, b);
  sort_scatter_block(args[job], b, off, s_base);
}

hipError_t launch_batch_sort(const SortArgs* args, int n, int64_t total_blocks, int nx_max,
                             hipStream_t s) {
  if (n < 1 || n > kMaxBatch || total_blocks < 1 || nx_max < 3) return hipErrorInvalidValue;
  const size_t lds = (size_t)(nx_max - 1) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_sort_count_b, dim3((unsigned)total_blocks), dim3(kSortThreads), lds, s, args,
                     n);
  hipLaunchKernelGGL(k_scan_reduce_b, dim3(n * kScanSegs), dim3(kSortThreads), 0, s, args);
  hipLaunchKernelGGL(k_scan_top_b, dim3(n), dim3(kScanSegs), 0, s, args);
  hipLaunchKernelGGL(k_scan_down_b, dim3(n * kScanSegs), dim3(kSortThreads), 0, s, args);
  hipLaunchKernelGGL(k_sort_scatter_b, dim3((unsigned)total_blocks), dim3(kSortThreads), lds, s,
                     args, n);
  return hipGetLastError();
}

// The pool in slot order without moving the slots: entry i of the new pool
// is slot i's (v_y, v_z), and slot i's index becomes i.
__global__ __launch_bounds__(kSortThreads) void k_repack(SortArgs a) {
  const int64_t n = min(*a.count, a.cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.pool_n = n;
  for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kSortThreads) {
    const uint32_t id = a.sid[i];
    a.dpvy[i] = a.spvy[id];
    a.dpvz[i] = a.spvz[id];
    a.did[i] = (uint32_t)i;
  }
}

hipError_t launch_repack(const SortArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_repack, dim3(1024), dim3(kSortThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sort(const SortArgs& a, hipStream_t s) {
  const size_t lds = (size_t)(a.nx - 1) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_sort_count, dim3(a.nblocks), dim3(kSortThreads), lds, s, a);
  hipLaunchKernelGGL(k_scan_reduce, dim3(kScanSegs), dim3(kSortThreads), 0, s, a);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanSegs), 0, s, a);
  hipLaunchKernelGGL(k_scan_down, dim3(kScanSegs), dim3(kSortThreads), 0, s, a);
  hipLaunchKernelGGL(k_sort_scatter, dim3(a.nblocks), dim3(kSortThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace pic
