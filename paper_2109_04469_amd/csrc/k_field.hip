// Field kernel: the field step of arXiv:2109.04469, Sec. 2 steps 1-2, in one
// workgroup (field_block.h).
#include "field_block.h"
#include "pic_internal.h"

namespace pic {

__global__ __launch_bounds__(kFieldThreads) void k_field(FieldArgs a) { field_block(a); }

hipError_t launch_field(const FieldArgs& a, hipStream_t s) {
  if (a.nx > kMaxNx || a.nx < 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_field, dim3(1), dim3(kFieldThreads), 0, s, a);
  return hipGetLastError();
}

// Workgroups 1.. of k_field_cand: bit i of word i / 32 is the collision
// candidacy of electron slot i of the step f.cand_step (Philox word i mod 4 of
// the block (step, i / 4, 4, 0) below the threshold), for the slots the
// deciding pass outputs: the sum of its tile totals' output counts.
__device__ void candidacy_bits(const FieldArgs& f, int wg, int nwg) {
  __shared__ unsigned long long s_w[kFieldThreads / kWave];
  const int tid = threadIdx.x;
  // tiles of the deciding pass (its slot count), four loads per thread in
  // flight at a time
  int64_t np = *f.cand_count;
  if (np > f.cand_cap) np = f.cand_cap;
  const int64_t ntiles = (np + kTile - 1) / kTile;
  unsigned long long own = 0;
  for (int64_t t0 = tid; t0 < ntiles; t0 += 4 * kFieldThreads) {
    uint64_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t t = t0 + (int64_t)k * kFieldThreads;
      v[k] = t < ntiles ? f.cand_tcnt[t] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) own += v[k] & 0xFFFFull;
  }
  own = wave_sum<unsigned long long>(own);
  if ((tid & (kWave - 1)) == 0) s_w[tid / kWave] = own;
  __syncthreads();
  int64_t n = 0;
  for (int w = 0; w < kFieldThreads / kWave; ++w) n += (int64_t)s_w[w];
  if (n > f.cand_cap) n = f.cand_cap;
  const int64_t words = (n + 31) / 32;
  for (int64_t wi = (int64_t)wg * kFieldThreads + tid; wi < words;
       wi += (int64_t)nwg * kFieldThreads) {
    uint32_t bits = 0;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const uint4 r = draw(f.cand_step, (uint32_t)(wi * 8 + g), 0, 4, f.seed, f.run);
      bits |= ((uint64_t)r.x < f.cand_thr ? 1u : 0u) << (4 * g);
      bits |= ((uint64_t)r.y < f.cand_thr ? 1u : 0u) << (4 * g + 1);
      bits |= ((uint64_t)r.z < f.cand_thr ? 1u : 0u) << (4 * g + 2);
      bits |= ((uint64_t)r.w < f.cand_thr ? 1u : 0u) << (4 * g + 3);
    }
    f.cand[wi] = bits;
  }
}

// Also, for the fused electron pass that follows: its tile totals buffer
// zeroed, and the first pool entries of its births (the pools' fill levels
// before it), which its workgroups read while its last tile advances them.
__global__ __launch_bounds__(kFieldThreads) void k_field_cand(FieldArgs a) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      a.ctl->pbase[0] = a.ctl->pool_n[0];
      a.ctl->pbase[1] = a.ctl->pool_n[1];
    }
    field_block(a);
  } else {
    for (int64_t i = (int64_t)(blockIdx.x - 1) * kFieldThreads + threadIdx.x; i < a.cand_zero_n;
         i += (int64_t)(gridDim.x - 1) * kFieldThreads)
      a.cand_zero[i] = 0ull;
    candidacy_bits(a, (int)blockIdx.x - 1, (int)gridDim.x - 1);
  }
}

hipError_t launch_field_cand(const FieldArgs& a, int num_cu, hipStream_t s) {
  if (a.nx > kMaxNx || a.nx < 3 || !a.cand || !a.cand_tcnt || !a.cand_zero || num_cu < 1)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_field_cand, dim3(1 + num_cu), dim3(kFieldThreads), 0, s, a);
  return hipGetLastError();
}

// the fields of n discharges, one workgroup each
__global__ __launch_bounds__(kFieldThreads) void k_field_b(const FieldArgs* __restrict__ f) {
  field_block(f[blockIdx.x]);
}

hipError_t launch_batch_field(const FieldArgs* f, int n, hipStream_t s) {
  if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_field_b, dim3(n), dim3(kFieldThreads), 0, s, f);
  return hipGetLastError();
}

}  // namespace pic
