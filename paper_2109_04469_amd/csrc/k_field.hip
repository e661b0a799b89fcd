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
