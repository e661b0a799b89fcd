// Device-side definitions shared by the libpic kernels (gfx950, wave64).
//
// Arithmetic conventions (they make every decision of a step bitwise
// reproducible on any execution order): FP64 IEEE round-to-nearest with no
// contraction (-ffp-contract=off), correctly rounded division and sqrt, CIC
// weights in 2^-32 fixed point with integer accumulation, and all random
// draws from Philox4x32-10 keyed by (seed, run) with counter
// (step, slot, 16*species + purpose, 0), except the collision-candidacy
// uniform of slot i: word i mod 4 of the block (step, i / 4, 16*species + 4,
// 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kBlock = 256;          // threads per particle workgroup (4 waves)
#ifndef PIC_PPT
#define PIC_PPT 8
#endif
constexpr int kPPT = PIC_PPT;        // particles per thread per tile
constexpr int kTile = kBlock * kPPT;  // particles per tile
static_assert(kPPT % 4 == 0, "k_decide takes runs of four slots");
constexpr int kWave = 64;

constexpr double kTwoPi = 6.283185307179586;
constexpr double kTwo32 = 4294967296.0;
constexpr double kInvTwo32 = 2.3283064365386963e-10;
constexpr int64_t kOne32 = 4294967296LL;

// latched device error bits
constexpr uint32_t kErrUnstable = 1u;
constexpr uint32_t kErrCapacity = 2u;

// decision code bits (per pushed slot)
constexpr uint8_t kCodePushed = 0x80;

enum Counter {
  C_STEPS = 0, C_E_PUSHED, C_I_PUSHED, C_E_ABSORBED, C_E_REFLECTED, C_I_ABSORBED,
  C_SE_EMITTED, C_E_CAND, C_E_ELASTIC, C_E_EXC, C_E_ION, C_I_CAND, C_I_ISO, C_I_BACK,
  C_REFLECT_LOST, C_BEYOND_TABLE, NCOUNTERS
};

// Copies of the event counters: a workgroup adds into copy blockIdx mod
// kCounterSlots, so that the end-of-workgroup flushes of a large grid do not
// all queue on one address; readers sum the copies.
constexpr int kCounterSlots = 64;

// Control block in device memory. Counts are double-buffered by step parity:
// step n reads n_*[n & 1] and produces n_*[(n + 1) & 1].
struct DevCtl {
  int64_t n_e[2];
  int64_t n_i[2];
  int64_t e_out;      // outputs of this step's electron kernel
  int64_t i_births;   // ions appended by this step's electron kernel
  int64_t ncodes[2];  // slots with a decision code from the last step
  int64_t msteps;     // measured steps
  int64_t n_rare[2];  // slots queued for the rare pass of the last step
  int64_t pool_n[2];  // velocity-pool entries in use (live + orphaned + new)
  int64_t pbase[2];   // first pool entry of the last pass's births, per pool
  alignas(128) unsigned long long counters[kCounterSlots][NCOUNTERS];  // one 128-byte line each
  // electrode diagnostics while measuring, [species][wall] (wall 0: x = 0)
  unsigned long long wall_hits[2][2];      // arrivals (reflected electrons included)
  unsigned long long wall_absorbed[2][2];  // of which absorbed
  double wall_esum[2][2];                  // sum of impact energies, eV
  unsigned long long ioniz_meas;           // ionizations
  uint32_t err;
  uint32_t pad;
};

// Adds v to event counter i in this workgroup's copy.
__device__ __forceinline__ void count_add(DevCtl* c, int i, unsigned long long v) {
  atomicAdd(&c->counters[blockIdx.x % kCounterSlots][i], v);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
  }
  return c;
}

__device__ __forceinline__ uint4 draw(uint32_t step, uint32_t slot, uint32_t species,
                                      uint32_t purpose, uint32_t seed, uint32_t run) {
  return philox(make_uint4(step, slot, 16u * species + purpose, 0u), seed, run);
}

// u32 -> (r + 1/2) 2^-32, exact in FP64, strictly inside (0, 1)
__device__ __forceinline__ double u01(uint32_t r) { return ((double)r + 0.5) * kInvTwo32; }

__device__ __forceinline__ void box_muller(double u1, double u2, double& a, double& b) {
  const double rad = sqrt(-2.0 * log(u1));
  const double th = kTwoPi * u2;
  double s, c;
  sincos(th, &s, &c);
  a = rad * c;
  b = rad * s;
}

__device__ __forceinline__ void iso_dir(double ua, double ub, double& nx, double& ny,
                                        double& nz) {
  const double cth = 1.0 - 2.0 * ua;
  const double sth = 2.0 * sqrt(ua * (1.0 - ua));
  const double ph = kTwoPi * ub;
  double s, c;
  sincos(ph, &s, &c);
  nx = cth;
  ny = sth * c;
  nz = sth * s;
}

// Cell index j in [0, nx-2], fraction f and fixed-point weight w1 of node
// j+1 (node j receives 2^32 - w1).
__device__ __forceinline__ void cell_of(double x, double inv_dx, int nx, int& j, double& f,
                                        int64_t& w1) {
  const double t = x * inv_dx;
  int jj = (int)t;
  if (jj > nx - 2) jj = nx - 2;
  if (jj < 0) jj = 0;
  j = jj;
  f = t - (double)jj;
  // round to nearest 2^-32 and clamp to [0, 2^32] in FP64, then convert
  // through uint32 (one instruction) with 2^32 itself handled apart
  const double wf = fmin(fmax(floor(f * kTwo32 + 0.5), 0.0), kTwo32);
  w1 = wf >= kTwo32 ? kOne32 : (int64_t)(uint32_t)wf;
}

__device__ __forceinline__ int cell_key(double x, double inv_dx, int nx) {
  const double t = x * inv_dx;
  int jj = (int)t;
  if (jj > nx - 2) jj = nx - 2;
  if (jj < 0) jj = 0;
  return jj;
}

// Wave-uniform copies of values every lane holds alike. Loop bounds and
// exits of loops that contain workgroup barriers must be visibly uniform to
// the compiler; otherwise it may restructure the loop so that lanes take
// different paths around the barrier.
__device__ __forceinline__ int uniform32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void latch_error(DevCtl* ctl, uint32_t bit) {
  atomicOr(&ctl->err, bit);
}

// wave-level inclusive scan (64 lanes)
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  return v;
}

// The same inclusive scan of 32-bit values with data-parallel lane moves
// (no LDS traffic): shifts by 1, 2, 4 and 8 lanes inside each row of 16, then
// the last lane of row 0 (and of row 2) added to row 1 (and row 3), then
// the last lane of row 1 added to rows 2 and 3. Lanes without a source add 0.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31, rows 2, 3
  return (uint32_t)x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}

// Exclusive prefix sums of v (one value per thread, threads at or beyond n
// hold none) into out[0..n], out[n] being the total. NT threads, n <= NT.
// Ends with a barrier.
template <int NT>
__device__ __forceinline__ void block_exclusive(int64_t v, int n, int64_t* out, int64_t* s_w) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  if (tid >= n) v = 0;
  const int64_t inc = wave_incl_scan<int64_t>(v);
  if (lane == kWave - 1) s_w[wave] = inc;
  __syncthreads();
  int64_t off = 0;
  for (int w = 0; w < wave; ++w) off += s_w[w];
  if (tid < n) out[tid] = off + inc - v;
  if (tid == NT - 1) out[n] = off + inc;
  __syncthreads();
}

}  // namespace pic
