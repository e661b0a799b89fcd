// Field step as a device function run by one workgroup: charge density from
// the integer CIC deposits, the Poisson solve with Dirichlet walls
// phi(0) = V(t), phi(L) = 0, and E by numerical differentiation
// (arXiv:2109.04469, Sec. 2 steps 1-2). The grid (<= 4097 nodes) lives in
// LDS. Used by k_field and by the particle pass's tail kernel, which solves
// the next step's field while other workgroups finish this step.
//
// Default solver (FIELD_EXACT). With s_j = -dx^2 rho_j / eps0 = -K C_j, where
// C_j is the net deposit in 2^-32 units (an exact int64), the finite
// difference system phi_{j-1} - 2 phi_j + phi_{j+1} = s_j has the closed
// solution
//     D_j = phi_{j+1} - phi_j = D_0 - K Q_j,      Q_j = sum_{k=1..j} C_k
//     phi_j = V + j D_0 - K R_j,                  R_j = sum_{i<j} Q_i
//     D_0 = (K R_{N-1} - V) / (N - 1)             (from phi_{N-1} = 0)
// so the solve is two integer prefix sums (exact, order-free, parallel)
// followed by a few roundings per node, instead of a serial recurrence.
// FIELD_THOMAS runs the textbook Thomas recurrence serially instead, with the
// same operation order as the reference implementation (bitwise equal).
#pragma once

#include "pic_internal.h"

namespace pic {

constexpr int kFieldThreads = 1024;
constexpr int kFieldWaves = kFieldThreads / kWave;
constexpr int kMaxNx = 4097;
constexpr int kFieldPer = (kMaxNx + kFieldThreads - 1) / kFieldThreads;  // 5

struct i128p {
  uint64_t lo;
  int64_t hi;
};

__device__ __forceinline__ i128p add128(i128p a, i128p b) {
  i128p r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

__device__ __forceinline__ i128p from64(int64_t v) {
  i128p r;
  r.lo = (uint64_t)v;
  r.hi = v < 0 ? -1 : 0;
  return r;
}

// nearest-ish double of a 128-bit integer: sign-magnitude, two roundings
__device__ __forceinline__ double to_double(i128p v) {
  bool neg = v.hi < 0;
  if (neg) {  // two's complement negate
    v.lo = ~v.lo + 1;
    v.hi = ~v.hi + (v.lo == 0 ? 1 : 0);
  }
  const double r = (double)(uint64_t)v.hi * 18446744073709551616.0 + (double)v.lo;
  return neg ? -r : r;
}

// One step of a wave scan with data-parallel lane moves on each 32-bit word
// of a multi-word integer: the moved value (0 where a lane has no source)
// added with carries. CTRL, ROW_MASK, BOUND as in wave_incl_scan_dpp.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp_word(uint32_t w) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, CTRL, ROW_MASK, 0xF, BOUND);
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ void scan_step64(uint64_t& v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint64_t u = (uint64_t)dpp_word<CTRL, ROW_MASK, BOUND>(lo) |
                     ((uint64_t)dpp_word<CTRL, ROW_MASK, BOUND>(hi) << 32);
  v += u;
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ void scan_step128(i128p& v) {
  const uint64_t lo = v.lo, hi = (uint64_t)v.hi;
  i128p u;
  u.lo = (uint64_t)dpp_word<CTRL, ROW_MASK, BOUND>((uint32_t)lo) |
         ((uint64_t)dpp_word<CTRL, ROW_MASK, BOUND>((uint32_t)(lo >> 32)) << 32);
  u.hi = (int64_t)((uint64_t)dpp_word<CTRL, ROW_MASK, BOUND>((uint32_t)hi) |
                   ((uint64_t)dpp_word<CTRL, ROW_MASK, BOUND>((uint32_t)(hi >> 32)) << 32));
  v = add128(v, u);
}

// Wave-level inclusive scans of 64- and 128-bit integers with lane moves:
// the same steps as wave_incl_scan_dpp (shifts by 1, 2, 4, 8 inside each
// row of 16, then the row broadcasts), two's complement sums with carries.
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x) {
  uint64_t v = (uint64_t)x;
  scan_step64<0x111, 0xF, true>(v);
  scan_step64<0x112, 0xF, true>(v);
  scan_step64<0x114, 0xF, true>(v);
  scan_step64<0x118, 0xF, true>(v);
  scan_step64<0x142, 0xA, false>(v);
  scan_step64<0x143, 0xC, false>(v);
  return (int64_t)v;
}

__device__ __forceinline__ i128p wave_incl_scan128(i128p v) {
  scan_step128<0x111, 0xF, true>(v);
  scan_step128<0x112, 0xF, true>(v);
  scan_step128<0x114, 0xF, true>(v);
  scan_step128<0x118, 0xF, true>(v);
  scan_step128<0x142, 0xA, false>(v);
  scan_step128<0x143, 0xC, false>(v);
  return v;
}

// Block-wide exclusive scan of one int64 per thread; returns the total. The
// wave totals stay in s_wave: a caller that reuses it synchronises first.
__device__ __forceinline__ int64_t block_excl_scan64(int64_t v, int64_t& excl, int64_t* s_wave) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t inc = wave_incl_scan64(v);
  if (lane == kWave - 1) s_wave[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    // exclusive scan of the wave totals by the first wave
    const int64_t t = lane < kFieldWaves ? s_wave[lane] : 0;
    const int64_t ti = wave_incl_scan64(t);
    if (lane < kFieldWaves) s_wave[lane] = ti - t;
    if (lane == kFieldWaves - 1) s_wave[kFieldWaves] = ti;
  }
  __syncthreads();
  excl = s_wave[wave] + inc - v;
  return s_wave[kFieldWaves];
}

__device__ __forceinline__ i128p block_excl_scan128(i128p v, i128p& excl, i128p* s_wave) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const i128p inc = wave_incl_scan128(v);
  if (lane == kWave - 1) s_wave[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    // exclusive scan of the wave totals by the first wave
    const i128p t = lane < kFieldWaves ? s_wave[lane] : from64(0);
    const i128p ti = wave_incl_scan128(t);
    i128p neg_t;
    neg_t.lo = ~t.lo + 1;
    neg_t.hi = ~t.hi + (neg_t.lo == 0 ? 1 : 0);
    if (lane < kFieldWaves) s_wave[lane] = add128(ti, neg_t);
    if (lane == kFieldWaves - 1) s_wave[kFieldWaves] = ti;
  }
  __syncthreads();
  // excl = s_wave[wave] + inc - v
  i128p neg_v;
  neg_v.lo = ~v.lo + 1;
  neg_v.hi = ~v.hi + (neg_v.lo == 0 ? 1 : 0);
  excl = add128(add128(s_wave[wave], inc), neg_v);
  return s_wave[kFieldWaves];
}

// The whole field step, run by one workgroup of kFieldThreads threads.
// Thread t takes the nodes [t per, (t + 1) per) (the last thread also any
// node past them), per = ceil((N - 1) / threads): their deposits, rho, and
// in the exact solve their scan elements, potentials and fields, so that
// the exact solve needs no exchange through LDS beyond the two scans.
__device__ __forceinline__ void field_block(const FieldArgs& a) {
  __shared__ double sRho[kMaxNx];
  __shared__ double sPhi[kMaxNx];
  __shared__ int64_t s_wave64[kFieldWaves + 1];
  __shared__ i128p s_wave128[kFieldWaves + 1];

  const int tid = threadIdx.x;
  const int nx = a.nx;
  const int m = nx - 1;  // scan elements 0..N-2
  if (tid == 0) {
    // stores and non-returning atomics: the first wave does not wait on a
    // read of the control block
    a.ctl->ncodes[1] = 0;
    count_add(a.ctl, C_STEPS, 1ull);
    if (a.measuring) atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctl->msteps), 1ull);
  }
  constexpr int kOwn = kFieldPer + 1;
  const int per = (m + kFieldThreads - 1) / kFieldThreads;
  const int j0 = tid * per;
  const int j1 = tid == kFieldThreads - 1 ? nx : min(j0 + per, nx);
  // every deposit load of this thread in flight before the first use
  int64_t c[kOwn];
  double rho[kOwn];
  {
    int64_t de[kOwn], di[kOwn];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
      const int j = j0 + q;
      de[q] = j < j1 ? a.dep_e[j] : 0;
      di[q] = j < j1 ? a.dep_i[j] : 0;
    }
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
      const int j = j0 + q;
      c[q] = di[q] - de[q];
      rho[q] = 0.0;
      if (j >= j1) continue;
      if (a.zero_a) a.zero_a[j] = 0;
      if (a.zero_b) a.zero_b[j] = 0;
      double r = (double)c[q] * a.qfac32;
      const bool wall = (j == 0) || (j == nx - 1);
      if (wall) r = 2.0 * r;  // half-cell volume at the electrodes
      rho[q] = r;
      sRho[j] = r;
      a.rho[j] = r;
      if (a.measuring) {
        double ne = (double)de[q] * a.nfac32;
        double ni = (double)di[q] * a.nfac32;
        if (wall) {
          ne = 2.0 * ne;
          ni = 2.0 * ni;
        }
        a.acc_ne[j] += ne;
        a.acc_ni[j] += ni;
        a.acc_w[j] += (double)de[q] * kInvTwo32;
      }
    }
  }

  if (a.mode == FIELD_ZERO || a.mode == FIELD_FIXED) {
    for (int j = j0; j < j1; ++j) {
      a.phi[j] = 0.0;
      if (a.mode == FIELD_ZERO) a.E[j] = 0.0;
    }
    return;
  }

  const double dx = a.dx;
  const double V = a.V;
  if (a.mode == FIELD_THOMAS) {
    __syncthreads();  // sRho complete
    // d_i = -(dx dx) rho_{i+1} / eps0 for the unknowns phi_1..phi_{N-2}
    const int n = nx - 2;
    for (int i = tid; i < n; i += kFieldThreads) sPhi[i + 1] = -(dx * dx) * sRho[i + 1] / kEps0;
    __syncthreads();
    if (tid == 0) {
      // forward elimination: dp_i = (d_i - dp_{i-1}) / m_i, stored in place
      double prev = (sPhi[1] - V) / -2.0;
      if (n == 1) prev = ((sPhi[1] - V) - 0.0) / -2.0;
      sPhi[1] = prev;
      for (int i = 1; i < n; ++i) {
        double d = sPhi[i + 1];
        if (i == n - 1) d = d - 0.0;
        prev = (d - prev) / a.th_m[i];
        sPhi[i + 1] = prev;
      }
      // back substitution: y_i = dp_i - cp_i y_{i+1}
      double y = prev;
      for (int i = n - 2; i >= 0; --i) {
        y = sPhi[i + 1] - a.th_cp[i] * y;
        sPhi[i + 1] = y;
      }
      sPhi[0] = V;
      sPhi[nx - 1] = 0.0;
    }
    __syncthreads();
    for (int j = tid; j < nx; j += kFieldThreads) {
      double e;
      if (j == 0)
        e = (sPhi[0] - sPhi[1]) / dx - sRho[0] * dx / (2.0 * kEps0);
      else if (j == nx - 1)
        e = (sPhi[nx - 2] - sPhi[nx - 1]) / dx + sRho[nx - 1] * dx / (2.0 * kEps0);
      else
        e = (sPhi[j - 1] - sPhi[j + 1]) / (2.0 * dx);
      a.phi[j] = sPhi[j];
      a.E[j] = e;
      if (!isfinite(e)) latch_error(a.ctl, kErrUnstable);
    }
    return;
  }

  // ---- exact integer prefix form ----------------------------------------
  // c_0 = 0, c_k = C_k (k = 1..N-2); Q = inclusive scan of c over N-1
  // entries, R its exclusive scan. This thread's elements: its nodes below
  // N-1.
  int64_t loc[kOwn];  // local inclusive sums
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < kOwn; ++q) {
    const int k = j0 + q;
    if (k < j1 && k < m && k >= 1) s += c[q];
    loc[q] = s;
  }
  int64_t qb;  // Q before this thread's elements
  block_excl_scan64(s, qb, s_wave64);
  // R contributions: the sum of this thread's Q values
  i128p rsum = from64(0);
#pragma unroll
  for (int q = 0; q < kOwn; ++q)
    if (j0 + q < j1 && j0 + q < m) rsum = add128(rsum, from64(qb + loc[q]));
  i128p rb;  // R before this thread's elements
  const i128p rtot = block_excl_scan128(rsum, rb, s_wave128);
  // every thread has R_{N-1}: D0, then the potential phi_j = V + j D0 - K R_j
  // and the field from D_j = D0 - K Q_j at its own nodes (Q_{j-1} of its
  // first node is qb)
  const double D0 = (a.kpois * to_double(rtot) - V) / (double)(nx - 1);
  const double K = a.kpois;
  i128p r = rb;
  int64_t qprev = qb;
#pragma unroll
  for (int q = 0; q < kOwn; ++q) {
    const int j = j0 + q;
    if (j >= j1) continue;
    const int64_t qj = qb + loc[q];  // Q_j (j < N-1)
    if (j < m) {
      a.phi[j] = V + (double)j * D0 - K * to_double(r);
      r = add128(r, from64(qj));
    } else {
      a.phi[j] = 0.0;
    }
    double e;
    if (j == 0) {
      e = -D0 / dx - rho[q] * dx / (2.0 * kEps0);
    } else if (j == nx - 1) {
      const double Dlast = D0 - K * (double)qprev;
      e = -Dlast / dx + rho[q] * dx / (2.0 * kEps0);
    } else {
      e = (K * (double)(qprev + qj) - 2.0 * D0) / (2.0 * dx);
    }
    a.E[j] = e;
    if (!isfinite(e)) latch_error(a.ctl, kErrUnstable);
    qprev = qj;
  }
}


}  // namespace pic
