// Particle pass of one species for one step: field gather, leap-frog push,
// the wall model and null-collision MCC, with order-preserving compaction,
// births and the CIC deposit of the new positions (arXiv:2109.04469, Sec. 2
// steps 3-6 and step 1 of the next step).
//
// Two kernels per species step, with no dependency between workgroups inside
// either of them:
//   k_decide  streams x and vx, pushes, applies the wall and draws the
//             collision candidacy (and for electrons the process, which fixes
//             the number of outputs). The candidacy uniform of slot i is word
//             i mod 4 of the block with counter (step, i / 4, 16 sp + 4, 0),
//             so one block serves four slots; the wall and process uniforms
//             come from the slot's own block (step, i, 16 sp, 0), drawn only
//             for the few slots that need them. It writes a one-byte decision code per
//             slot and the output, birth and queued-slot totals per tile of
//             kTile slots,
//             and deposits the new positions (and those of births) into LDS
//             fixed-point histograms flushed with integer atomics.
//   k_emit    takes a contiguous run of tiles per workgroup for electrons and
//             tiles blockIdx.x, blockIdx.x + gridDim.x, ... for ions (carrying
//             the prefix over the tiles in between), forms its prefix
//             from the per-tile totals, scans the codes inside each tile and
//             writes every output to its compacted slot: it re-reads the
//             particle and repeats the push bit for bit (same arithmetic, no
//             contraction). Slots that need draws (collision kinematics, an
//             ion process still to choose, a secondary electron) are queued
//             with their output slots instead.
//   k_rare    takes the queued slots, one per thread: a small fraction, kept
//             out of the streaming kernels because their transcendental-heavy
//             code would set those kernels' register budget.
// Survivors keep their relative order and an ionization electron follows its
// parent; births of the other species (Ar+ from ionization, secondary
// electrons from ion impact) are appended after that species' particles in
// parent-slot order.
//
// Pipelined electron steps (pic_set_pipeline) replace k_decide of step n+1:
//   k_emit_decide  is k_emit of step n that also decides step n+1 for each
//             output (the push with the next field staged in LDS, the
//             candidacy bit k_field_cand drew, and for the few outputs that
//             leave the gap or are candidates the wall and process decisions),
//             writing the next step's decision codes, tile totals and
//             deposit; each workgroup then runs its own queued slots of step n
//             and the decisions it deferred, one item per thread.
// The arithmetic of every decision is the same in all kernels, so pipelined
// and unpipelined steps give identical results.
#include <climits>

#include "field_block.h"
#include "pic_internal.h"

namespace pic {

// Copies a field of nx values into LDS, PER loads of each thread issued
// before its first store (one memory round trip per PER strides of the
// workgroup instead of one per stride).
template <int NT, int PER>
__device__ __forceinline__ void stage_field(double* sE, const double* E, int nx) {
  for (int j0 = (int)threadIdx.x; j0 < nx; j0 += PER * NT) {
    double v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = j0 + k * NT;
      v[k] = j < nx ? E[j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = j0 + k * NT;
      if (j < nx) sE[j] = v[k];
    }
  }
}
// Code bit used between the kernels of a pass only: an Ar+ collision
// candidate whose process (which needs a thermal atom velocity) is chosen by
// rare_slot in k_rare / k_tail, which replaces it with the process bits, so a
// code read by the caller has bit 6 clear.
constexpr uint32_t kIonPending = 0x40u;

struct Outcome {
  uint32_t own;    // output slots of this species: 0, 1 or 2
  uint32_t birth;  // births of the other species: 0 or 1
  bool rare;       // queued: needs draws in k_rare / k_tail
};

// What a decision code implies for the outputs. Slots carried without a
// push (bit 7 clear) give one output.
template <int SP>
__device__ __forceinline__ Outcome outcome(uint32_t c) {
  Outcome r{0u, 0u, false};
  if (!(c & kCodePushed)) {
    r.own = 1u;
    return r;
  }
  const uint32_t wall = c & 7u;
  const uint32_t proc = (c >> 3) & 7u;
  if (SP == 0) {
    const bool alive = wall == 0u || wall == 2u;
    const bool ion = alive && proc == 4u;
    r.own = alive ? (ion ? 2u : 1u) : 0u;
    r.birth = ion ? 1u : 0u;
    r.rare = alive && proc >= 2u;
  } else {
    const bool alive = wall == 0u;
    r.own = alive ? 1u : 0u;
    r.birth = wall == 3u ? 1u : 0u;
    r.rare = (alive && (c & kIonPending)) || wall == 3u;
  }
  return r;
}

// Gather (linear interpolation in the particle's cell) and leap-frog push.
// Both kernels call this on the same inputs and get the same bits.
__device__ __forceinline__ void push(const double* E, int j, double f, double acc, double dts,
                                     double& x, double& vx) {
  const double Ep = (1.0 - f) * E[j] + f * E[j + 1];
  vx = vx + acc * Ep;
  x = x + vx * dts;
}

__device__ __forceinline__ void deposit_lds(unsigned long long* sH, double x, double inv_dx, int nx,
                                            unsigned long long mul, int& jlo, int& jhi) {
  int j;
  double f;
  int64_t w1;
  cell_of(x, inv_dx, nx, j, f, w1);
  atomicAdd(&sH[j], mul * (unsigned long long)(kOne32 - w1));
  atomicAdd(&sH[j + 1], mul * (unsigned long long)w1);
  jlo = min(jlo, j);
  jhi = max(jhi, j + 1);
}

__device__ __forceinline__ void deposit_global(unsigned long long* dep, double x, double inv_dx,
                                               int nx) {
  int j;
  double f;
  int64_t w1;
  cell_of(x, inv_dx, nx, j, f, w1);
  atomicAdd(&dep[j], (unsigned long long)(kOne32 - w1));
  atomicAdd(&dep[j + 1], (unsigned long long)w1);
}

// Cumulative collision frequency of table `p` at table variable tv (speed /
// table step), linear in tv; beyond the last table speed, the last entry.
__device__ __forceinline__ double cum_nu(const double* cum, int ntab, int p, double tv) {
  const double* c = cum + (int64_t)p * ntab;
  if (tv < (double)(ntab - 1)) {
    const int kk = (int)tv;
    const double tt = tv - (double)kk;
    return (1.0 - tt) * c[kk] + tt * c[kk + 1];
  }
  return c[ntab - 1];
}

// ---------------------------------------------------------------------------
// k_decide

// k_decide's threads per workgroup: the default instance, and the other
// compiled size (pic_set_decide_block), which takes the same tiles with
// twice the runs of four slots per thread. The batched kernels use kDB.
constexpr int kDB = kDecideBlocks[0];
constexpr int kDBAlt = kDecideBlocks[1];

// The wall model and the collision decision of one pushed slot whose new
// position is not a finite point inside the gap, or that is a collision
// candidate: a small fraction of slots. x and vx are the pushed values and
// are updated (reflection); the code, the number of own outputs and of
// births are returned through c, o and b.
// A particle of species SP reaching electrode `wall` (0: x = 0) with the
// pushed velocity (vx and the pool's v_y, v_z): arrival count, absorption,
// impact energy and its bin of the flux-energy distribution (Sec. 3.3).
template <int SP>
__device__ __forceinline__ void record_arrival(const PartArgs& a, int64_t slot, double vx, int wall,
                                               bool absorbed) {
  const uint32_t id = a.idin[slot];
  const double vy = a.pvy[id], vz = a.pvz[id];
  const double eps = a.ek_s * (vx * vx + vy * vy + vz * vz);
  DevCtl* ctl = a.ctl;
  atomicAdd(&ctl->wall_hits[SP][wall], 1ull);
  if (absorbed) atomicAdd(&ctl->wall_absorbed[SP][wall], 1ull);
  atomicAdd(&ctl->wall_esum[SP][wall], eps);
  const int64_t bin = (int64_t)(eps * a.fedf_inv_de);
  if (bin >= 0 && bin < a.nbins) atomicAdd(&a.fedf[(int64_t)wall * a.nbins + bin], 1ull);
}

// pool index unknown to the caller: decide_rare reads it from a.idin
constexpr uint32_t kNoId = 0xFFFFFFFFu;

// EAGER: an electron candidate's three cumulative frequencies are read
// together, not each after the previous comparison (the same values; more
// registers, one memory round trip instead of up to three). vyz: the
// particle's v_y, v_z when the caller holds them (else read from the pool).
template <int SP, bool MEASURE, bool EAGER = false>
__device__ __forceinline__ void decide_rare(const PartArgs& a, unsigned long long* s_cnt,
                                            int64_t slot, bool cand, double& x, double& vx,
                                            uint32_t& c, uint32_t& o, uint32_t& b,
                                            uint32_t pid = kNoId, const double* vyz = nullptr) {
  const double L = a.L;
  const uint32_t step = a.step;
  bool alive = true;
  uint32_t mul = 1;
  if (!isfinite(x) || !isfinite(vx)) {
    latch_error(a.ctl, kErrUnstable);
    alive = false;
    c |= 1u;
  } else if (x < 0.0 || x > L) {
    const int wall = x < 0.0 ? 0 : 1;
    const double vx_hit = vx;
    const double ub = u01(draw(step, (uint32_t)slot, SP, 0, a.seed, a.run).x);
    if (SP == 0) {
      if (ub < a.p_wall) {
        x = (x < 0.0) ? -x : (L + L) - x;
        vx = -vx;
        if (x < 0.0 || x > L) {
          alive = false;
          c |= 4u;
          atomicAdd(&s_cnt[C_REFLECT_LOST], 1ull);
        } else {
          c |= 2u;
          atomicAdd(&s_cnt[C_E_REFLECTED], 1ull);
        }
      } else {
        alive = false;
        c |= 1u;
        atomicAdd(&s_cnt[C_E_ABSORBED], 1ull);
      }
    } else {
      alive = false;
      atomicAdd(&s_cnt[C_I_ABSORBED], 1ull);
      if (ub < a.p_wall) {
        // a secondary electron leaves the wall the ion hit
        c |= 3u;
        b = 1;
        atomicAdd(&s_cnt[C_SE_EMITTED], 1ull);
        deposit_global(a.dep_other, x < 0.0 ? 0.0 : L, a.inv_dx, a.nx);
      } else {
        c |= 1u;
      }
    }
    // electrons record arrivals only in the measuring variant (the same
    // condition: it runs exactly when measuring), ions by the runtime flag
    if (SP == 0 ? MEASURE : (a.measure_walls != 0)) record_arrival<SP>(a, slot, vx_hit, wall, !alive);
  }
  if (alive && cand) {
    if (SP == 0) {
      // electron candidate: the process at this speed decides whether a
      // second electron and an ion are born
      atomicAdd(&s_cnt[C_E_CAND], 1ull);
      double vy, vz;
      if (vyz) {
        vy = vyz[0];
        vz = vyz[1];
      } else {
        const uint32_t id = pid != kNoId ? pid : a.idin[slot];
        vy = a.pvy[id];
        vz = a.pvz[id];
      }
      const double g2 = sqrt(vx * vx + vy * vy + vz * vz);
      const double tv = g2 * a.inv_dv;
      const double r = u01(draw(step, (uint32_t)slot, SP, 0, a.seed, a.run).z) * a.numax;
      if (!(tv < (double)(a.ntab - 1))) atomicAdd(&s_cnt[C_BEYOND_TABLE], 1ull);
      uint32_t proc = 1;
      double n0 = 0.0, n1 = 0.0, n2 = 0.0;
      if (EAGER) {
        n0 = cum_nu(a.cum, a.ntab, 0, tv);
        n1 = cum_nu(a.cum, a.ntab, 1, tv);
        n2 = cum_nu(a.cum, a.ntab, 2, tv);
      }
      if (r < (EAGER ? n0 : cum_nu(a.cum, a.ntab, 0, tv))) {
        proc = 2;
        atomicAdd(&s_cnt[C_E_ELASTIC], 1ull);
      } else if (r < (EAGER ? n1 : cum_nu(a.cum, a.ntab, 1, tv))) {
        proc = 3;
        atomicAdd(&s_cnt[C_E_EXC], 1ull);
      } else if (r < (EAGER ? n2 : cum_nu(a.cum, a.ntab, 2, tv))) {
        proc = 4;
        b = 1;
        mul = 2;
        atomicAdd(&s_cnt[C_E_ION], 1ull);
        if (MEASURE) atomicAdd(&a.ctl->ioniz_meas, 1ull);
        deposit_global(a.dep_other, x, a.inv_dx, a.nx);
      }
      c |= proc << 3;
    } else {
      atomicAdd(&s_cnt[C_I_CAND], 1ull);
      c |= kIonPending;
    }
  }
  o = alive ? mul : 0u;
}

// The tiles t_begin, t_begin + t_step, ... below t_end of one particle pass
// of discharge a: push, wall and candidacy decisions, decision codes, tile
// totals and the deposit of the new positions. The waves do not wait for
// each other inside the loop: each adds its share of a tile's totals to
// a.tcnt (zeroed by the previous pass) with one atomic, and the deposits
// collect in LDS until one flush at the end. sH (and, measuring, sEW) are all
// zero on entry and on exit; sE holds a's field; s_lo > s_hi on entry and on
// exit, and the caller synchronises the workgroup before the next call.
template <int SP, bool MEASURE, int DB = kDB>
__device__ __forceinline__ void decide_tiles(const PartArgs& a, int t_begin, int t_end, int t_step,
                                             int64_t n_push, int64_t n_tot, const double* sE,
                                             unsigned long long* sH, double* sEW,
                                             unsigned int* sEEPF, int& s_lo, int& s_hi,
                                             unsigned long long* s_cnt) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int nx = a.nx;
  const uint32_t step = a.step;
  const double inv_dx = a.inv_dx;
  const double L = a.L;
  const bool no_coll = a.no_coll != 0;
  const uint64_t cand_thr = no_coll ? 0ull : a.pcoll_thr;
  // runs of four slots per thread per tile
  constexpr int kDGroups = kTile / (4 * DB);
  static_assert(kDGroups >= 1 && kTile % (4 * DB) == 0, "a tile is whole runs of four slots");

  int jlo = INT_MAX, jhi = -1;
  for (int t = t_begin; t < t_end; t += t_step) {
    const int64_t base = (int64_t)t * kTile;
    uint32_t own = 0, births = 0, rares = 0;
    // each thread takes runs of four consecutive slots: 16-byte loads, one
    // Philox block for the four candidacy draws, one 4-byte code store
#pragma unroll
    for (int g = 0; g < kDGroups; ++g) {
      const int64_t s0 = base + (int64_t)g * (4 * DB) + 4 * tid;
      if (s0 >= n_tot) continue;
      const bool full = s0 + 3 < n_tot;
      double xs[4], vxs[4];
      if (full) {
        const double2* xp = reinterpret_cast<const double2*>(a.xin + s0);
        const double2* vp = reinterpret_cast<const double2*>(a.vxin + s0);
        const double2 x01 = xp[0], x23 = xp[1], v01 = vp[0], v23 = vp[1];
        xs[0] = x01.x, xs[1] = x01.y, xs[2] = x23.x, xs[3] = x23.y;
        vxs[0] = v01.x, vxs[1] = v01.y, vxs[2] = v23.x, vxs[3] = v23.y;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          xs[q] = s0 + q < n_tot ? a.xin[s0 + q] : 0.0;
          vxs[q] = s0 + q < n_tot ? a.vxin[s0 + q] : 0.0;
        }
      }
      uint4 rc = make_uint4(0u, 0u, 0u, 0u);
      if (s0 < n_push) rc = draw(step, (uint32_t)(s0 >> 2), SP, 4, a.seed, a.run);
      const uint32_t ucs[4] = {rc.x, rc.y, rc.z, rc.w};

      // push all four, then the few slots that left the gap or are
      // candidates
      uint32_t c[4], o[4], b[4];
      bool need[4], cand[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t slot = s0 + q;
        const bool in = slot < n_tot;
        const bool pushed = slot < n_push;
        c[q] = pushed ? (uint32_t)kCodePushed : 0u;
        o[q] = in ? 1u : 0u;
        b[q] = 0u;
        cand[q] = false;
        need[q] = false;
        if (pushed) {
          int j;
          double f;
          int64_t w1;
          cell_of(xs[q], inv_dx, nx, j, f, w1);
          if (MEASURE) {
            const uint32_t id = a.idin[slot];
            const double vy = a.pvy[id], vz = a.pvz[id];
            const double vx0 = vxs[q];
            const double eps = a.ek * (vx0 * vx0 + vy * vy + vz * vz);
            atomicAdd(&sEW[j], ((double)(kOne32 - w1) * kInvTwo32) * eps);
            atomicAdd(&sEW[j + 1], ((double)w1 * kInvTwo32) * eps);
            jlo = min(jlo, j);
            jhi = max(jhi, j + 1);
            if (fabs(xs[q] - a.half) <= a.eepf_hw) {
              const int64_t bin = (int64_t)(eps * a.inv_de);
              if (bin >= 0 && bin < a.nbins) atomicAdd(&sEEPF[bin], 1u);
            }
          }
          push(sE, j, f, a.acc, a.dts, xs[q], vxs[q]);
          // u01(r) < pcoll, decided exactly on the integer word
          cand[q] = (uint64_t)ucs[q] < cand_thr;
          need[q] = cand[q] || !(xs[q] >= 0.0 && xs[q] <= L) || !isfinite(vxs[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (need[q])
          decide_rare<SP, MEASURE>(a, s_cnt, s0 + q, cand[q], xs[q], vxs[q], c[q], o[q], b[q]);

      // deposit of the new positions (an ionization electron is born at its
      // parent's position), combined when the four share a cell
      int jq[4];
      unsigned long long h0[4], h1[4];
      int jr = -1;
      bool same = true;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double f;
        int64_t w1;
        cell_of(xs[q], inv_dx, nx, jq[q], f, w1);
        h0[q] = (unsigned long long)o[q] * (unsigned long long)(kOne32 - w1);
        h1[q] = (unsigned long long)o[q] * (unsigned long long)w1;
        if (o[q]) {
          if (jr < 0) jr = jq[q];
          same = same && jq[q] == jr;
          jlo = min(jlo, jq[q]);
          jhi = max(jhi, jq[q] + 1);
        }
      }
      if (jr >= 0) {
        if (same) {
          atomicAdd(&sH[jr], h0[0] + h0[1] + h0[2] + h0[3]);
          atomicAdd(&sH[jr + 1], h1[0] + h1[1] + h1[2] + h1[3]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (o[q]) {
              atomicAdd(&sH[jq[q]], h0[q]);
              atomicAdd(&sH[jq[q] + 1], h1[q]);
            }
        }
      }
      const uint32_t codes4 = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
      if (full) {
        *reinterpret_cast<uint32_t*>(a.codes + s0) = codes4;
      } else {
        for (int q = 0; q < 4 && s0 + q < n_tot; ++q) a.codes[s0 + q] = (uint8_t)c[q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        own += o[q];
        births += b[q];
        rares += (s0 + q < n_tot && outcome<SP>(c[q]).rare) ? 1u : 0u;
      }
    }

    // this wave's share of the tile totals, summed in one 32-bit word (per
    // wave at most 2 * 4 * kDGroups * 64 outputs and half as many births or
    // queued slots: 11, 11 and 10 bits) with lane moves, then widened to the
    // totals' layout
    static_assert(kDGroups <= 2, "wave totals fit the 11/11/10-bit fields");
    const uint32_t packed = own | (births << 11) | (rares << 22);
    const uint32_t ws =
        (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(packed), kWave - 1);
    const unsigned long long tot = (unsigned long long)(ws & 0x7FFu) |
                                   ((unsigned long long)((ws >> 11) & 0x7FFu) << 16) |
                                   ((unsigned long long)(ws >> 22) << 32);
    if (lane == 0 && tot) atomicAdd(&a.tcnt[t], tot);
  }

  // one flush of the deposit range touched by this workgroup's tiles
  jlo = wave_min(jlo);
  jhi = wave_max(jhi);
  if (lane == 0) {
    atomicMin(&s_lo, jlo);
    atomicMax(&s_hi, jhi);
  }
  __syncthreads();
  const int lo = s_lo, hi = s_hi;  // lo > hi when nothing was deposited
  for (int j = (lo <= hi ? lo : hi + 1) + tid; j <= hi; j += DB) {
    const unsigned long long v = sH[j];
    if (v) {
      atomicAdd(&a.dep_own[j], v);
      sH[j] = 0ull;
    }
    if (MEASURE) {
      const double e = sEW[j];
      if (e != 0.0) {
        atomicAdd(&a.acc_ew[j], e);
        sEW[j] = 0.0;
      }
    }
  }
  __syncthreads();  // s_lo and s_hi have been read
  if (tid == 0) {
    s_lo = INT_MAX;
    s_hi = -1;
  }
}

// Zeroes this workgroup's share of the tile totals buffer of the next pass
// of discharge a (the previous pass of this species read it).
template <int DB>
__device__ __forceinline__ void clear_next_totals(const PartArgs& a) {
  for (int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x; i < a.max_tiles;
       i += (int64_t)gridDim.x * DB)
    a.tcnt_next[i] = 0ull;
}

template <int SP, bool MEASURE, int DB = kDB>
__global__ __launch_bounds__(DB) void k_decide(PartArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx;
  double* sE = reinterpret_cast<double*>(smem);
  unsigned long long* sH = reinterpret_cast<unsigned long long*>(sE + nx);
  double* sEW = reinterpret_cast<double*>(sH + nx);                 // MEASURE
  unsigned int* sEEPF = reinterpret_cast<unsigned int*>(sEW + nx);  // MEASURE

  __shared__ int s_lo, s_hi;
  __shared__ unsigned long long s_cnt[NCOUNTERS];

  const int tid = threadIdx.x;
  DevCtl* ctl = a.ctl;
  const int par = a.parity;

  clear_next_totals<DB>(a);

  stage_field<DB, (kMaxNx + DB - 1) / DB>(sE, a.E, nx);
  for (int j = tid; j < nx; j += DB) {
    sH[j] = 0ull;
    if (MEASURE) sEW[j] = 0.0;
  }
  if (MEASURE)
    for (int b = tid; b < a.nbins; b += DB) sEEPF[b] = 0u;
  if (tid < NCOUNTERS) s_cnt[tid] = 0ull;
  if (tid == 0) {
    s_lo = INT_MAX;
    s_hi = -1;
  }

  // slots [0, n_push) are pushed; [n_push, n_tot) were born earlier in this
  // step (ions from this step's electron pass) and are carried unchanged
  int64_t n_push = uniform64(SP == 0 ? ctl->n_e[par] : ctl->n_i[par]);
  int64_t n_tot = SP == 0 ? n_push : n_push + uniform64(ctl->i_births);
  if (n_tot > a.cap) {
    if (tid == 0 && blockIdx.x == 0) latch_error(ctl, kErrCapacity);
    n_tot = a.cap;
    if (n_push > n_tot) n_push = n_tot;
  }
  const int ntiles = uniform32((int)((n_tot + kTile - 1) / kTile));

  if (blockIdx.x == 0 && tid == 0) {
    if (a.record) ctl->ncodes[SP] = n_push;
    count_add(ctl, SP == 0 ? C_E_PUSHED : C_I_PUSHED, (unsigned long long)n_push);
  }
  __syncthreads();

  decide_tiles<SP, MEASURE, DB>(a, blockIdx.x, ntiles, gridDim.x, n_push, n_tot, sE, sH,
                                sEW, sEEPF, s_lo, s_hi, s_cnt);

  if (tid < NCOUNTERS && s_cnt[tid]) count_add(ctl, tid, s_cnt[tid]);
  if (MEASURE) {
    for (int b = tid; b < a.nbins; b += DB)
      if (sEEPF[b]) atomicAdd(&a.eepf[b], (unsigned long long)sEEPF[b]);
  }
}

// ---------------------------------------------------------------------------
// k_emit

__device__ __forceinline__ void store3(const PartArgs& a, int64_t i, double x, double vx,
                                       uint32_t id) {
  a.xout[i] = x;
  a.vxout[i] = vx;
  a.idout[i] = id;
}

// k_decide's push and reflection, repeated on the slot's input state.
__device__ __forceinline__ void repush(const PartArgs& a, const double* E, uint32_t c, double& x,
                                       double& vx) {
  if (c & kCodePushed) {
    int j;
    double f;
    int64_t w1;
    cell_of(x, a.inv_dx, a.nx, j, f, w1);
    push(E, j, f, a.acc, a.dts, x, vx);
    if ((c & 7u) == 2u) {
      x = (x < 0.0) ? -x : (a.L + a.L) - x;
      vx = -vx;
    }
  }
}

__device__ __forceinline__ void reload(const PartArgs& a, const double* E, int64_t slot,
                                       uint32_t c, double& x, double& vx, uint32_t& id,
                                       double& vy, double& vz) {
  x = a.xin[slot];
  vx = a.vxin[slot];
  id = a.idin[slot];
  vy = a.pvy[id];
  vz = a.pvz[id];
  repush(a, E, c, x, vx);
}

// Tile totals word of one slot's outcome: outputs | births << 16 |
// queued << 32.
__device__ __forceinline__ unsigned long long totals_word(uint32_t c, uint32_t o, uint32_t bb) {
  return (unsigned long long)o | ((unsigned long long)bb << 16) |
         ((unsigned long long)(outcome<0>(c).rare ? 1u : 0u) << 32);
}

// tile totals each thread reads at once per step of a strided run
constexpr int kStrideLoads = 8;

// pairs of consecutive slots per lane and tile in k_emit
constexpr int kEPairs = kPPT / 2;
// candidacy bit words covering the outputs of one tile (at most 2 kTile)
constexpr int kCandWords = 2 * kTile / 32 + 1;
static_assert(kPPT % 2 == 0, "k_emit takes pairs of slots");

// Counts of a particle pass with no slots.
template <int SP>
__device__ __forceinline__ void emit_empty(DevCtl* ctl, int par) {
  ctl->n_rare[SP] = 0;
  ctl->pbase[0] = ctl->pool_n[0];
  ctl->pbase[1] = ctl->pool_n[1];
  if (SP == 0) {
    ctl->e_out = 0;
    ctl->n_e[par ^ 1] = 0;
    ctl->i_births = 0;
    ctl->n_i[par ^ 1] = ctl->n_i[par];
  } else {
    ctl->n_i[par ^ 1] = 0;
    ctl->n_e[par ^ 1] = ctl->e_out;
  }
}

// The tiles t0, t0 + t_step, ... below t1 of a particle pass of discharge a
// (ntiles tiles, n_tot slots): compacted outputs, queued rare slots and, at
// the last tile, the pass's counts. With t_step > 1 the totals of the tiles
// between two of this workgroup's tiles are summed while the first of them is
// loaded, so the prefix reaches the next one without another pass. sE holds a's field. The per-wave totals of
// outputs and births (s_wtot) and of queued slots (s_wr) have two copies
// used by alternate tiles, and every wave scans a tile's totals itself, so
// a tile needs one workgroup barrier; queued slots take their places in
// slot order from the same scans.
//
// MODE 0: the input holds the state before the push, which is repeated
// here (sE: a's field). MODE 1: the input holds the pushed state (the
// previous step's fused emit stored it), written out as it is. MODE 2
// (electrons): as MODE 1, and each output that needs no queued work is then
// pushed for the next step b with b's field in sE; an output that stays in
// the gap and is no collision candidate (its bit in b.cand) is decided there:
// the output slot receives the pushed state of that step, its decision code
// goes to b.codes, its deposit to the LDS histogram sH (flushed by the caller
// over [jlo, jhi]), its outcome to the next pass's tile totals b.tcnt. The
// other outputs are listed in b.dq from this workgroup's first output slot
// on (their count in s_dcnt), and rq_range returns the workgroup's queued
// slots [rq_range[0], rq_range[1]) and first output slot rq_range[2], for
// the caller to finish. MODE 3: as MODE 2 on an input that holds the state
// before the push, which is repeated first with a's field (in sE0).
template <int SP, int STAGE_PER, int MODE = 0>
__device__ __forceinline__ void emit_tiles(const PartArgs& a, int t0, int t1, int t_step,
                                           int ntiles, int64_t n_tot, int64_t bbase, double* sE,
                                           uint32_t (*s_wtot)[kEPairs][kBlock / kWave],
                                           uint32_t (*s_wr)[kEPairs][kBlock / kWave],
                                           uint32_t (*s_ps)[3][kBlock / kWave],
                                           uint64_t (*s_red)[kBlock / kWave],
                                           const PartArgs* b = nullptr,
                                           unsigned long long* sH = nullptr,
                                           unsigned long long* s_cnt = nullptr,
                                           int* jlo_out = nullptr, int* jhi_out = nullptr,
                                           uint32_t (*s_cand)[kCandWords] = nullptr,
                                           uint32_t* s_dcnt = nullptr, double* sE0 = nullptr,
                                           int64_t* rq_range = nullptr) {
  constexpr bool FUSE = MODE >= 2;
  static_assert(!FUSE || SP == 0, "only electron passes decide the next step");
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  DevCtl* ctl = a.ctl;
  const int par = a.parity;
  // outputs, births and queued slots of all earlier tiles (eight loads per
  // thread in flight at a time), and a's field staged into sE while the
  // first of those loads are in flight
  unsigned long long po = 0, pb = 0, pr = 0;
  bool staged = false;
  for (int tb = 0; tb < t0; tb += 8 * kBlock) {
    uint64_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tb + u * kBlock + tid;
      v[u] = t < t0 ? a.tcnt[t] : 0ull;
    }
    if (!staged) {
      if (MODE != 1) stage_field<kBlock, STAGE_PER>(sE, FUSE ? b->E : a.E, a.nx);
      if (MODE == 3) stage_field<kBlock, STAGE_PER>(sE0, a.E, a.nx);
      staged = true;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      po += v[u] & 0xFFFFull;
      pb += (v[u] >> 16) & 0xFFFFull;
      pr += v[u] >> 32;
    }
  }
  if (!staged && MODE != 1) stage_field<kBlock, STAGE_PER>(sE, FUSE ? b->E : a.E, a.nx);
  if (!staged && MODE == 3) stage_field<kBlock, STAGE_PER>(sE0, a.E, a.nx);
  po = wave_sum<unsigned long long>(po);
  pb = wave_sum<unsigned long long>(pb);
  pr = wave_sum<unsigned long long>(pr);
  if (lane == 0) {
    s_red[0][wave] = po;
    s_red[1][wave] = pb;
    s_red[2][wave] = pr;
  }
  __syncthreads();
  int64_t prefO = 0, prefB = 0, prefR = 0;
  for (int w = 0; w < kBlock / kWave; ++w) {
    prefO += (int64_t)s_red[0][w];
    prefB += (int64_t)s_red[1][w];
    prefR += (int64_t)s_red[2][w];
  }

  // MODE 2: this lane's deposit run (cell jr, weights of nodes jr, jr + 1);
  // the workgroup's first output slot (its deferred list starts there: the
  // workgroup defers at most its own outputs) and first queued slot
  const int64_t wg_out0 = prefO;
  const int64_t wg_rq0 = prefR;
  int jr = -1, jlo = INT_MAX, jhi = -1;
  unsigned long long h0 = 0ull, h1 = 0ull;
  for (int t = t0; t < t1; t += t_step) {
    const int p = ((t - t0) / t_step) & 1;
    const int64_t base = (int64_t)t * kTile;
    // strided runs: the totals of tiles t .. t + t_step - 1 carry the prefix
    // to this workgroup's next tile (loads issued with the tile's own)
    uint32_t nso = 0, nsb = 0, nsr = 0;
    if (t_step > 1 && t + t_step < t1) {
      const int ue = min(t + t_step, ntiles);
      for (int c0 = t; c0 < ue; c0 += kStrideLoads * kBlock) {  // once for grids <= 2048
#pragma unroll
        for (int k = 0; k < kStrideLoads; ++k) {
          const int u = c0 + k * kBlock + tid;
          const uint64_t v = u < ue ? a.tcnt[u] : 0ull;
          nso += (uint32_t)(v & 0xFFFFull);
          nsb += (uint32_t)((v >> 16) & 0xFFFFull);
          nsr += (uint32_t)(v >> 32);
        }
      }
    }
    // the fused pass: the next step's candidacy bits of this tile's outputs
    // (at most 2 kTile slots from the tile's first output), one word per
    // thread, requested with the tile's loads and put into LDS before the
    // tile's barrier
    static_assert(kCandWords <= kBlock, "one candidacy word per thread");
    uint32_t cw_tile = 0u;
    if (FUSE) {
      const int64_t w0 = prefO >> 5;
      const int64_t nwords = (a.cap + 31) / 32 + 1;
      if (tid < kCandWords && w0 + tid < nwords) cw_tile = b->cand[w0 + tid];
    }
    // pairs of consecutive slots per lane: 16-byte loads of x and v_x, an
    // 8-byte load of the two pool indices, one 2-byte load of the codes.
    // The plain emit counts and scans each pair row after its own loads
    // (issuing every row's loads first measured slower there); the fused
    // pass, latency-bound at three workgroups per CU, requests the codes of
    // all rows of a whole tile first and then every row's x, v_x and
    // indices, so the tile waits for one round trip before its counts
    // instead of one per row.
    uint32_t code[kPPT], loc[kEPairs], rloc[kEPairs];
    double px[kPPT], pvx[kPPT];
    uint32_t pid[kPPT];
    // a whole tile (all but the last of a pass): no slot tests, so that the
    // loads are issued back to back
    const bool whole = FUSE && base + kTile <= n_tot;
    if (whole) {
#pragma unroll
      for (int k = 0; k < kEPairs; ++k) {
        const int64_t s0 = base + k * (2 * kBlock) + 2 * tid;
        // the two slots' codes (bytes 0, 1) and presence flags (bits 16, 17)
        code[2 * k] = (uint32_t)*reinterpret_cast<const uint16_t*>(a.codes + s0) | 0x30000u;
      }
#pragma unroll
      for (int k = 0; k < kEPairs; ++k) {
        const int64_t s0 = base + k * (2 * kBlock) + 2 * tid;
        const double2 xx = *reinterpret_cast<const double2*>(a.xin + s0);
        const double2 vv = *reinterpret_cast<const double2*>(a.vxin + s0);
        const uint2 ii = *reinterpret_cast<const uint2*>(a.idin + s0);
        px[2 * k] = xx.x;
        px[2 * k + 1] = xx.y;
        pvx[2 * k] = vv.x;
        pvx[2 * k + 1] = vv.y;
        pid[2 * k] = ii.x;
        pid[2 * k + 1] = ii.y;
      }
#pragma unroll
      for (int k = 0; k < kEPairs; ++k) {
        // each slot's code with its presence flag in bit 8
        const uint32_t c2 = code[2 * k];
        code[2 * k] = (c2 & 0xFFu) | ((c2 >> 8) & 0x100u);
        code[2 * k + 1] = ((c2 >> 8) & 0xFFu) | ((c2 >> 9) & 0x100u);
      }
    }
#pragma unroll
    for (int k = 0; k < kEPairs; ++k) {
      const int64_t s0 = base + k * (2 * kBlock) + 2 * tid;
      uint32_t cnt = 0, rcnt = 0;
      if (!whole) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        code[2 * k + h] = 0;
        px[2 * k + h] = pvx[2 * k + h] = 0.0;
        pid[2 * k + h] = 0u;
      }
      if (s0 + 1 < n_tot) {
        const uint32_t c2 = *reinterpret_cast<const uint16_t*>(a.codes + s0);
        const double2 xx = *reinterpret_cast<const double2*>(a.xin + s0);
        const double2 vv = *reinterpret_cast<const double2*>(a.vxin + s0);
        const uint2 ii = *reinterpret_cast<const uint2*>(a.idin + s0);
        code[2 * k] = (c2 & 0xFFu) | 0x100u;
        code[2 * k + 1] = (c2 >> 8) | 0x100u;
        px[2 * k] = xx.x;
        px[2 * k + 1] = xx.y;
        pvx[2 * k] = vv.x;
        pvx[2 * k + 1] = vv.y;
        pid[2 * k] = ii.x;
        pid[2 * k + 1] = ii.y;
      } else if (s0 < n_tot) {
        code[2 * k] = (uint32_t)a.codes[s0] | 0x100u;
        px[2 * k] = a.xin[s0];
        pvx[2 * k] = a.vxin[s0];
        pid[2 * k] = a.idin[s0];
      }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t c = code[2 * k + h];
        if (c & 0x100u) {
          const Outcome oc = outcome<SP>(c);
          cnt += oc.own | (oc.birth << 16);
          rcnt += oc.rare ? 1u : 0u;
        }
      }
      const uint32_t inc = wave_incl_scan_dpp(cnt);
      const uint32_t rinc = wave_incl_scan_dpp(rcnt);
      loc[k] = inc - cnt;
      rloc[k] = rinc - rcnt;
      if (lane == kWave - 1) {
        s_wtot[p][k][wave] = inc;
        s_wr[p][k][wave] = rinc;
      }
    }
    if (t_step > 1 && t + t_step < t1) {
      const uint32_t wo = wave_incl_scan_dpp(nso), wb = wave_incl_scan_dpp(nsb),
                     wr = wave_incl_scan_dpp(nsr);
      if (lane == kWave - 1) {
        s_ps[p][0][wave] = wo;
        s_ps[p][1][wave] = wb;
        s_ps[p][2][wave] = wr;
      }
    }
    if (FUSE && tid < kCandWords) s_cand[p][tid] = cw_tile;
    __syncthreads();
    // every wave scans the tile's segment totals (segment k * nw + w) itself,
    // so no second barrier is needed; the other copy of the totals belongs
    // to the next tile
    constexpr int nw = kBlock / kWave;
    constexpr int nseg = kEPairs * nw;
    const uint32_t sv = lane < nseg ? (&s_wtot[p][0][0])[lane] : 0u;
    const uint32_t sr = lane < nseg ? (&s_wr[p][0][0])[lane] : 0u;
    const uint32_t si = wave_incl_scan_dpp(sv);
    const uint32_t sri = wave_incl_scan_dpp(sr);
    const uint32_t tile_ob = (uint32_t)__builtin_amdgcn_readlane((int)si, nseg - 1);
    const uint32_t tile_r = (uint32_t)__builtin_amdgcn_readlane((int)sri, nseg - 1);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // MODE 2: outcomes of the next step per output tile, relative to the
    // tile of this tile's first output (its outputs span at most 2 kTile
    // slots, so three tiles)
    const int64_t tA = prefO / kTile;
    uint32_t nt[3] = {0u, 0u, 0u};


#pragma unroll
    for (int k = 0; k < kEPairs; ++k) {
      uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)(si - sv), k * nw + wv) + loc[k];
      uint32_t roff = (uint32_t)__builtin_amdgcn_readlane((int)(sri - sr), k * nw + wv) + rloc[k];
      uint32_t dq_slot[2] = {0xFFFFFFFFu, 0xFFFFFFFFu};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = 2 * k + h;
        const uint32_t c = code[q];
        const bool in = (c & 0x100u) != 0;
        const Outcome oc = outcome<SP>(c);
        const bool rare = in && oc.rare;
        const int64_t slot = base + k * (2 * kBlock) + 2 * tid + h;
        if (rare) {
          // queue the slot for the rare work with its output slots
          a.rq[prefR + roff] = make_uint4((uint32_t)slot, c & 0xFFu,
                                          (uint32_t)(prefO + (off & 0xFFFFu)),
                                          (uint32_t)(prefB + (off >> 16)));
          ++roff;
        }
        if (in && !rare && oc.own) {
          const int64_t dest = prefO + (int64_t)(off & 0xFFFFu);
          double x = px[q], vx = pvx[q];
          if (MODE == 0) repush(a, sE, c, x, vx);
          if (MODE == 3) repush(a, sE0, c, x, vx);
          bool defer = false;
          if (FUSE && dest < a.cap) {
            // the next step's push; a slot that leaves the gap or is a
            // collision candidate is decided after this workgroup's tiles
            int jd;
            double fd;
            int64_t w1;
            cell_of(x, b->inv_dx, b->nx, jd, fd, w1);
            push(sE, jd, fd, b->acc, b->dts, x, vx);
            const uint32_t cw = s_cand[p][(int)((dest >> 5) - (prefO >> 5))];
            defer = ((cw >> (dest & 31)) & 1u) != 0 || !(x >= 0.0 && x <= b->L) || !isfinite(vx);
            if (!defer) {
              b->codes[dest] = (uint8_t)kCodePushed;
              const uint32_t rel = (uint32_t)(dest / kTile - tA);
              nt[0] += rel == 0u ? 1u : 0u;
              nt[1] += rel == 1u ? 1u : 0u;
              nt[2] += rel == 2u ? 1u : 0u;
              cell_of(x, b->inv_dx, b->nx, jd, fd, w1);
              if (jd != jr) {
                if (jr >= 0) {
                  atomicAdd(&sH[jr], h0);
                  atomicAdd(&sH[jr + 1], h1);
                }
                jr = jd;
                h0 = h1 = 0ull;
                jlo = min(jlo, jd);
                jhi = max(jhi, jd + 1);
              }
              h0 += (unsigned long long)(kOne32 - w1);
              h1 += (unsigned long long)w1;
            }
          }
          if (dest < a.cap) store3(a, dest, x, vx, pid[q]);
          if (FUSE) dq_slot[h] = defer ? (uint32_t)dest : 0xFFFFFFFFu;
        }
        if (in) off += oc.own | (oc.birth << 16);
      }
      if (FUSE) {
        // this row's deferred slots appended to the workgroup's list (an
        // LDS counter, one atomic per wave, only for rows that have any)
        const uint32_t nd = (dq_slot[0] != 0xFFFFFFFFu ? 1u : 0u) + (dq_slot[1] != 0xFFFFFFFFu ? 1u : 0u);
        if (__ballot(nd != 0u)) {
          const uint32_t inc = wave_incl_scan_dpp(nd);
          const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
          uint32_t base = 0u;
          if (lane == 0) base = atomicAdd(s_dcnt, tot);
          base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
          int64_t idx = wg_out0 + (int64_t)(base + inc - nd);
          if (dq_slot[0] != 0xFFFFFFFFu) b->dq[idx++] = dq_slot[0];
          if (dq_slot[1] != 0xFFFFFFFFu) b->dq[idx] = dq_slot[1];
        }
      }
    }
    if (FUSE) {
      // this wave's share of the next pass's tile totals (per wave at most
      // 2 * kPPT * 64 outputs, kPPT * 64 births and queued slots: 11, 11
      // and 10 bits), widened to the totals' layout
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const uint32_t ws = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(nt[r]), kWave - 1);
        if (lane == 0 && ws) {
          const unsigned long long tot = (unsigned long long)(ws & 0x7FFu) |
                                         ((unsigned long long)((ws >> 11) & 0x7FFu) << 16) |
                                         ((unsigned long long)(ws >> 22) << 32);
          atomicAdd(&b->tcnt[tA + r], tot);
        }
      }
    }
    if (t_step > 1 && t + t_step < t1) {
      // the next tile of this workgroup is t + t_step
      int64_t ao = 0, ab = 0, ar = 0;
#pragma unroll
      for (int w = 0; w < kBlock / kWave; ++w) {
        ao += s_ps[p][0][w];
        ab += s_ps[p][1][w];
        ar += s_ps[p][2][w];
      }
      prefO += ao;
      prefB += ab;
      prefR += ar;
      continue;
    }
    prefO += tile_ob & 0xFFFFu;
    prefB += tile_ob >> 16;
    prefR += tile_r;
    if (t == ntiles - 1 && tid == 0) {
      ctl->n_rare[SP] = prefR;
      if (SP == 0) {
        ctl->e_out = prefO;
        ctl->n_e[par ^ 1] = prefO;
        ctl->i_births = prefB;
        ctl->n_i[par ^ 1] = bbase + prefB;
      } else {
        ctl->n_i[par ^ 1] = prefO;
        ctl->n_e[par ^ 1] = bbase + prefB;
      }
      if (prefO > a.cap || bbase + prefB > a.bcap) latch_error(ctl, kErrCapacity);
      // pool entries of this pass's births: an ionization takes one in each
      // pool (the new electron and the new ion), an emission one electron
      // entry; k_rare fills them from these bases
      const int other = 1 - SP;
      if (!FUSE) {
        // (a fused pass reads them while this runs: the field kernel before
        // it has set them)
        ctl->pbase[SP] = ctl->pool_n[SP];
        ctl->pbase[other] = ctl->pool_n[other];
      }
      if (SP == 0) ctl->pool_n[SP] += prefB;
      ctl->pool_n[other] += prefB;
      if (ctl->pool_n[SP] > a.pcap || ctl->pool_n[other] > a.bpcap) latch_error(ctl, kErrCapacity);
      if (FUSE) {
        // the next step pushes every output of this one
        const int64_t np = prefO < a.cap ? prefO : a.cap;
        if (b->record) ctl->ncodes[SP] = np;
        count_add(ctl, C_E_PUSHED, (unsigned long long)np);
      }
    }
  }
  if (FUSE) {
    if (jr >= 0) {
      atomicAdd(&sH[jr], h0);
      atomicAdd(&sH[jr + 1], h1);
    }
    *jlo_out = jlo;
    *jhi_out = jhi;
  }
  __syncthreads();  // the field and the totals may be reused by the caller
  if (FUSE && rq_range) {
    rq_range[0] = wg_rq0;
    rq_range[1] = prefR;
    rq_range[2] = wg_out0;
  }
}

template <int SP, int MODE>
__global__ __launch_bounds__(kBlock) void k_emit(PartArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* sE = reinterpret_cast<double*>(smem);
  __shared__ uint32_t s_wtot[2][kEPairs][kBlock / kWave];
  __shared__ uint32_t s_wr[2][kEPairs][kBlock / kWave];
  __shared__ uint32_t s_ps[2][3][kBlock / kWave];
  __shared__ uint64_t s_red[3][kBlock / kWave];

  const int tid = threadIdx.x;
  DevCtl* ctl = a.ctl;
  const int par = a.parity;
  // MODE 1 follows a fused pass that decided this step; the decide pass that
  // would have zeroed the next pass's totals buffer did not run
  if (MODE == 1)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < a.max_tiles;
         i += (int64_t)gridDim.x * kBlock)
      a.tcnt_next[i] = 0ull;

  int64_t n_push = uniform64(SP == 0 ? ctl->n_e[par] : ctl->n_i[par]);
  int64_t n_tot = SP == 0 ? n_push : n_push + uniform64(ctl->i_births);
  if (n_tot > a.cap) n_tot = a.cap;  // k_decide has latched the error
  const int64_t bbase = uniform64(SP == 0 ? ctl->n_i[par] : ctl->e_out);
  const int ntiles = uniform32((int)((n_tot + kTile - 1) / kTile));

  if (ntiles == 0) {
    if (blockIdx.x == 0 && tid == 0) emit_empty<SP>(ctl, par);
    return;
  }
  // this workgroup's tiles. Electrons: a contiguous run (measured faster for
  // them). Ions, whose arrays were last touched several steps ago: tiles
  // blockIdx.x, blockIdx.x + gridDim.x, ..., which keeps all workgroups
  // inside one moving window of the arrays (measured 12 % faster for them).
  int t0, t1, t_step;
  if (SP == 0) {
    // the longer runs on the workgroups dispatched first on each CU (as in
    // k_emit_decide)
    const int g = (int)gridDim.x, b_ = (int)blockIdx.x;
    const int q = ntiles / g, r = ntiles % g;
    t0 = b_ < r ? b_ * (q + 1) : r * (q + 1) + (b_ - r) * q;
    t1 = t0 + (b_ < r ? q + 1 : q);
    t_step = 1;
  } else {
    t0 = blockIdx.x;
    t1 = ntiles;
    t_step = gridDim.x;
  }
  if (t0 >= t1) return;

  emit_tiles<SP, (kMaxNx + kBlock - 1) / kBlock, MODE>(a, t0, t1, t_step, ntiles, n_tot, bbase,
                                                        sE, s_wtot, s_wr, s_ps, s_red);
}

// ---------------------------------------------------------------------------
// k_rare: the queued slots, one per thread

// Collision kinematics, the ion process choice and secondary emission for
// one slot, and its outputs at dest (own species) and, for a birth of rank r
// in this pass, at slot bbase + r of the other species with pool entries
// pbase + r. E is read from global memory here (the same values k_decide
// used).
// Direction after a deflection by chi from the incident unit vector e, with
// cos chi = (2 + eps - 2 (1 + eps)^u) / eps (eps in eV; uniform cos chi when
// eps = 0) and azimuth 2 pi w, about e: n = cos chi e + sin chi (cos phi b1 +
// sin phi b2), b1 the unit vector along e x (1, 0, 0) (e x (0, 1, 0) when e
// is within 26 degrees of the x axis), b2 = e x b1.
__device__ __forceinline__ void aniso_dir(double ex, double ey, double ez, double eps, double u,
                                          double w, double& nx, double& ny, double& nz) {
  double c = eps > 0.0 ? (2.0 + eps - 2.0 * pow(1.0 + eps, u)) / eps : 1.0 - 2.0 * u;
  c = fmin(fmax(c, -1.0), 1.0);
  const double sn = sqrt(fmax(1.0 - c * c, 0.0));
  const double ph = kTwoPi * w;
  double sp, cp;
  sincos(ph, &sp, &cp);
  double b1x, b1y, b1z;
  if (fabs(ex) < 0.9) {  // e x (1, 0, 0) = (0, ez, -ey)
    const double r = sqrt(ey * ey + ez * ez);
    b1x = 0.0;
    b1y = ez / r;
    b1z = -ey / r;
  } else {  // e x (0, 1, 0) = (-ez, 0, ex)
    const double r = sqrt(ez * ez + ex * ex);
    b1x = -ez / r;
    b1y = 0.0;
    b1z = ex / r;
  }
  const double b2x = ey * b1z - ez * b1y;
  const double b2y = ez * b1x - ex * b1z;
  const double b2z = ex * b1y - ey * b1x;
  nx = c * ex + sn * (cp * b1x + sp * b2x);
  ny = c * ey + sn * (cp * b1y + sp * b2y);
  nz = c * ez + sn * (cp * b1z + sp * b2z);
}

// The deposit of one position with weight mul (an ionization electron and
// its parent share a position) into a histogram: global memory, or the
// fused emit's LDS histogram, which the workgroup flushes once at its end
// (device-scope atomics of every workgroup on the few lines of the deposit
// array stalled single items of the fused emit by up to 20 us).
__device__ __forceinline__ void deposit_global_n(unsigned long long* dep, double x, double inv_dx,
                                                 int nx, uint32_t mul) {
  int j;
  double f;
  int64_t w1;
  cell_of(x, inv_dx, nx, j, f, w1);
  atomicAdd(&dep[j], (unsigned long long)mul * (unsigned long long)(kOne32 - w1));
  atomicAdd(&dep[j + 1], (unsigned long long)mul * (unsigned long long)w1);
}

// An electron output of pass a at slot dest (state x, vx, vy, vz after a's
// step, pool entry id already written) decided for the next step b, one slot
// at a time: the push with b's field, the wall and collision decisions where
// needed, the decision code, the next pass's tile totals and the deposit
// (into sH, the workgroup's LDS histogram), and the pushed state stored at
// the slot.
// ef[2]: b's field at the two nodes of x's cell and cw the candidacy word of
// dest, loaded by the caller ahead of the collision kinematics.
__device__ __forceinline__ void next_step_output(const PartArgs& a, const PartArgs& b,
                                                 unsigned long long* s_cnt, int64_t dest,
                                                 double x, double vx, double vy, double vz,
                                                 uint32_t id, const double* ef, uint32_t cw,
                                                 unsigned long long* sH) {
  uint32_t c2 = kCodePushed, o2 = 1u, b2 = 0u;
  int j;
  double f;
  int64_t w1;
  cell_of(x, b.inv_dx, b.nx, j, f, w1);
  // push() on the prefetched node values: the same operations and operands
  const double Ep = (1.0 - f) * ef[0] + f * ef[1];
  vx = vx + b.acc * Ep;
  x = x + vx * b.dts;
  const bool cand = ((cw >> (dest & 31)) & 1u) != 0;
  if (cand || !(x >= 0.0 && x <= b.L) || !isfinite(vx)) {
    const double vyz[2] = {vy, vz};
    decide_rare<0, false, true>(b, s_cnt, dest, cand, x, vx, c2, o2, b2, id, vyz);
  }
  b.codes[dest] = (uint8_t)c2;
  atomicAdd(&b.tcnt[dest / kTile], totals_word(c2, o2, b2));
  if (o2) deposit_global_n(sH, x, b.inv_dx, b.nx, o2);
  store3(a, dest, x, vx, id);
}

// VAR: the method-variant paths (anisotropic elastic scattering, Opal
// sharing) are compiled in; without them the kernels stay smaller.
// PUSHED: the slot's input holds the pushed state (the previous step's
// fused emit stored it), so it is not pushed again. FUSED (electrons, with PUSHED): the outputs are
// then decided for the next step nb (next_step_output).
template <int SP, bool VAR, bool PUSHED = false, bool FUSED = false>
__device__ __forceinline__ void rare_slot(const PartArgs& a, unsigned long long* s_cnt,
                                          int64_t slot, uint32_t c, int64_t dest, int64_t r,
                                          int64_t bbase, const PartArgs* nb = nullptr,
                                          unsigned long long* sHn = nullptr) {
  static_assert(!FUSED || SP == 0, "only electron slots are fused");
  const uint32_t step = a.step;
  const double L = a.L;
  const int64_t bdest = bbase + r;
  double x, vx, vy, vz;
  uint32_t id;
  // FUSED: the next step's field at the particle's cell (collisions do not
  // move it; an ionization electron is born there) and the candidacy words
  // of its output slots, loaded with the particle
  double ef[2] = {0.0, 0.0};
  uint32_t cw0 = 0u, cw1 = 0u;
  if (PUSHED) {
    x = a.xin[slot];
    vx = a.vxin[slot];
    id = a.idin[slot];
    if (FUSED) {
      if (dest < a.cap) cw0 = nb->cand[dest >> 5];
      if (dest + 1 < a.cap) cw1 = nb->cand[(dest + 1) >> 5];
      const int jn = cell_key(x, nb->inv_dx, nb->nx);
      ef[0] = nb->E[jn];
      ef[1] = nb->E[jn + 1];
    }
    vy = a.pvy[id];
    vz = a.pvz[id];
  } else {
    reload(a, a.E, slot, c, x, vx, id, vy, vz);
    if (FUSED) {
      if (dest < a.cap) cw0 = nb->cand[dest >> 5];
      if (dest + 1 < a.cap) cw1 = nb->cand[(dest + 1) >> 5];
      const int jn = cell_key(x, nb->inv_dx, nb->nx);
      ef[0] = nb->E[jn];
      ef[1] = nb->E[jn + 1];
    }
  }
  const Outcome oc = outcome<SP>(c);
  bool child = false;
  double cvx = 0, cvy = 0, cvz = 0, bxp = 0, bvx = 0, bvy = 0, bvz = 0;
  if (SP == 0) {
    const uint32_t proc = (c >> 3) & 7u;
    const uint4 r1 = draw(step, (uint32_t)slot, 0, 1, a.seed, a.run);
    const double v2 = vx * vx + vy * vy + vz * vz;
    if (proc == 2) {
      // elastic on an atom at rest: isotropic in the CM frame, or (variant)
      // deflected by the screened-Coulomb angle about the incident direction
      const double speed = sqrt(v2);
      double nx_, ny_, nz_;
      if (VAR && (a.model & kModelAniso) && speed > 0.0)
        aniso_dir(vx / speed, vy / speed, vz / speed, a.ek * v2, u01(r1.x), u01(r1.y), nx_, ny_,
                  nz_);
      else
        iso_dir(u01(r1.x), u01(r1.y), nx_, ny_, nz_);
      const double gg = a.mm * speed;
      vx = a.mr * vx + gg * nx_;
      vy = a.mr * vy + gg * ny_;
      vz = a.mr * vz + gg * nz_;
    } else if (proc == 3) {
      // excitation: threshold energy lost, new direction isotropic
      double eps = a.ek * v2 - a.exc_thr;
      if (eps < 0.0) eps = 0.0;
      const double s1 = sqrt(eps * a.ve);
      double nx_, ny_, nz_;
      iso_dir(u01(r1.x), u01(r1.y), nx_, ny_, nz_);
      vx = s1 * nx_;
      vy = s1 * ny_;
      vz = s1 * nz_;
    } else {
      // ionization: energy above threshold shared uniformly, both electrons
      // isotropic, the new ion thermal
      const uint4 r2 = draw(step, (uint32_t)slot, 0, 2, a.seed, a.run);
      const uint4 r3 = draw(step, (uint32_t)slot, 0, 3, a.seed, a.run);
      double eps = a.ek * v2 - a.ion_thr;
      if (eps < 0.0) eps = 0.0;
      // energy above threshold shared uniformly, or (variant) as Opal et al.
      const double e_ej = (VAR && (a.model & kModelOpal))
                              ? kOpalW * tan(u01(r2.x) * atan(eps / (2.0 * kOpalW)))
                              : u01(r2.x) * eps;
      const double e_sc = eps - e_ej;
      const double s_sc = sqrt(e_sc * a.ve);
      const double s_ej = sqrt(e_ej * a.ve);
      double ax, ay, az, bx, by, bz;
      iso_dir(u01(r1.x), u01(r1.y), ax, ay, az);
      iso_dir(u01(r1.z), u01(r1.w), bx, by, bz);
      vx = s_sc * ax;
      vy = s_sc * ay;
      vz = s_sc * az;
      child = true;
      cvx = s_ej * bx;
      cvy = s_ej * by;
      cvz = s_ej * bz;
      double n1, n2, n3, dmy;
      box_muller(u01(r3.x), u01(r3.y), n1, n2);
      box_muller(u01(r3.z), u01(r3.w), n3, dmy);
      bxp = x;
      bvx = a.sig_g * n1;
      bvy = a.sig_g * n2;
      bvz = a.sig_g * n3;
    }
  } else if (oc.own) {
    // Ar+ candidate on a thermal atom drawn for it: isotropic elastic in the
    // CM frame, backward (charge transfer), or null
    const uint4 r0 = draw(step, (uint32_t)slot, 1, 0, a.seed, a.run);
    const uint4 r1 = draw(step, (uint32_t)slot, 1, 1, a.seed, a.run);
    double n1, n2, n3, dmy;
    box_muller(u01(r1.x), u01(r1.y), n1, n2);
    box_muller(u01(r1.z), u01(r1.w), n3, dmy);
    const double ax = a.sig_g * n1, ay = a.sig_g * n2, az = a.sig_g * n3;
    const double gx = vx - ax, gy = vy - ay, gz = vz - az;
    const double g = sqrt(gx * gx + gy * gy + gz * gz);
    const double tv = g * a.inv_dv;
    if (!(tv < (double)(a.ntab - 1))) atomicAdd(&s_cnt[C_BEYOND_TABLE], 1ull);
    const double r = u01(r0.z) * a.numax;
    uint32_t proc = 1;
    if (r < cum_nu(a.cum, a.ntab, 0, tv)) {
      proc = 2;
      atomicAdd(&s_cnt[C_I_ISO], 1ull);
      const uint4 r2 = draw(step, (uint32_t)slot, 1, 2, a.seed, a.run);
      double ux, uy, uz;
      iso_dir(u01(r2.x), u01(r2.y), ux, uy, uz);
      const double hg = 0.5 * g;
      vx = 0.5 * (vx + ax) + hg * ux;
      vy = 0.5 * (vy + ay) + hg * uy;
      vz = 0.5 * (vz + az) + hg * uz;
    } else if (r < cum_nu(a.cum, a.ntab, 1, tv)) {
      proc = 3;
      atomicAdd(&s_cnt[C_I_BACK], 1ull);
      vx = ax;
      vy = ay;
      vz = az;
    }
    a.codes[slot] = (uint8_t)((c & ~kIonPending) | (proc << 3));
  } else {
    // secondary electron from the wall the ion hit, half-Maxwellian
    const uint4 r3 = draw(step, (uint32_t)slot, 1, 3, a.seed, a.run);
    double n1, n2, n3, dmy;
    box_muller(u01(r3.x), u01(r3.y), n1, n2);
    box_muller(u01(r3.z), u01(r3.w), n3, dmy);
    bxp = (x < 0.0) ? 0.0 : L;
    bvx = a.sig_se * fabs(n1);
    if (x > L) bvx = -bvx;
    bvy = a.sig_se * n2;
    bvz = a.sig_se * n3;
  }
  if (oc.own) {
    // the particle keeps its pool entry
    if (FUSED) {
      // pool entries first: the next step's decision reads them
      a.pvy[id] = vy;
      a.pvz[id] = vz;
      if (dest < a.cap) next_step_output(a, *nb, s_cnt, dest, x, vx, vy, vz, id, ef, cw0, sHn);
      if (child) {
        const int64_t cid = a.ctl->pbase[SP] + r;
        if (dest + 1 < a.cap && cid < a.pcap) {
          a.pvy[cid] = cvy;
          a.pvz[cid] = cvz;
          next_step_output(a, *nb, s_cnt, dest + 1, x, cvx, cvy, cvz, (uint32_t)cid, ef, cw1, sHn);
        }
      }
    } else {
      if (dest < a.cap) store3(a, dest, x, vx, id);
      a.pvy[id] = vy;
      a.pvz[id] = vz;
      if (child) {
        const int64_t cid = a.ctl->pbase[SP] + r;
        if (dest + 1 < a.cap && cid < a.pcap) {
          store3(a, dest + 1, x, cvx, (uint32_t)cid);
          a.pvy[cid] = cvy;
          a.pvz[cid] = cvz;
        }
      }
    }
  }
  if (oc.birth) {
    const int64_t bid = a.ctl->pbase[1 - SP] + r;
    if (bdest < a.bcap && bid < a.bpcap) {
      a.bx[bdest] = bxp;
      a.bvx[bdest] = bvx;
      a.bid[bdest] = (uint32_t)bid;
      a.bpvy[bid] = bvy;
      a.bpvz[bid] = bvz;
    }
  }
}

template <int SP, bool VAR, bool PUSHED>
__global__ __launch_bounds__(kBlock) void k_rare(PartArgs a) {
  __shared__ unsigned long long s_cnt[NCOUNTERS];
  const int tid = threadIdx.x;
  if (tid < NCOUNTERS) s_cnt[tid] = 0ull;
  __syncthreads();
  const int64_t n = a.ctl->n_rare[SP];
  // births are appended after the other species' particles (as in k_emit)
  const int64_t bbase = SP == 0 ? a.ctl->n_i[a.parity] : a.ctl->e_out;
  // entries interleaved over the workgroups so that they spread over CUs
  const int64_t nb = gridDim.x;
  for (int64_t i = (int64_t)blockIdx.x + nb * tid; i < n; i += nb * kBlock) {
    const uint4 q = a.rq[i];
    rare_slot<SP, VAR, PUSHED>(a, s_cnt, (int64_t)q.x, q.y, (int64_t)q.z, (int64_t)q.w, bbase);
  }
  __syncthreads();
  if (tid < NCOUNTERS && s_cnt[tid]) count_add(a.ctl, tid, s_cnt[tid]);
}

// ---------------------------------------------------------------------------
// An output at slot dest that the fused emit pushed for step b but left
// undecided (it left the gap or is a collision candidate): the wall and
// collision decisions, the decision code, the tile totals, the deposit into
// the workgroup's LDS histogram sH, and the (possibly mirrored) pushed state
// stored back.
__device__ __forceinline__ void deferred_decision(const PartArgs& a, const PartArgs& b,
                                                  unsigned long long* s_cnt, int64_t dest,
                                                  unsigned long long* sH) {
  double x = a.xout[dest], vx = a.vxout[dest];
  const uint32_t id = a.idout[dest];
  const bool cand = ((b.cand[dest >> 5] >> (dest & 31)) & 1u) != 0;
  uint32_t c = kCodePushed, o = 1u, bb = 0u;
  double vyz[2] = {0.0, 0.0};
  if (cand) {
    vyz[0] = a.pvy[id];
    vyz[1] = a.pvz[id];
  }
  decide_rare<0, false, true>(b, s_cnt, dest, cand, x, vx, c, o, bb, id, vyz);
  b.codes[dest] = (uint8_t)c;
  atomicAdd(&b.tcnt[dest / kTile], totals_word(c, o, bb));
  if (o) deposit_global_n(sH, x, b.inv_dx, b.nx, o);
  a.xout[dest] = x;
  a.vxout[dest] = vx;
}

// The electron emit of pass a fused with the electron decisions of the next
// step b (emit_tiles MODE 2): a's input holds pushed, decided state; the
// outputs that need no queued work leave pushed and decided for b, so the
// next step has no decide pass of its own. Contiguous runs of tiles per
// workgroup (as k_emit for electrons); b's field in LDS with the deposit
// histogram, which also takes the rare items' deposits and is flushed once
// per workgroup at its end.
// MODE 2: a's input holds the pushed, decided state; MODE 3: the state
// before the push (the first pipelined step after a plain decide), pushed
// again here with a's field.
#ifndef EMIT_DECIDE_MIN_WAVES
#define EMIT_DECIDE_MIN_WAVES 1  // waves per SIMD the register budget must allow
#endif
//
// Each workgroup ends with the rare work of its own tiles: its queued slots
// of pass a (collision kinematics, the outputs then decided for b) and the
// outputs it deferred, one item per thread; these are chains of dependent
// loads that other workgroups' streaming hides. VAR: the method-variant
// kinematics compiled in.
template <int MODE, bool VAR>
__global__ __launch_bounds__(kBlock, EMIT_DECIDE_MIN_WAVES) void k_emit_decide(PartArgs a, PartArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx;
  double* sE = reinterpret_cast<double*>(smem);
  unsigned long long* sH = reinterpret_cast<unsigned long long*>(sE + nx);
  double* sE0 = MODE == 3 ? reinterpret_cast<double*>(sH + nx) : nullptr;
  __shared__ uint32_t s_wtot[2][kEPairs][kBlock / kWave];
  __shared__ uint32_t s_wr[2][kEPairs][kBlock / kWave];
  __shared__ uint32_t s_ps[2][3][kBlock / kWave];
  __shared__ uint64_t s_red[3][kBlock / kWave];
  __shared__ unsigned long long s_cnt[NCOUNTERS];
  __shared__ uint32_t s_cand[2][kCandWords];
  __shared__ uint32_t s_dcnt[2];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  DevCtl* ctl = a.ctl;
  const int par = a.parity;
  for (int j = tid; j < nx; j += kBlock) sH[j] = 0ull;
  if (tid < NCOUNTERS) s_cnt[tid] = 0ull;
  if (tid == 0) s_dcnt[0] = s_dcnt[1] = 0u;

  int64_t n_tot = uniform64(ctl->n_e[par]);
  if (n_tot > a.cap) n_tot = a.cap;  // the decide has latched the error
  const int64_t bbase = uniform64(ctl->n_i[par]);
  const int ntiles = uniform32((int)((n_tot + kTile - 1) / kTile));
  if (ntiles == 0) {
    if (blockIdx.x == 0 && tid == 0) {
      emit_empty<0>(ctl, par);
      if (b.record) ctl->ncodes[0] = 0;
    }
    return;
  }
  // contiguous runs, the longer ones (one tile more) on the lower workgroup
  // indices: those are dispatched first on each CU, and the oldest waves of
  // a CU are issued first, so they stream faster (measured: workgroups
  // dispatched third on their CU took about 40 % longer per tile)
  const int g = (int)gridDim.x, b_ = (int)blockIdx.x;
  const int q = ntiles / g, r = ntiles % g;
  const int t0 = b_ < r ? b_ * (q + 1) : r * (q + 1) + (b_ - r) * q;
  const int t1 = t0 + (b_ < r ? q + 1 : q);
  __syncthreads();  // sH, s_cnt, s_dcnt set
  if (t0 >= t1) return;

  int jlo = INT_MAX, jhi = -1;
  int64_t rq_range[3];
  emit_tiles<0, (kMaxNx + kBlock - 1) / kBlock, MODE>(a, t0, t1, 1, ntiles, n_tot, bbase, sE,
                                                      s_wtot, s_wr, s_ps, s_red, &b, sH, s_cnt,
                                                      &jlo, &jhi, s_cand, s_dcnt, sE0, rq_range);
  // this workgroup's queued slots and deferred decisions, their deposits
  // into the same LDS histogram
  const int64_t q0 = uniform64(rq_range[0]);
  const int64_t nq = uniform64(rq_range[1]) - q0;
  const int64_t out0 = uniform64(rq_range[2]);
  const int64_t nd = (int64_t)s_dcnt[0];
  // queued slots from the first thread up, deferred outputs from the last
  // thread down: the two chains sit in different waves while they fit
  for (int64_t i = tid; i < nq; i += kBlock) {
    const uint4 q = a.rq[q0 + i];
    rare_slot<0, VAR, MODE == 2, true>(a, s_cnt, (int64_t)q.x, q.y, (int64_t)q.z, (int64_t)q.w,
                                       bbase, &b, sH);
  }
  for (int64_t i = kBlock - 1 - tid; i < nd; i += kBlock)
    deferred_decision(a, b, s_cnt, (int64_t)a.dq[out0 + i], sH);
  __syncthreads();
  // one flush of the histogram over the cells the workgroup's outputs and
  // rare items touched
  for (int j = tid; j < nx; j += kBlock) {
    const unsigned long long v = sH[j];
    if (v) atomicAdd(&b.dep_own[j], v);
  }
  if (tid < NCOUNTERS && s_cnt[tid]) count_add(ctl, tid, s_cnt[tid]);
}

// ---------------------------------------------------------------------------
// k_tail: the end of a step and the start of the next. Workgroup 0 solves
// the next step's field (it needs only the deposits k_decide made); the
// other workgroups take the queued slots of this step's last particle pass.
// The two are independent: the field goes to the other E buffer, and the
// queued slots read the E of this step.

template <int SP, bool VAR, bool PUSHED>
__global__ __launch_bounds__(kFieldThreads) void k_tail(FieldArgs f, PartArgs a) {
  if (blockIdx.x == 0) {
    field_block(f);
    return;
  }
  __shared__ unsigned long long s_cnt[NCOUNTERS];
  const int tid = threadIdx.x;
  if (tid < NCOUNTERS) s_cnt[tid] = 0ull;
  __syncthreads();
  const int64_t n = a.ctl->n_rare[SP];
  const int64_t bbase = SP == 0 ? a.ctl->n_i[a.parity] : a.ctl->e_out;
  // entries interleaved over the workgroups (one CU each) so that the few
  // hundred to thousands of queued slots spread over many CUs
  const int64_t nb = gridDim.x - 1;
  for (int64_t i = (int64_t)(blockIdx.x - 1) + nb * tid; i < n; i += nb * kFieldThreads) {
    const uint4 q = a.rq[i];
    rare_slot<SP, VAR, PUSHED>(a, s_cnt, (int64_t)q.x, q.y, (int64_t)q.z, (int64_t)q.w, bbase);
  }
  __syncthreads();
  if (tid < NCOUNTERS && s_cnt[tid]) count_add(a.ctl, tid, s_cnt[tid]);
}

hipError_t launch_tail(int species, const FieldArgs& f, const PartArgs& a, int rare_blocks,
                       hipStream_t s, bool pushed) {
  if (f.nx > kMaxNx || f.nx < 3 || rare_blocks < 1) return hipErrorInvalidValue;
  const dim3 g(1 + rare_blocks), t(kFieldThreads);
  if (species == 1)
    hipLaunchKernelGGL((k_tail<1, false, false>), g, t, 0, s, f, a);
  else if (pushed && a.model)
    hipLaunchKernelGGL((k_tail<0, true, true>), g, t, 0, s, f, a);
  else if (pushed)
    hipLaunchKernelGGL((k_tail<0, false, true>), g, t, 0, s, f, a);
  else if (a.model)
    hipLaunchKernelGGL((k_tail<0, true, false>), g, t, 0, s, f, a);
  else
    hipLaunchKernelGGL((k_tail<0, false, false>), g, t, 0, s, f, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched passes: one launch runs the same pass of many independent
// discharges. A kernel takes n argument blocks in device memory, one per
// discharge, and lays the discharges' tiles (or queued slots) end to end;
// each workgroup takes a contiguous run of that sequence and switches
// discharge at the boundaries, so that small discharges share the chip
// instead of each leaving most of it idle.

// Slots of a particle pass of discharge a: [0, n_push) are pushed and
// [n_push, n_tot) carried, clamped to the capacity.
template <int SP>
__device__ __forceinline__ void pass_slots(const PartArgs& a, int64_t& n_push, int64_t& n_tot) {
  const DevCtl* ctl = a.ctl;
  n_push = SP == 0 ? ctl->n_e[a.parity] : ctl->n_i[a.parity];
  n_tot = SP == 0 ? n_push : n_push + ctl->i_births;
  if (n_tot > a.cap) {
    n_tot = a.cap;
    if (n_push > n_tot) n_push = n_tot;
  }
}

// First discharge at or after d whose run of the sequence ends beyond t.
__device__ __forceinline__ int next_owner(const int64_t* s_start, int n, int d, int64_t t) {
  while (d < n && s_start[d + 1] <= t) ++d;
  return uniform32(d);
}

// This workgroup's run [tb, te) of a sequence of T items.
__device__ __forceinline__ void wg_run(int64_t T, int64_t& tb, int64_t& te) {
  tb = uniform64(T * (int64_t)blockIdx.x / (int64_t)gridDim.x);
  te = uniform64(T * ((int64_t)blockIdx.x + 1) / (int64_t)gridDim.x);
}

template <int SP, bool MEASURE>
__global__ __launch_bounds__(kDB) void k_decide_b(const PartArgs* __restrict__ args, int n,
                                                  int nx_max, int nbins_max) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* sE = reinterpret_cast<double*>(smem);
  unsigned long long* sH = reinterpret_cast<unsigned long long*>(sE + nx_max);
  double* sEW = reinterpret_cast<double*>(sH + nx_max);                 // MEASURE
  unsigned int* sEEPF = reinterpret_cast<unsigned int*>(sEW + nx_max);  // MEASURE

  __shared__ int s_lo, s_hi;
  __shared__ unsigned long long s_cnt[NCOUNTERS];
  __shared__ int64_t s_ts[kMaxBatch + 1];
  __shared__ int64_t s_w[kDB / kWave];

  const int tid = threadIdx.x;
  // workgroup d zeroes the next totals buffer of discharge d
  for (int d = blockIdx.x; d < n; d += gridDim.x) {
    const PartArgs& a = args[d];
    for (int64_t i = tid; i < a.max_tiles; i += kDB) a.tcnt_next[i] = 0ull;
  }
  for (int j = tid; j < nx_max; j += kDB) {
    sH[j] = 0ull;
    if (MEASURE) sEW[j] = 0.0;
  }
  if (MEASURE)
    for (int b = tid; b < nbins_max; b += kDB) sEEPF[b] = 0u;
  if (tid < NCOUNTERS) s_cnt[tid] = 0ull;
  if (tid == 0) {
    s_lo = INT_MAX;
    s_hi = -1;
  }

  int64_t tiles = 0;
  if (tid < n) {
    const PartArgs& a = args[tid];
    int64_t n_push, n_tot;
    pass_slots<SP>(a, n_push, n_tot);
    tiles = (n_tot + kTile - 1) / kTile;
    if (blockIdx.x == 0) {
      DevCtl* ctl = a.ctl;
      const int64_t np = SP == 0 ? ctl->n_e[a.parity] : ctl->n_i[a.parity];
      if ((SP == 0 ? np : np + ctl->i_births) > a.cap) latch_error(ctl, kErrCapacity);
      if (a.record) ctl->ncodes[SP] = n_push;
      count_add(ctl, SP == 0 ? C_E_PUSHED : C_I_PUSHED, (unsigned long long)n_push);
    }
  }
  block_exclusive<kDB>(tiles, n, s_ts, s_w);
  int64_t tb, te;
  wg_run(uniform64(s_ts[n]), tb, te);
  int d = next_owner(s_ts, n, 0, tb);
  for (int64_t t = tb; t < te;) {
    const PartArgs& a = args[d];
    const int64_t ts = uniform64(s_ts[d]);
    const int64_t se = min(te, uniform64(s_ts[d + 1]));
    int64_t n_push, n_tot;
    pass_slots<SP>(a, n_push, n_tot);
    n_push = uniform64(n_push);
    n_tot = uniform64(n_tot);
    stage_field<kDB, 2>(sE, a.E, a.nx);  // (register budget of the batched kernel)
    __syncthreads();
    decide_tiles<SP, MEASURE>(a, (int)(t - ts), (int)(se - ts), 1, n_push, n_tot, sE, sH, sEW,
                              sEEPF, s_lo, s_hi, s_cnt);
    // this discharge's event counts and EEPF counts
    if (tid < NCOUNTERS) {
      if (s_cnt[tid]) count_add(a.ctl, tid, s_cnt[tid]);
      s_cnt[tid] = 0ull;
    }
    if (MEASURE) {
      for (int b = tid; b < a.nbins; b += kDB)
        if (sEEPF[b]) {
          atomicAdd(&a.eepf[b], (unsigned long long)sEEPF[b]);
          sEEPF[b] = 0u;
        }
    }
    __syncthreads();  // sE is refilled for the next discharge
    t = se;
    d = next_owner(s_ts, n, d + 1, t);
  }
}

template <int SP>
__global__ __launch_bounds__(kBlock) void k_emit_b(const PartArgs* __restrict__ args, int n) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* sE = reinterpret_cast<double*>(smem);
  __shared__ uint32_t s_wtot[2][kEPairs][kBlock / kWave];
  __shared__ uint32_t s_wr[2][kEPairs][kBlock / kWave];
  __shared__ uint32_t s_ps[2][3][kBlock / kWave];
  __shared__ uint64_t s_red[3][kBlock / kWave];
  __shared__ int64_t s_ts[kMaxBatch + 1];
  __shared__ int64_t s_w[kBlock / kWave];

  const int tid = threadIdx.x;
  int64_t tiles = 0;
  if (tid < n) {
    const PartArgs& a = args[tid];
    int64_t n_push, n_tot;
    pass_slots<SP>(a, n_push, n_tot);
    tiles = (n_tot + kTile - 1) / kTile;
    if (tiles == 0 && blockIdx.x == 0) emit_empty<SP>(a.ctl, a.parity);
  }
  block_exclusive<kBlock>(tiles, n, s_ts, s_w);
  int64_t tb, te;
  wg_run(uniform64(s_ts[n]), tb, te);
  int d = next_owner(s_ts, n, 0, tb);
  for (int64_t t = tb; t < te;) {
    const PartArgs& a = args[d];
    const int64_t ts = uniform64(s_ts[d]);
    const int64_t tn = uniform64(s_ts[d + 1]);
    const int64_t se = min(te, tn);
    int64_t n_push, n_tot;
    pass_slots<SP>(a, n_push, n_tot);
    n_tot = uniform64(n_tot);
    const DevCtl* ctl = a.ctl;
    const int64_t bbase = uniform64(SP == 0 ? ctl->n_i[a.parity] : ctl->e_out);
    // (four staging loads per thread: register budget of the batched kernel)
    emit_tiles<SP, 4>(a, (int)(t - ts), (int)(se - ts), 1, (int)(tn - ts), n_tot, bbase, sE,
                      s_wtot, s_wr, s_ps, s_red);
    t = se;
    d = next_owner(s_ts, n, d + 1, t);
  }
}

// Queued slots of n discharges laid end to end (s_rs: prefix of their
// counts): this workgroup's contiguous run of them, one discharge segment at
// a time so that the discharge's arguments are uniform over the workgroup.
template <int SP, int NT, bool VAR>
__device__ __forceinline__ void rare_segments(const PartArgs* __restrict__ args, int n,
                                              const int64_t* s_rs, int wg, int nwg) {
  const int64_t R = uniform64(s_rs[n]);
  const int64_t tb = uniform64(R * (int64_t)wg / (int64_t)nwg);
  const int64_t te = uniform64(R * ((int64_t)wg + 1) / (int64_t)nwg);
  int d = next_owner(s_rs, n, 0, tb);
  for (int64_t t = tb; t < te;) {
    const PartArgs& a = args[d];
    const int64_t rs = uniform64(s_rs[d]);
    const int64_t se = min(te, uniform64(s_rs[d + 1]));
    const int64_t bbase = uniform64(SP == 0 ? a.ctl->n_i[a.parity] : a.ctl->e_out);
    unsigned long long* cnt = a.ctl->counters[blockIdx.x % kCounterSlots];
    for (int64_t i = t + threadIdx.x; i < se; i += NT) {
      const uint4 q = a.rq[i - rs];
      rare_slot<SP, VAR>(a, cnt, (int64_t)q.x, q.y, (int64_t)q.z, (int64_t)q.w, bbase);
    }
    t = se;
    d = next_owner(s_rs, n, d + 1, t);
  }
}

template <int SP, bool VAR>
__global__ __launch_bounds__(kBlock) void k_rare_b(const PartArgs* __restrict__ args, int n) {
  __shared__ int64_t s_rs[kMaxBatch + 1];
  __shared__ int64_t s_w[kBlock / kWave];
  const int tid = threadIdx.x;
  block_exclusive<kBlock>(tid < n ? args[tid].ctl->n_rare[SP] : 0, n, s_rs, s_w);
  rare_segments<SP, kBlock, VAR>(args, n, s_rs, blockIdx.x, gridDim.x);
}

// Workgroups [0, nf) solve the next step's field of nf discharges; the
// others take the queued slots of the last particle pass of n discharges.
template <int SP, bool VAR>
__global__ __launch_bounds__(kFieldThreads) void k_tail_b(const FieldArgs* __restrict__ f, int nf,
                                                          const PartArgs* __restrict__ args,
                                                          int n) {
  if ((int)blockIdx.x < nf) {
    field_block(f[blockIdx.x]);
    return;
  }
  __shared__ int64_t s_rs[kMaxBatch + 1];
  __shared__ int64_t s_w[kFieldThreads / kWave];
  const int tid = threadIdx.x;
  block_exclusive<kFieldThreads>(tid < n ? args[tid].ctl->n_rare[SP] : 0, n, s_rs, s_w);
  rare_segments<SP, kFieldThreads, VAR>(args, n, s_rs, (int)blockIdx.x - nf, (int)gridDim.x - nf);
}

// ---------------------------------------------------------------------------
// host side

static size_t decide_lds(int nx, bool measure, int nbins) {
  size_t b = (size_t)nx * 16;
  if (measure) b += (size_t)nx * 8 + (size_t)nbins * 4;
  return b;
}

static size_t emit_lds(int nx) { return (size_t)nx * 8; }

template <typename K>
static int blocks_per_cu(K kern, size_t lds, int threads = kBlock) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, lds) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

static int clamp_grid(int64_t g, int64_t max_tiles) {
  if (g > max_tiles) g = max_tiles;
  if (g < 1) g = 1;
  return (int)g;
}

static size_t emit_decide_lds(int nx) { return (size_t)nx * 16; }

PartLaunch particle_launch_config(int species, int nx, int nbins, int num_cu, int64_t max_tiles) {
  PartLaunch c{};
  c.max_tiles = max_tiles;
  for (int m = 0; m < 2; ++m) {
    c.lds_decide[m] = decide_lds(nx, m == 1, nbins);
    const size_t l = c.lds_decide[m];
    if (species == 0) {
      c.bpc_decide_by[0][m] = m ? blocks_per_cu(k_decide<0, true, kDB>, l, kDB)
                                : blocks_per_cu(k_decide<0, false, kDB>, l, kDB);
      c.bpc_decide_by[1][m] = m ? blocks_per_cu(k_decide<0, true, kDBAlt>, l, kDBAlt)
                                : blocks_per_cu(k_decide<0, false, kDBAlt>, l, kDBAlt);
    } else {
      c.bpc_decide_by[0][m] = blocks_per_cu(k_decide<1, false, kDB>, l, kDB);
      c.bpc_decide_by[1][m] = blocks_per_cu(k_decide<1, false, kDBAlt>, l, kDBAlt);
    }
  }
  particle_launch_block(c, num_cu, kDB);
  c.lds_emit = emit_lds(nx);
  const int bpc = species == 0 ? blocks_per_cu(k_emit<0, 0>, c.lds_emit)
                               : blocks_per_cu(k_emit<1, 0>, c.lds_emit);
  c.grid_emit = clamp_grid((int64_t)bpc * num_cu, max_tiles);
  c.bpc_emit = bpc;
  c.lds_emit_decide = emit_decide_lds(nx);
  c.bpc_emit_decide = species == 0 ? blocks_per_cu(k_emit_decide<2, false>, c.lds_emit_decide) : 1;
  c.grid_emit_decide = clamp_grid((int64_t)c.bpc_emit_decide * num_cu, max_tiles);
  c.bpc_emit_decide3 =
      species == 0 ? blocks_per_cu(k_emit_decide<3, false>, c.lds_emit_decide + (size_t)nx * 8) : 1;
  c.grid_emit_decide3 = clamp_grid((int64_t)c.bpc_emit_decide3 * num_cu, max_tiles);
  c.grid_rare = num_cu * 2;
  return c;
}

bool particle_launch_block(PartLaunch& c, int num_cu, int threads) {
  if (threads != kDB && threads != kDBAlt) return false;
  const int k = threads == kDB ? 0 : 1;
  c.decide_block = threads;
  for (int m = 0; m < 2; ++m) {
    c.bpc_decide[m] = c.bpc_decide_by[k][m];
    c.grid_decide[m] = clamp_grid((int64_t)c.bpc_decide[m] * num_cu, c.max_tiles);
  }
  return true;
}

void particle_launch_set(PartLaunch& c, int num_cu, int kd, int ke) {
  for (int m = 0; m < 2; ++m) {
    const int k = kd < 1 ? 1 : (kd > c.bpc_decide[m] ? c.bpc_decide[m] : kd);
    c.grid_decide[m] = clamp_grid((int64_t)k * num_cu, c.max_tiles);
  }
  const int k = ke < 1 ? 1 : (ke > c.bpc_emit ? c.bpc_emit : ke);
  c.grid_emit = clamp_grid((int64_t)k * num_cu, c.max_tiles);
  const int k2 = ke < 1 ? 1 : (ke > c.bpc_emit_decide ? c.bpc_emit_decide : ke);
  c.grid_emit_decide = clamp_grid((int64_t)k2 * num_cu, c.max_tiles);
  const int k3 = ke < 1 ? 1 : (ke > c.bpc_emit_decide3 ? c.bpc_emit_decide3 : ke);
  c.grid_emit_decide3 = clamp_grid((int64_t)k3 * num_cu, c.max_tiles);
}

hipError_t launch_particle_kernel(int kernel, int species, bool measure, const PartArgs& a,
                                  const PartLaunch& c, hipStream_t s, int flags) {
  const int m = (species == 0 && measure) ? 1 : 0;
  const bool pushed = (flags & kLaunchPushed) != 0;
  if (species == 1 && pushed) return hipErrorInvalidValue;
  if (kernel == 0) {
    const dim3 g(c.grid_decide[m]);
    const size_t lds = c.lds_decide[m];
    if (c.decide_block == kDB) {
      const dim3 t(kDB);
      if (species == 1)
        hipLaunchKernelGGL((k_decide<1, false, kDB>), g, t, lds, s, a);
      else if (m)
        hipLaunchKernelGGL((k_decide<0, true, kDB>), g, t, lds, s, a);
      else
        hipLaunchKernelGGL((k_decide<0, false, kDB>), g, t, lds, s, a);
    } else if (c.decide_block == kDBAlt) {
      const dim3 t(kDBAlt);
      if (species == 1)
        hipLaunchKernelGGL((k_decide<1, false, kDBAlt>), g, t, lds, s, a);
      else if (m)
        hipLaunchKernelGGL((k_decide<0, true, kDBAlt>), g, t, lds, s, a);
      else
        hipLaunchKernelGGL((k_decide<0, false, kDBAlt>), g, t, lds, s, a);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (kernel == 1) {
    const dim3 g(c.grid_emit), t(kBlock);
    if (species == 1)
      hipLaunchKernelGGL((k_emit<1, 0>), g, t, c.lds_emit, s, a);
    else if (pushed)
      hipLaunchKernelGGL((k_emit<0, 1>), g, t, c.lds_emit, s, a);
    else
      hipLaunchKernelGGL((k_emit<0, 0>), g, t, c.lds_emit, s, a);
  } else {
    const dim3 g(c.grid_rare), t(kBlock);
    if (species == 1)
      hipLaunchKernelGGL((k_rare<1, false, false>), g, t, 0, s, a);
    else if (pushed && a.model)
      hipLaunchKernelGGL((k_rare<0, true, true>), g, t, 0, s, a);
    else if (pushed)
      hipLaunchKernelGGL((k_rare<0, false, true>), g, t, 0, s, a);
    else if (a.model)
      hipLaunchKernelGGL((k_rare<0, true, false>), g, t, 0, s, a);
    else
      hipLaunchKernelGGL((k_rare<0, false, false>), g, t, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_emit_decide(const PartArgs& a, const PartArgs& b, const PartLaunch& c,
                              hipStream_t s, bool pushed) {
  if (a.nx > kMaxNx || a.nx != b.nx) return hipErrorInvalidValue;
  const dim3 g2(c.grid_emit_decide), g3(c.grid_emit_decide3), t(kBlock);
  const size_t l2 = c.lds_emit_decide, l3 = c.lds_emit_decide + (size_t)a.nx * 8;
  if (pushed && a.model)
    hipLaunchKernelGGL((k_emit_decide<2, true>), g2, t, l2, s, a, b);
  else if (pushed)
    hipLaunchKernelGGL((k_emit_decide<2, false>), g2, t, l2, s, a, b);
  else if (a.model)
    hipLaunchKernelGGL((k_emit_decide<3, true>), g3, t, l3, s, a, b);
  else
    hipLaunchKernelGGL((k_emit_decide<3, false>), g3, t, l3, s, a, b);
  return hipGetLastError();
}


BatchLaunch batch_launch_config(int nx_max, int nbins_max, int num_cu, const int64_t max_tiles[2]) {
  BatchLaunch c{};
  c.nx_max = nx_max;
  c.nbins_max = nbins_max;
  for (int sp = 0; sp < 2; ++sp) {
    for (int m = 0; m < 2; ++m) {
      c.lds_decide[sp][m] = decide_lds(nx_max, m == 1, nbins_max);
      int bpc;
      if (sp == 0)
        bpc = m ? blocks_per_cu(k_decide_b<0, true>, c.lds_decide[sp][m], kDB)
                : blocks_per_cu(k_decide_b<0, false>, c.lds_decide[sp][m], kDB);
      else
        bpc = blocks_per_cu(k_decide_b<1, false>, c.lds_decide[sp][m], kDB);
      c.grid_decide[sp][m] = clamp_grid((int64_t)bpc * num_cu, max_tiles[sp]);
    }
  }
  c.lds_emit = emit_lds(nx_max);
  for (int sp = 0; sp < 2; ++sp) {
    const int bpc = sp == 0 ? blocks_per_cu(k_emit_b<0>, c.lds_emit)
                            : blocks_per_cu(k_emit_b<1>, c.lds_emit);
    c.grid_emit[sp] = clamp_grid((int64_t)bpc * num_cu, max_tiles[sp]);
  }
  c.grid_rare = num_cu * 2;
  return c;
}

hipError_t launch_batch_pass(int kernel, int species, bool measure, const PartArgs* args, int n,
                             const BatchLaunch& c, hipStream_t s, bool variants) {
  if (n < 1 || n > kMaxBatch || species < 0 || species > 1) return hipErrorInvalidValue;
  const int m = (species == 0 && measure) ? 1 : 0;
  if (kernel == 0) {
    const dim3 g(c.grid_decide[species][m]);
    const size_t lds = c.lds_decide[species][m];
    if (species == 1)
      hipLaunchKernelGGL((k_decide_b<1, false>), g, dim3(kDB), lds, s, args, n, c.nx_max,
                         c.nbins_max);
    else if (m)
      hipLaunchKernelGGL((k_decide_b<0, true>), g, dim3(kDB), lds, s, args, n, c.nx_max,
                         c.nbins_max);
    else
      hipLaunchKernelGGL((k_decide_b<0, false>), g, dim3(kDB), lds, s, args, n, c.nx_max,
                         c.nbins_max);
  } else if (kernel == 1) {
    if (species == 0)
      hipLaunchKernelGGL((k_emit_b<0>), dim3(c.grid_emit[0]), dim3(kBlock), c.lds_emit, s, args, n);
    else
      hipLaunchKernelGGL((k_emit_b<1>), dim3(c.grid_emit[1]), dim3(kBlock), c.lds_emit, s, args, n);
  } else {
    if (species == 0 && variants)
      hipLaunchKernelGGL((k_rare_b<0, true>), dim3(c.grid_rare), dim3(kBlock), 0, s, args, n);
    else if (species == 0)
      hipLaunchKernelGGL((k_rare_b<0, false>), dim3(c.grid_rare), dim3(kBlock), 0, s, args, n);
    else
      hipLaunchKernelGGL((k_rare_b<1, false>), dim3(c.grid_rare), dim3(kBlock), 0, s, args, n);
  }
  return hipGetLastError();
}

hipError_t launch_batch_tail(int species, const FieldArgs* f, int nf, const PartArgs* args, int n,
                             int rare_blocks, hipStream_t s, bool variants) {
  if (nf < 0 || nf > kMaxBatch || n < 0 || n > kMaxBatch || rare_blocks < 1)
    return hipErrorInvalidValue;
  const dim3 g(nf + rare_blocks);
  if (species == 0 && variants)
    hipLaunchKernelGGL((k_tail_b<0, true>), g, dim3(kFieldThreads), 0, s, f, nf, args, n);
  else if (species == 0)
    hipLaunchKernelGGL((k_tail_b<0, false>), g, dim3(kFieldThreads), 0, s, f, nf, args, n);
  else
    hipLaunchKernelGGL((k_tail_b<1, false>), g, dim3(kFieldThreads), 0, s, f, nf, args, n);
  return hipGetLastError();
}

}  // namespace pic
