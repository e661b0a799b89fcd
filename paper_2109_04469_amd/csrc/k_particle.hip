// Particle kernel: one pass over a species' SoA streams per step, fusing
// field gather, leap-frog push, the wall model and null-collision MCC with
// order-preserving compaction, inline births and the CIC deposit of the new
// positions (arXiv:2109.04469, Sec. 2 steps 3-6 and step 1 of the next step).
//
// Schedule. A persistent grid (a few workgroups per CU) takes tiles of
// kTile consecutive slots from an atomic ticket, so tiles are started in slot
// order; the next ticket is requested while the current tile is processed.
// Per tile:
//   A  each thread loads kPPT particles (coalesced 8-byte streams), pushes
//      them, applies the wall and decides the collision candidacy (and, for
//      electrons, the process, which fixes the number of outputs); only the
//      pushed state and a decision code stay in registers;
//   B  a block scan of the per-particle output counts (0, 1 or 2 slots for
//      the own species, 0 or 1 birth of the other species) and a decoupled
//      look-back over earlier tiles (two lanes, one per count) give every
//      output its global slot;
//   C  outputs are written and the new positions deposited into an LDS
//      histogram in 2^-32 fixed point. Particles that need collision
//      kinematics, an ion process choice or a secondary electron (a small
//      fraction) are handled afterwards in one non-unrolled loop, so the
//      transcendental-heavy code exists once and does not set the register
//      budget of the streaming part. The touched node range is then added to
//      the global deposit with integer atomics (a few nodes per tile once the
//      particles are cell-sorted) and cleared.
// Survivors keep their relative order and an ionization electron follows its
// parent; births of the other species (Ar+ from ionization, secondary
// electrons from ion impact) are appended after that species' particles in
// parent-slot order.
#include <climits>

#include "pic_internal.h"

#ifndef PIC_TICKETS
#define PIC_TICKETS 1
#endif
#ifndef PIC_COOP
#define PIC_COOP 0
#endif
#ifdef PIC_WAVES_PER_EU
#define PIC_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(PIC_WAVES_PER_EU)))
#else
#define PIC_WAVES_ATTR
#endif

namespace pic {

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t value) {
  return ((uint64_t)(epoch & 0x3FFFFFFFu) << 34) | ((uint64_t)flag << 32) | (uint64_t)value;
}

// The wait on a predecessor is bounded: a tile is published by the
// workgroup that took its ticket, which is already running, so the bound is
// never reached in a correct run; if it were, the error is latched and the
// kernel still ends.
constexpr uint32_t kMaxSpin = 1u << 22;

// Exclusive prefix of value `which` (0: own outputs, 1: births) over tiles
// [0, t), from the status words of the earlier tiles.
__device__ uint64_t look_back(uint64_t* tstat, int64_t t, int which, uint32_t epoch,
                              DevCtl* ctl) {
  uint64_t excl = 0;
  int64_t pos = t - 1;
  const uint64_t want = epoch & 0x3FFFFFFFu;
  uint32_t spins = 0;
  while (pos >= 0) {
    const uint64_t w = ld_agent(tstat + 2 * pos + which);
    const uint32_t flag = (uint32_t)(w >> 32) & 3u;
    if ((w >> 34) != want || flag == 0) {
      if (++spins >= kMaxSpin) {
        latch_error(ctl, kErrLookback);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += (uint32_t)w;
    if (flag == 2) break;
    --pos;
  }
  return excl;
}

// internal code bits beyond the recorded byte
constexpr uint32_t kAlive = 1u << 8;
constexpr uint32_t kPass = 1u << 9;
constexpr uint32_t kIonCand = 1u << 10;  // ion collision candidate, process not yet chosen

template <int SP>
__device__ __forceinline__ bool is_rare(uint32_t c) {
  if (SP == 0) return (c & kAlive) && ((c >> 3) & 7u) >= 2u;
  return ((c & kAlive) && (c & kIonCand)) || (!(c & kAlive) && (c & 7u) == 3u && (c & kCodePushed));
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

__device__ __forceinline__ void store4(const PartArgs& a, int64_t i, double x, double vx, double vy,
                                       double vz) {
  a.xout[i] = x;
  a.vxout[i] = vx;
  a.vyout[i] = vy;
  a.vzout[i] = vz;
}

// Collision kinematics, the ion process choice and secondary emission for
// one particle, then its outputs and deposit. Kept out of line: it runs for a
// small fraction of particles and its transcendental-heavy code would
// otherwise set the register budget of the whole streaming pass.
template <int SP>
__device__ __forceinline__ void rare_particle(const PartArgs& a, unsigned long long* sH,
                                           unsigned long long* s_cnt, int64_t slot, uint32_t c,
                                           double x, double vx, double vy, double vz,
                                           int64_t dest, int64_t bdest, int& jlo, int& jhi) {
  const uint32_t step = a.step;
  const double L = a.L;
  bool child = false, birth = false;
  double cvx = 0, cvy = 0, cvz = 0, bxp = 0, bvx = 0, bvy = 0, bvz = 0;
  if (SP == 0) {
    const uint32_t proc = (c >> 3) & 7u;
    const uint4 r1 = draw(step, (uint32_t)slot, 0, 1, a.seed, a.run);
    const double v2 = vx * vx + vy * vy + vz * vz;
    if (proc == 2) {
      // elastic on an atom at rest, isotropic in the CM frame
      const double speed = sqrt(v2);
      double nx_, ny_, nz_;
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
      const double e_ej = u01(r2.x) * eps;
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
      birth = true;
      bxp = x;
      bvx = a.sig_g * n1;
      bvy = a.sig_g * n2;
      bvz = a.sig_g * n3;
    }
  } else if (c & kAlive) {
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
    const double* c0 = a.cum;
    const double* c1 = a.cum + a.ntab;
    double nu0, nu1;
    if (tv < (double)(a.ntab - 1)) {
      const int kk = (int)tv;
      const double tt = tv - (double)kk;
      nu0 = (1.0 - tt) * c0[kk] + tt * c0[kk + 1];
      nu1 = (1.0 - tt) * c1[kk] + tt * c1[kk + 1];
    } else {
      atomicAdd(&s_cnt[C_BEYOND_TABLE], 1ull);
      nu0 = c0[a.ntab - 1];
      nu1 = c1[a.ntab - 1];
    }
    const double r = u01(r0.z) * a.numax;
    uint32_t proc = 1;
    if (r < nu0) {
      proc = 2;
      atomicAdd(&s_cnt[C_I_ISO], 1ull);
      const uint4 r2 = draw(step, (uint32_t)slot, 1, 2, a.seed, a.run);
      double ux, uy, uz;
      iso_dir(u01(r2.x), u01(r2.y), ux, uy, uz);
      const double hg = 0.5 * g;
      vx = 0.5 * (vx + ax) + hg * ux;
      vy = 0.5 * (vy + ay) + hg * uy;
      vz = 0.5 * (vz + az) + hg * uz;
    } else if (r < nu1) {
      proc = 3;
      atomicAdd(&s_cnt[C_I_BACK], 1ull);
      vx = ax;
      vy = ay;
      vz = az;
    }
    c |= proc << 3;
    if (a.record) a.codes[slot] = (uint8_t)(c & 0xFFu);
  } else {
    // secondary electron from the wall the ion hit, half-Maxwellian
    const uint4 r3 = draw(step, (uint32_t)slot, 1, 3, a.seed, a.run);
    double n1, n2, n3, dmy;
    box_muller(u01(r3.x), u01(r3.y), n1, n2);
    box_muller(u01(r3.z), u01(r3.w), n3, dmy);
    birth = true;
    bxp = (x < 0.0) ? 0.0 : L;
    bvx = a.sig_se * fabs(n1);
    if (x > L) bvx = -bvx;
    bvy = a.sig_se * n2;
    bvz = a.sig_se * n3;
  }
  if (c & kAlive) {
    if (dest < a.cap) store4(a, dest, x, vx, vy, vz);
    if (child && dest + 1 < a.cap) store4(a, dest + 1, x, cvx, cvy, cvz);
    deposit_lds(sH, x, a.inv_dx, a.nx, child ? 2ull : 1ull, jlo, jhi);
  }
  if (birth) {
    if (bdest < a.bcap) {
      a.bx[bdest] = bxp;
      a.bvx[bdest] = bvx;
      a.bvy[bdest] = bvy;
      a.bvz[bdest] = bvz;
    }
    deposit_global(a.dep_other, bxp, a.inv_dx, a.nx);
  }
}

template <int SP, bool MEASURE>
__global__ __launch_bounds__(kBlock) PIC_WAVES_ATTR void k_particle(PartArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx;
  double* sE = reinterpret_cast<double*>(smem);
  unsigned long long* sH = reinterpret_cast<unsigned long long*>(sE + nx);
  double* sEW = reinterpret_cast<double*>(sH + nx);                 // MEASURE
  unsigned int* sEEPF = reinterpret_cast<unsigned int*>(sEW + nx);  // MEASURE

  __shared__ uint32_t s_wtot[kPPT][kBlock / kWave];
  __shared__ uint32_t s_woff[kPPT][kBlock / kWave];
  __shared__ uint32_t s_agg[2];
  __shared__ int s_tile;
  __shared__ uint64_t s_pref[2];
  __shared__ int s_lo, s_hi;
  __shared__ unsigned long long s_cnt[NCOUNTERS];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  DevCtl* ctl = a.ctl;
  const int par = a.parity;

  for (int j = tid; j < nx; j += kBlock) {
    sE[j] = a.E[j];
    sH[j] = 0ull;
    if (MEASURE) sEW[j] = 0.0;
  }
  if (MEASURE)
    for (int b = tid; b < a.nbins; b += kBlock) sEEPF[b] = 0u;
  if (tid < NCOUNTERS) s_cnt[tid] = 0ull;
  if (tid == 0) {
    s_lo = INT_MAX;
    s_hi = -1;
  }

  // counts beyond the buffers only arise after a capacity error, which is
  // latched; clamp so no access leaves the arrays
  int64_t n_push = uniform64(SP == 0 ? ctl->n_e[par] : ctl->n_i[par]);
  int64_t n_tot = SP == 0 ? n_push : n_push + uniform64(ctl->i_births);
  if (n_tot > a.cap) {
    if (tid == 0) latch_error(ctl, kErrCapacity);
    n_tot = a.cap;
    if (n_push > n_tot) n_push = n_tot;
  }
  const int64_t bbase = uniform64(SP == 0 ? ctl->n_i[par] : ctl->e_out);
  const int ntiles = uniform32((int)((n_tot + kTile - 1) / kTile));

  if (blockIdx.x == 0 && tid == 0) {
    if (a.record) ctl->ncodes[SP] = n_push;
    atomicAdd(&ctl->counters[SP == 0 ? C_E_PUSHED : C_I_PUSHED], (unsigned long long)n_push);
    if (ntiles == 0) {
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
  }

  const uint32_t step = a.step;
  const double inv_dx = a.inv_dx;
  const double L = a.L;

  // The ticket is fetched by one thread in the middle of the loop body, never
  // at the loop header: with a divergent region at the header the compiler
  // may rotate the loop so that only the fetching lane goes round through the
  // fetch while the others re-enter at the barrier and re-read a stale tile.
#if PIC_TICKETS
  if (tid == 0) s_tile = (int)atomicAdd(&ctl->ticket[SP], 1u);
  __syncthreads();
  int t = uniform32(s_tile);
#else
  int t = (int)blockIdx.x;
#endif
  while (t < ntiles) {
    const int64_t base = (int64_t)t * kTile;
#if PIC_TICKETS
    // the next ticket is requested now; its latency hides behind this tile
    uint32_t next_ticket = 0;
    if (tid == 0) next_ticket = atomicAdd(&ctl->ticket[SP], 1u);
#endif

    // ---------------- phase A: push, wall, collision decision -------------
    double px[kPPT], pvx[kPPT], pvy[kPPT], pvz[kPPT];
    uint32_t code[kPPT], cnt[kPPT];
    int jlo = INT_MAX, jhi = -1;
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
      const int64_t slot = base + k * kBlock + tid;
      uint32_t c = 0, o = 0, b = 0;
      double x = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
      if (slot < n_tot) {
        x = a.xin[slot];
        vx = a.vxin[slot];
        vy = a.vyin[slot];
        vz = a.vzin[slot];
        if (slot >= n_push) {
          c = kPass;  // born earlier this step: carried, not pushed
          o = 1;
        } else {
          c = kCodePushed;
          int j;
          double f;
          int64_t w1;
          cell_of(x, inv_dx, nx, j, f, w1);
          if (MEASURE) {
            const double eps = a.ek * (vx * vx + vy * vy + vz * vz);
            atomicAdd(&sEW[j], ((double)(kOne32 - w1) * kInvTwo32) * eps);
            atomicAdd(&sEW[j + 1], ((double)w1 * kInvTwo32) * eps);
            jlo = min(jlo, j);
            jhi = max(jhi, j + 1);
            if (fabs(x - a.half) <= a.eepf_hw) {
              const int64_t bin = (int64_t)(eps * a.inv_de);
              if (bin >= 0 && bin < a.nbins) atomicAdd(&sEEPF[bin], 1u);
            }
          }
          // gather (linear interpolation) and leap-frog push
          const double Ep = (1.0 - f) * sE[j] + f * sE[j + 1];
          vx = vx + a.acc * Ep;
          x = x + vx * a.dts;
          const uint4 r0 = draw(step, (uint32_t)slot, SP, 0, a.seed, a.run);
          bool alive = true;
          if (!isfinite(x) || !isfinite(vx)) {
            latch_error(ctl, kErrUnstable);
            alive = false;
            c |= 1u;
          } else if (x < 0.0 || x > L) {
            const double ub = u01(r0.x);
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
                c |= 3u;
                b = 1;
                atomicAdd(&s_cnt[C_SE_EMITTED], 1ull);
              } else {
                c |= 1u;
              }
            }
          }
          if (alive && !a.no_coll && u01(r0.y) < a.pcoll) {
            if (SP == 0) {
              // electron candidate: the process at this speed (it decides
              // whether a second electron and an ion are born)
              atomicAdd(&s_cnt[C_E_CAND], 1ull);
              const double g = sqrt(vx * vx + vy * vy + vz * vz);
              const double tv = g * a.inv_dv;
              const double r = u01(r0.z) * a.numax;
              const double* c0 = a.cum;
              const double* c1 = a.cum + a.ntab;
              const double* c2 = a.cum + 2 * a.ntab;
              int kk = a.ntab - 1;
              double tt = 0.0;
              const bool inside = tv < (double)(a.ntab - 1);
              double nu0, nu1;
              if (inside) {
                kk = (int)tv;
                tt = tv - (double)kk;
                nu0 = (1.0 - tt) * c0[kk] + tt * c0[kk + 1];
                nu1 = (1.0 - tt) * c1[kk] + tt * c1[kk + 1];
              } else {
                // beyond the last table speed: its entry (still <= nu_max)
                atomicAdd(&s_cnt[C_BEYOND_TABLE], 1ull);
                nu0 = c0[kk];
                nu1 = c1[kk];
              }
              uint32_t proc = 1;
              if (r < nu0) {
                proc = 2;
                atomicAdd(&s_cnt[C_E_ELASTIC], 1ull);
              } else if (r < nu1) {
                proc = 3;
                atomicAdd(&s_cnt[C_E_EXC], 1ull);
              } else {
                const double nu2 = inside ? (1.0 - tt) * c2[kk] + tt * c2[kk + 1] : c2[kk];
                if (r < nu2) {
                  proc = 4;
                  b = 1;
                  atomicAdd(&s_cnt[C_E_ION], 1ull);
                }
              }
              c |= proc << 3;
            } else {
              // ion candidate: the process needs a thermal atom velocity and
              // does not change the number of outputs; chosen in the rare pass
              atomicAdd(&s_cnt[C_I_CAND], 1ull);
              c |= kIonCand;
            }
          }
          if (alive) {
            c |= kAlive;
            o = 1 + ((SP == 0 && ((c >> 3) & 7u) == 4u) ? 1 : 0);
          }
          if (a.record && !(SP == 1 && (c & kIonCand))) a.codes[slot] = (uint8_t)(c & 0xFFu);
        }
      }
      px[k] = x;
      pvx[k] = vx;
      pvy[k] = vy;
      pvz[k] = vz;
      code[k] = c;
      cnt[k] = o | (b << 16);
    }

    // ---------------- phase B: tile scan and decoupled look-back ----------
    uint32_t loc[kPPT];
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
      const uint32_t inc = wave_incl_scan<unsigned int>(cnt[k]);
      loc[k] = inc - cnt[k];
      if (lane == kWave - 1) s_wtot[k][wave] = inc;
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t run = 0;
      for (int k = 0; k < kPPT; ++k)
        for (int w = 0; w < kBlock / kWave; ++w) {
          s_woff[k][w] = run;
          run += s_wtot[k][w];
        }
      s_agg[0] = run & 0xFFFFu;
      s_agg[1] = run >> 16;
    }
    __syncthreads();
    if (tid < 2) {
      // lane 0: own outputs, lane 1: births of the other species
      const uint32_t agg = s_agg[tid];
      uint64_t* st = a.tstat + 2 * (int64_t)t + tid;
      uint64_t pre = 0;
      if (t == 0) {
        st_agent(st, pack_status(a.epoch, 2, agg));
      } else {
        st_agent(st, pack_status(a.epoch, 1, agg));
        pre = look_back(a.tstat, t, tid, a.epoch, ctl);
        st_agent(st, pack_status(a.epoch, 2, (uint32_t)(pre + agg)));
      }
      s_pref[tid] = pre;
    }
    __syncthreads();
    const int64_t prefO = (int64_t)s_pref[0];
    const int64_t prefB = (int64_t)s_pref[1];
    if (tid == 0 && t == ntiles - 1) {
      const int64_t totO = prefO + (int64_t)s_agg[0], totB = prefB + (int64_t)s_agg[1];
      if (SP == 0) {
        ctl->e_out = totO;
        ctl->n_e[par ^ 1] = totO;
        ctl->i_births = totB;
        ctl->n_i[par ^ 1] = bbase + totB;
      } else {
        ctl->n_i[par ^ 1] = totO;
        ctl->n_e[par ^ 1] = bbase + totB;
      }
      if (totO > a.cap || bbase + totB > a.bcap) latch_error(ctl, kErrCapacity);
    }

    // ---------------- phase C: write and deposit ----------------------------
    bool any_rare = false;
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
      const uint32_t c = code[k];
      if (is_rare<SP>(c)) {
        any_rare = true;
        continue;
      }
      if (!((c & kAlive) || (c & kPass))) continue;
      const int64_t dest = prefO + (int64_t)((s_woff[k][wave] + loc[k]) & 0xFFFFu);
      if (dest < a.cap) store4(a, dest, px[k], pvx[k], pvy[k], pvz[k]);
      deposit_lds(sH, px[k], inv_dx, nx, 1ull, jlo, jhi);
    }
    if (any_rare) {
#pragma unroll
      for (int k = 0; k < kPPT; ++k) {
        if (!is_rare<SP>(code[k])) continue;
        const uint32_t off = s_woff[k][wave] + loc[k];
        rare_particle<SP>(a, sH, s_cnt, base + k * kBlock + tid, code[k], px[k], pvx[k], pvy[k],
                          pvz[k], prefO + (int64_t)(off & 0xFFFFu),
                          bbase + prefB + (int64_t)(off >> 16), jlo, jhi);
      }
    }

    // ---------------- flush the touched deposit range ----------------------
    jlo = wave_min(jlo);
    jhi = wave_max(jhi);
    if (lane == 0) {
      atomicMin(&s_lo, jlo);
      atomicMax(&s_hi, jhi);
    }
    __syncthreads();
    const int lo = s_lo, hi = s_hi;  // lo > hi when the tile deposited nothing
    for (int j = (lo <= hi ? lo : hi + 1) + tid; j <= hi; j += kBlock) {
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
    __syncthreads();  // every thread has read s_lo/s_hi
    if (tid == 0) {
#if PIC_TICKETS
      s_tile = (int)next_ticket;
#endif
      s_lo = INT_MAX;
      s_hi = -1;
    }
    __syncthreads();
#if PIC_TICKETS
    t = uniform32(s_tile);
#else
    t += (int)gridDim.x;
#endif
  }

  if (tid < NCOUNTERS && s_cnt[tid]) atomicAdd(&ctl->counters[tid], s_cnt[tid]);
  if (MEASURE) {
    for (int b = tid; b < a.nbins; b += kBlock)
      if (sEEPF[b]) atomicAdd(&a.eepf[b], (unsigned long long)sEEPF[b]);
  }
}

size_t particle_lds_bytes(int nx, bool measure, int nbins) {
  size_t b = (size_t)nx * 16;
  if (measure) b += (size_t)nx * 8 + (size_t)nbins * 4;
  return b;
}

int particle_blocks_per_cu(int species, bool measure, size_t lds) {
  int nb = 0;
  hipError_t e;
  if (species == 0)
    e = measure ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particle<0, true>, kBlock, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particle<0, false>, kBlock, lds);
  else
    e = measure ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particle<1, true>, kBlock, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particle<1, false>, kBlock, lds);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

template <typename K>
static hipError_t launch_one(K kern, int grid, size_t lds, const PartArgs& a, hipStream_t s) {
#if PIC_COOP
  void* args[] = {const_cast<PartArgs*>(&a)};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(kBlock),
                                    args, (unsigned)lds, s);
#else
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, a);
  return hipGetLastError();
#endif
}

hipError_t launch_particles(int species, bool measure, const PartArgs& a, int grid, size_t lds,
                            hipStream_t s) {
  if (species == 0)
    return measure ? launch_one(k_particle<0, true>, grid, lds, a, s)
                   : launch_one(k_particle<0, false>, grid, lds, a, s);
  return launch_one(k_particle<1, false>, grid, lds, a, s);
}

}  // namespace pic
