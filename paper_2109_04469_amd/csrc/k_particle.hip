// Particle kernel: one pass over a species' SoA streams per step, fusing
// field gather, leap-frog push, the wall model and null-collision MCC with
// order-preserving compaction, inline births and the CIC deposit of the new
// positions (arXiv:2109.04469, Sec. 2 steps 3-6 and step 1 of the next step).
//
// Schedule. A persistent grid (a few workgroups per CU) takes tiles of
// kTile = 1024 consecutive slots from an atomic ticket, so tiles are started
// in slot order. Per tile:
//   A  each thread loads 4 particles (4 coalesced 8-byte streams x 4), pushes
//      them, applies the wall and picks the collision process; only the
//      decision and the pushed state stay in registers;
//   B  a block scan of the per-particle output counts (0, 1 or 2 slots for
//      the own species, 0 or 1 birth of the other species) and a decoupled
//      look-back over earlier tiles give every output its global slot;
//   C  post-collision velocities are computed (their extra Philox blocks are
//      drawn only here, for the few colliding particles), outputs are written
//      and the new positions deposited into an LDS histogram in 2^-32 fixed
//      point; the touched node range is added to the global deposit with
//      integer atomics (a few nodes per tile once particles are cell-sorted)
//      and cleared.
// Survivors keep their relative order and an ionization electron follows its
// parent; births of the other species (Ar+ from ionization, secondary
// electrons from ion impact) are appended after that species' particles in
// parent-slot order.
#include <climits>

#include "pic_internal.h"

namespace pic {

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t value) {
  return ((uint64_t)(epoch & 0x3FFFFFFFu) << 34) | ((uint64_t)flag << 32) | (uint64_t)value;
}

// Exclusive prefix of value `which` (0: own outputs, 1: births) over tiles
// [0, t), from the status words of the earlier tiles.
// The wait on a predecessor is bounded: a tile is published by the
// workgroup that took its ticket, which is already running, so the bound is
// never reached in a correct run; if it were, the error is latched and the
// kernel still ends.
constexpr uint32_t kMaxSpin = 1u << 22;

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

template <int SP, bool MEASURE>
__global__ __launch_bounds__(kBlock) void k_particle(PartArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx;
  double* sE = reinterpret_cast<double*>(smem);
  unsigned long long* sH = reinterpret_cast<unsigned long long*>(sE + nx);
  double* sEW = reinterpret_cast<double*>(sH + nx);                 // MEASURE
  unsigned int* sEEPF = reinterpret_cast<unsigned int*>(sEW + nx);  // MEASURE

  __shared__ uint32_t s_wtot[kPPT][kBlock / kWave];
  __shared__ uint32_t s_total;
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
  __syncthreads();

  const uint32_t step = a.step;
  const double inv_dx = a.inv_dx;
  const double L = a.L;

  // The ticket is fetched by one thread in the middle of the loop body, never
  // at the loop header: with a divergent region at the header the compiler
  // may rotate the loop so that only the fetching lane goes round through the
  // fetch while the others re-enter at the barrier and re-read a stale tile.
  if (tid == 0) s_tile = (int)atomicAdd(&ctl->ticket[SP], 1u);
  __syncthreads();
  int t = uniform32(s_tile);
  while (t < ntiles) {
    const int64_t base = (int64_t)t * kTile;

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
            // null-collision candidate: choose the process at this speed
            double g;
            if (SP == 0) {
              atomicAdd(&s_cnt[C_E_CAND], 1ull);
              g = sqrt(vx * vx + vy * vy + vz * vz);
            } else {
              atomicAdd(&s_cnt[C_I_CAND], 1ull);
              const uint4 r1 = draw(step, (uint32_t)slot, 1, 1, a.seed, a.run);
              double n1, n2, n3, dmy;
              box_muller(u01(r1.x), u01(r1.y), n1, n2);
              box_muller(u01(r1.z), u01(r1.w), n3, dmy);
              const double gx = vx - a.sig_g * n1;
              const double gy = vy - a.sig_g * n2;
              const double gz = vz - a.sig_g * n3;
              g = sqrt(gx * gx + gy * gy + gz * gz);
            }
            // cumulative frequencies interpolated in speed; beyond the last
            // table speed the last entry is used (still <= nu_max) and the
            // event is counted
            const double tv = g * a.inv_dv;
            uint32_t proc = 1;
            const double r = u01(r0.z) * a.numax;
            const double* c0 = a.cum;
            const double* c1 = a.cum + a.ntab;
            const double* c2 = a.cum + 2 * a.ntab;
            double nu0, nu1;
            int kk = a.ntab - 1;
            double tt = 0.0;
            const bool inside = tv < (double)(a.ntab - 1);
            if (inside) {
              kk = (int)tv;
              tt = tv - (double)kk;
              nu0 = (1.0 - tt) * c0[kk] + tt * c0[kk + 1];
              nu1 = (1.0 - tt) * c1[kk] + tt * c1[kk + 1];
            } else {
              atomicAdd(&s_cnt[C_BEYOND_TABLE], 1ull);
              nu0 = c0[kk];
              nu1 = c1[kk];
            }
            if (r < nu0) {
              proc = 2;
            } else if (r < nu1) {
              proc = 3;
            } else if (SP == 0) {
              const double nu2 = inside ? (1.0 - tt) * c2[kk] + tt * c2[kk + 1] : c2[kk];
              if (r < nu2) proc = 4;
            }
            c |= proc << 3;
            if (SP == 0) {
              if (proc == 2) atomicAdd(&s_cnt[C_E_ELASTIC], 1ull);
              if (proc == 3) atomicAdd(&s_cnt[C_E_EXC], 1ull);
              if (proc == 4) {
                atomicAdd(&s_cnt[C_E_ION], 1ull);
                b = 1;
              }
            } else {
              if (proc == 2) atomicAdd(&s_cnt[C_I_ISO], 1ull);
              if (proc == 3) atomicAdd(&s_cnt[C_I_BACK], 1ull);
            }
          }
          if (alive) {
            c |= kAlive;
            o = 1 + ((SP == 0 && ((c >> 3) & 7u) == 4u) ? 1 : 0);
          }
          if (a.record) a.codes[slot] = (uint8_t)(c & 0xFFu);
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
          const uint32_t v = s_wtot[k][w];
          s_wtot[k][w] = run;
          run += v;
        }
      s_total = run;
      const uint32_t aggO = run & 0xFFFFu, aggB = run >> 16;
      uint64_t* st = a.tstat + 2 * (int64_t)t;
      uint64_t pO = 0, pB = 0;
      if (t == 0) {
        st_agent(st, pack_status(a.epoch, 2, aggO));
        st_agent(st + 1, pack_status(a.epoch, 2, aggB));
      } else {
        st_agent(st, pack_status(a.epoch, 1, aggO));
        st_agent(st + 1, pack_status(a.epoch, 1, aggB));
        pO = look_back(a.tstat, t, 0, a.epoch, ctl);
        pB = look_back(a.tstat, t, 1, a.epoch, ctl);
        st_agent(st, pack_status(a.epoch, 2, (uint32_t)(pO + aggO)));
        st_agent(st + 1, pack_status(a.epoch, 2, (uint32_t)(pB + aggB)));
      }
      s_pref[0] = pO;
      s_pref[1] = pB;
      if (t == ntiles - 1) {
        const int64_t totO = (int64_t)(pO + aggO), totB = (int64_t)(pB + aggB);
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
    }
    __syncthreads();
    const int64_t prefO = (int64_t)s_pref[0];
    const int64_t prefB = (int64_t)s_pref[1];

    // ---------------- phase C: scatter, write, deposit --------------------
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
      if (cnt[k] == 0) continue;
      const uint32_t off = s_wtot[k][wave] + loc[k];
      const int64_t dest = prefO + (int64_t)(off & 0xFFFFu);
      const int64_t bdest = bbase + prefB + (int64_t)(off >> 16);
      const int64_t slot = base + k * kBlock + tid;
      const uint32_t c = code[k];
      double x = px[k], vx = pvx[k], vy = pvy[k], vz = pvz[k];
      const uint32_t proc = (c >> 3) & 7u;
      bool child = false;
      double cvx = 0, cvy = 0, cvz = 0;
      bool birth = false;
      double bxp = 0, bvx = 0, bvy = 0, bvz = 0;
      if (!(c & kPass) && (c & kAlive) && proc >= 2) {
        if (SP == 0) {
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
            double eps = a.ek * v2 - a.exc_thr;
            if (eps < 0.0) eps = 0.0;
            const double s1 = sqrt(eps * a.ve);
            double nx_, ny_, nz_;
            iso_dir(u01(r1.x), u01(r1.y), nx_, ny_, nz_);
            vx = s1 * nx_;
            vy = s1 * ny_;
            vz = s1 * nz_;
          } else {
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
        } else {
          const uint4 r1 = draw(step, (uint32_t)slot, 1, 1, a.seed, a.run);
          double n1, n2, n3, dmy;
          box_muller(u01(r1.x), u01(r1.y), n1, n2);
          box_muller(u01(r1.z), u01(r1.w), n3, dmy);
          const double ax = a.sig_g * n1, ay = a.sig_g * n2, az = a.sig_g * n3;
          if (proc == 2) {
            const double gx = vx - ax, gy = vy - ay, gz = vz - az;
            const double g = sqrt(gx * gx + gy * gy + gz * gz);
            const uint4 r2 = draw(step, (uint32_t)slot, 1, 2, a.seed, a.run);
            double ux, uy, uz;
            iso_dir(u01(r2.x), u01(r2.y), ux, uy, uz);
            const double hg = 0.5 * g;
            vx = 0.5 * (vx + ax) + hg * ux;
            vy = 0.5 * (vy + ay) + hg * uy;
            vz = 0.5 * (vz + az) + hg * uz;
          } else if (proc == 3) {
            vx = ax;
            vy = ay;
            vz = az;
          }
        }
      }
      if (SP == 1 && !(c & kAlive) && (c & 7u) == 3u) {
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
      if ((c & kAlive) || (c & kPass)) {
        if (dest < a.cap) {
          a.xout[dest] = x;
          a.vxout[dest] = vx;
          a.vyout[dest] = vy;
          a.vzout[dest] = vz;
        }
        int j;
        double f;
        int64_t w1;
        cell_of(x, inv_dx, nx, j, f, w1);
        const unsigned long long mul = child ? 2ull : 1ull;
        atomicAdd(&sH[j], mul * (unsigned long long)(kOne32 - w1));
        atomicAdd(&sH[j + 1], mul * (unsigned long long)w1);
        jlo = min(jlo, j);
        jhi = max(jhi, j + 1);
        if (child && dest + 1 < a.cap) {
          a.xout[dest + 1] = x;
          a.vxout[dest + 1] = cvx;
          a.vyout[dest + 1] = cvy;
          a.vzout[dest + 1] = cvz;
        }
      }
      if (birth) {
        if (bdest < a.bcap) {
          a.bx[bdest] = bxp;
          a.bvx[bdest] = bvx;
          a.bvy[bdest] = bvy;
          a.bvz[bdest] = bvz;
        }
        int j;
        double f;
        int64_t w1;
        cell_of(bxp, inv_dx, nx, j, f, w1);
        atomicAdd(&a.dep_other[j], (unsigned long long)(kOne32 - w1));
        atomicAdd(&a.dep_other[j + 1], (unsigned long long)w1);
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
      s_tile = (int)atomicAdd(&ctl->ticket[SP], 1u);
      s_lo = INT_MAX;
      s_hi = -1;
    }
    __syncthreads();
    t = uniform32(s_tile);
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

hipError_t launch_particles(int species, bool measure, const PartArgs& a, int grid, size_t lds,
                            hipStream_t s) {
  if (species == 0) {
    if (measure)
      hipLaunchKernelGGL((k_particle<0, true>), dim3(grid), dim3(kBlock), lds, s, a);
    else
      hipLaunchKernelGGL((k_particle<0, false>), dim3(grid), dim3(kBlock), lds, s, a);
  } else {
    hipLaunchKernelGGL((k_particle<1, false>), dim3(grid), dim3(kBlock), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace pic
