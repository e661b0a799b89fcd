// libpic C ABI: parameter validation, derived constants, workspace layout
// and the per-step launch schedule. Host code only; every step of the method
// runs in the kernels of k_field / k_particle / k_sort.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/warmstart.h"
#include "pic_internal.h"

using namespace pic;

struct pic_batch {
  std::vector<pic_handle*> hs;
  hipStream_t stream;
  BatchLaunch launch;
  bool variants;      // some discharge uses a method variant
  int chunk;          // steps per upload of argument blocks
  size_t step_bytes;  // argument bytes of one step (worst case)
  unsigned char* dev[2];
  unsigned char* host[2];
  hipEvent_t copied[2];
  int slot;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxCells = 4096;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Velocity-pool entries per buffer: the live particles plus the entries of
// particles absorbed and born since the last repack (every sort, or every
// kRepackSteps steps when sorts are rarer). Running out latches
// PIC_ECAPACITY.
constexpr int kRepackSteps = 256;
int64_t pool_capacity(int64_t cap) { return cap + (cap / 2 > 4096 ? cap / 2 : 4096); }

// Upper edge of the ion arrival-energy bins: ions gain at most about the
// peak sheath voltage, so 1.25 phi_0 (at least 10 eV).
double fedf_ion_emax(double rf_voltage_v) {
  const double e = 1.25 * rf_voltage_v;
  return e > 10.0 ? e : 10.0;
}

struct Layout {
  size_t ctl, part[2][2][2], pid[2][2], pool[2][2][2], codes[2][2], tcnt[2][2], rq[2], dep_e[2], dep_i[2], rho, phi, E[2], cum[2], th_cp,
      th_m, acc_ne, acc_ni, acc_w, acc_ew, eepf, fedf[2], sort_cnt, sort_seg, cand, dq, total;
  int64_t max_tiles[2];
  int sort_blocks;
};

int validate(const pic_params* p, const pic_xsec* xs) {
  if (!p || !xs) return PIC_EINVAL;
  if (!(p->gap_m > 0) || !(p->rf_freq_hz > 0) || p->steps_per_cycle < 1) return PIC_EINVAL;
  if (p->n_cells < 2 || p->n_cells > kMaxCells) return PIC_EINVAL;
  if (!(p->weight > 0) || !(p->area_m2 > 0) || !(p->gas_temp_k > 0) || !(p->pressure_pa >= 0))
    return PIC_EINVAL;
  if (!(p->reflection >= 0 && p->reflection <= 1) || !(p->gamma_see >= 0 && p->gamma_see <= 1))
    return PIC_EINVAL;
  if (!(p->see_temp_ev >= 0)) return PIC_EINVAL;
  for (int s = 0; s < 2; ++s)
    if (p->capacity[s] < 0 || p->capacity[s] > ((int64_t)1 << 31) - kTile) return PIC_EINVAL;
  if (p->ion_subcycle < 1 || p->sort_interval < 0) return PIC_EINVAL;
  if (p->eepf_bins < 1 || p->eepf_bins > 4096 || !(p->eepf_emax_ev > 0) ||
      !(p->eepf_halfwidth_m >= 0))
    return PIC_EINVAL;
  if (xs->n < 2 || !(xs->dv_e > 0) || !(xs->dv_i > 0)) return PIC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!xs->sigma_e[k]) return PIC_EINVAL;
  for (int k = 0; k < 2; ++k)
    if (!xs->sigma_i[k]) return PIC_EINVAL;
  if (!(xs->exc_threshold_ev >= 0) || !(xs->ion_threshold_ev >= 0)) return PIC_EINVAL;
  const uint32_t known = PIC_FLAG_NO_FIELD | PIC_FLAG_FIXED_E | PIC_FLAG_NO_COLL |
                         PIC_FLAG_IMMOBILE_IONS | PIC_FLAG_RECORD | PIC_FLAG_THOMAS |
                         PIC_FLAG_ANISO_ELASTIC | PIC_FLAG_OPAL_SHARING;
  if (p->flags & ~known) return PIC_EINVAL;
  return PIC_OK;
}

Layout make_layout(const pic_params* p, const pic_xsec* xs) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes > 0 ? bytes : 1);
    return o;
  };
  const int nx = p->n_cells + 1;
  L.ctl = take(sizeof(DevCtl));
  for (int s = 0; s < 2; ++s) {
    const int64_t cap = p->capacity[s];
    L.max_tiles[s] = (cap + kTile - 1) / kTile + 1;
    for (int b = 0; b < 2; ++b) {
      for (int q = 0; q < 2; ++q) L.part[s][b][q] = take((size_t)cap * sizeof(double));
      L.pid[s][b] = take((size_t)cap * sizeof(uint32_t));
      for (int q = 0; q < 2; ++q) L.pool[s][b][q] = take((size_t)pool_capacity(cap) * 8);
    }
    for (int b = 0; b < 2; ++b) L.codes[s][b] = take((size_t)cap);
    for (int b = 0; b < 2; ++b) L.tcnt[s][b] = take((size_t)L.max_tiles[s] * sizeof(uint64_t));
    L.rq[s] = take((size_t)cap * 16);
  }
  for (int b = 0; b < 2; ++b) L.dep_e[b] = take((size_t)nx * 8);
  for (int b = 0; b < 2; ++b) L.dep_i[b] = take((size_t)nx * 8);
  L.rho = take((size_t)nx * 8);
  L.phi = take((size_t)nx * 8);
  for (int b = 0; b < 2; ++b) L.E[b] = take((size_t)nx * 8);
  L.cum[0] = take((size_t)3 * xs->n * 8);
  L.cum[1] = take((size_t)2 * xs->n * 8);
  L.th_cp = take((size_t)nx * 8);
  L.th_m = take((size_t)nx * 8);
  L.acc_ne = take((size_t)nx * 8);
  L.acc_ni = take((size_t)nx * 8);
  L.acc_w = take((size_t)nx * 8);
  L.acc_ew = take((size_t)nx * 8);
  L.eepf = take((size_t)p->eepf_bins * 8);
  for (int sp = 0; sp < 2; ++sp) L.fedf[sp] = take((size_t)2 * p->eepf_bins * 8);
  int64_t capmax = p->capacity[0] > p->capacity[1] ? p->capacity[0] : p->capacity[1];
  int sb = (int)((capmax + 16383) / 16384);
  if (sb < 1) sb = 1;
  if (sb > 512) sb = 512;
  L.sort_blocks = sb;
  L.sort_cnt = take((size_t)sb * (size_t)(nx - 1) * sizeof(uint32_t));
  L.sort_seg = take(256 * sizeof(uint32_t));
  // candidacy bits of the electron slots of a pipelined step
  L.cand = take((size_t)((p->capacity[0] + 31) / 32 + 1) * sizeof(uint32_t));
  L.dq = take((size_t)p->capacity[0] * sizeof(uint32_t));
  L.total = off;
  return L;
}

// u01(r) = (r + 1/2) 2^-32 is exact in FP64, so u01(r) < p holds exactly
// when r + 1/2 < P = p 2^32 (scaling by a power of two is exact), i.e. for
// integers r < ceil(P - 1/2); P - 1/2 is exact for P < 2^32.
uint64_t candidacy_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  const double t = std::ceil(std::ldexp(p, 32) - 0.5);
  return t <= 0.0 ? 0 : (uint64_t)t;
}

int hip_status(hipError_t e) { return e == hipSuccess ? PIC_OK : PIC_EHIP; }

#define HIP_TRY(expr)                        \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return PIC_EHIP;   \
  } while (0)

// Starts a timed launch: returns the event index or -1 when timing is off.
int timer_begin(pic_handle* h) {
  if (!h->timing) return -1;
  const size_t need = 2 * (h->ev_next + 1);
  while (h->ev_pool.size() < need) {
    hipEvent_t e;
    // timing-only events: no system-scope fence (no cache writeback) on record
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
    h->ev_pool.push_back(e);
  }
  const int idx = (int)(2 * h->ev_next);
  if (hipEventRecord(h->ev_pool[idx], h->stream) != hipSuccess) return -1;
  h->ev_next += 1;
  return idx;
}

void timer_end(pic_handle* h, int timer, int idx) {
  if (idx < 0) return;
  if (hipEventRecord(h->ev_pool[idx + 1], h->stream) == hipSuccess)
    h->ev_used.emplace_back(timer, idx);
}

// Folds the recorded event pairs into the per-timer sums (synchronises).
int timer_collect(pic_handle* h) {
  if (h->ev_used.empty()) {
    h->ev_next = 0;
    return PIC_OK;
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_EHIP;
  for (const auto& u : h->ev_used) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev_pool[u.second], h->ev_pool[u.second + 1]) != hipSuccess)
      return PIC_EHIP;
    h->t_ms[u.first] += ms;
    h->t_n[u.first] += 1;
  }
  h->ev_used.clear();
  h->ev_next = 0;
  return PIC_OK;
}

int latched(pic_handle* h) {
  uint32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, &h->ctl->err, sizeof(err), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (err & kErrUnstable) return PIC_EUNSTABLE;
  if (err & kErrCapacity) return PIC_ECAPACITY;
  return PIC_OK;
}

int field_mode(const pic_handle* h) {
  const uint32_t f = h->p.flags;
  if (f & PIC_FLAG_NO_FIELD) return FIELD_ZERO;
  if (f & PIC_FLAG_FIXED_E) return FIELD_FIXED;
  if (f & PIC_FLAG_THOMAS) return FIELD_THOMAS;
  return FIELD_EXACT;
}

PartArgs particle_args(pic_handle* h, int sp, int parity) {
  PartArgs a{};
  const int in = h->cur[sp], out = 1 - h->cur[sp];
  a.xin = h->part[sp][in][0];
  a.vxin = h->part[sp][in][1];
  a.idin = h->pid[sp][in];
  a.xout = h->part[sp][out][0];
  a.vxout = h->part[sp][out][1];
  a.idout = h->pid[sp][out];
  a.pvy = h->pool[sp][h->pcur[sp]][0];
  a.pvz = h->pool[sp][h->pcur[sp]][1];
  a.pcap = h->pcap[sp];
  const int other = 1 - sp;
  // electrons append ions to the current ion buffer; ions append secondary
  // electrons to the electron buffer the electron kernel has just written
  const int ob = h->cur[other];
  a.bx = h->part[other][ob][0];
  a.bvx = h->part[other][ob][1];
  a.bid = h->pid[other][ob];
  a.bpvy = h->pool[other][h->pcur[other]][0];
  a.bpvz = h->pool[other][h->pcur[other]][1];
  a.bpcap = h->pcap[other];
  a.E = h->Ebuf[parity];
  if (sp == 0) {
    a.dep_own = reinterpret_cast<unsigned long long*>(h->dep_e[parity ^ 1]);
    a.dep_other = reinterpret_cast<unsigned long long*>(h->dep_i[h->cur_hi]);
  } else {
    a.dep_own = reinterpret_cast<unsigned long long*>(h->dep_i[1 - h->cur_hi]);
    a.dep_other = reinterpret_cast<unsigned long long*>(h->dep_e[parity ^ 1]);
  }
  a.cum = h->cum[sp];
  a.ctl = h->ctl;
  // tile totals are summed with atomics into a buffer the previous pass of
  // this species zeroed; this pass zeroes the other one
  a.tcnt = h->tcnt[sp][h->tsel[sp]];
  a.tcnt_next = h->tcnt[sp][h->tsel[sp] ^ 1];
  a.rq = h->rq[sp];
  // decision codes of alternate passes in alternate buffers: a pass fused
  // with the next step's decisions reads one and writes the other
  a.codes = h->codes[sp][h->csel[sp]];
  a.cand = sp == 0 ? h->cand : nullptr;
  a.dq = sp == 0 ? h->dq : nullptr;
  a.acc_ew = h->acc_ew;
  a.eepf = h->eepf;
  a.fedf = h->fedf[sp];
  a.ek_s = 0.5 * h->mass[sp] / kQe;
  a.fedf_inv_de = (double)h->p.eepf_bins / h->fedf_emax[sp];
  a.measure_walls = h->measuring;
  a.cap = h->p.capacity[sp];
  a.bcap = h->p.capacity[other];
  a.max_tiles = h->max_tiles[sp];
  a.inv_dx = h->inv_dx;
  a.L = h->L;
  a.acc = h->acc[sp];
  a.dts = h->dts[sp];
  a.p_wall = sp == 0 ? h->p.reflection : h->p.gamma_see;
  a.pcoll = h->pcoll[sp];
  a.pcoll_thr = candidacy_threshold(h->pcoll[sp]);
  a.numax = h->numax[sp];
  a.inv_dv = h->inv_dv[sp];
  a.mr = h->mr_e;
  a.mm = h->mm_e;
  a.ek = h->ek_e;
  a.ve = h->ve_e;
  a.exc_thr = h->exc_thr;
  a.ion_thr = h->ion_thr;
  a.sig_g = h->sig_g;
  a.sig_se = h->sig_se;
  a.half = 0.5 * h->L;
  a.eepf_hw = h->p.eepf_halfwidth_m;
  a.inv_de = h->inv_de;
  a.nx = h->nx;
  a.ntab = h->ntab;
  a.nbins = h->p.eepf_bins;
  a.parity = parity;
  a.step = (uint32_t)h->step;
  a.seed = h->p.seed;
  a.run = h->p.run;
  a.no_coll = (h->p.flags & PIC_FLAG_NO_COLL) ? 1 : 0;
  a.record = (h->p.flags & PIC_FLAG_RECORD) ? 1 : 0;
  a.model = ((h->p.flags & PIC_FLAG_ANISO_ELASTIC) ? kModelAniso : 0) |
            ((h->p.flags & PIC_FLAG_OPAL_SHARING) ? kModelOpal : 0);
  return a;
}

SortArgs sort_args(pic_handle* h, int sp, bool reorder) {
  SortArgs a{};
  const int in = h->cur[sp], out = reorder ? 1 - h->cur[sp] : h->cur[sp];
  const int pin = h->pcur[sp], pout = 1 - h->pcur[sp];
  a.sx = h->part[sp][in][0];
  a.svx = h->part[sp][in][1];
  a.sid = h->pid[sp][in];
  a.spvy = h->pool[sp][pin][0];
  a.spvz = h->pool[sp][pin][1];
  a.dx = h->part[sp][out][0];
  a.dvx = h->part[sp][out][1];
  a.did = h->pid[sp][out];
  a.dpvy = h->pool[sp][pout][0];
  a.dpvz = h->pool[sp][pout][1];
  a.pool_n = &h->ctl->pool_n[sp];
  a.count = sp == 0 ? &h->ctl->n_e[h->step & 1] : &h->ctl->n_i[h->step & 1];
  a.cap = h->p.capacity[sp];
  a.cnt = h->sort_cnt;
  a.seg = h->sort_seg;
  a.inv_dx = h->inv_dx;
  a.nx = h->nx;
  a.nblocks = h->sort_blocks;
  return a;
}

// Stable sort of one species by cell; the pool is rebuilt in the new slot
// order.
int sort_species(pic_handle* h, int sp) {
  const SortArgs a = sort_args(h, sp, true);
  const int ev = timer_begin(h);
  HIP_TRY(launch_sort(a, h->stream));
  timer_end(h, PIC_TIMER_SORT, ev);
  h->cur[sp] ^= 1;
  h->pcur[sp] ^= 1;
  return PIC_OK;
}

// Pool rebuilt in slot order, slots unchanged: drops the entries of
// absorbed particles.
int repack_species(pic_handle* h, int sp) {
  HIP_TRY(launch_repack(sort_args(h, sp, false), h->stream));
  h->pcur[sp] ^= 1;
  return PIC_OK;
}

FieldArgs field_args(pic_handle* h, int field_mode_, bool ion_step) {
  const int par = (int)(h->step & 1);
  FieldArgs f{};
  f.dep_e = h->dep_e[par];
  f.dep_i = h->dep_i[h->cur_hi];
  f.zero_a = h->dep_e[par ^ 1];
  f.zero_b = ion_step ? h->dep_i[1 - h->cur_hi] : nullptr;
  f.rho = h->rho;
  f.phi = h->phi;
  f.E = h->Ebuf[par];
  f.th_cp = h->th_cp;
  f.th_m = h->th_m;
  f.acc_ne = h->acc_ne;
  f.acc_ni = h->acc_ni;
  f.acc_w = h->acc_w;
  f.ctl = h->ctl;
  f.V = h->vtab[(size_t)(h->step % h->p.steps_per_cycle)];
  f.dx = h->dx;
  f.qfac32 = h->qfac32;
  f.nfac32 = h->nfac32;
  f.kpois = h->kpois;
  f.nx = h->nx;
  f.mode = field_mode_;
  f.measuring = h->measuring;
  f.parity = par;
  return f;
}

bool is_ion_step(const pic_handle* h, int64_t step) {
  return !(h->p.flags & PIC_FLAG_IMMOBILE_IONS) && (step % h->p.ion_subcycle == 0);
}

constexpr int kTailRareBlocks = 128;

// What one step of one discharge launches, in order:
//   [field(n)]  e_decide e_emit  [e_rare i_decide i_emit on ion steps]
//   then either the tail (queued slots of the last pass + field(n+1)) when
//   another step follows, or the last pass's rare kernel alone;
//   then a sort or repack of each species when due.
//
// Electron steps are pipelined when enabled and the schedule allows: the
// emit of step n then also decides step n+1 (k_emit_decide, which also runs
// step n's queued slots), so step n+1 has no decide pass and step n no tail.
// That needs the field of step n+1 before the emit of step n, so it applies
// to steps that are not the last of a call, not ion steps (the ions' deposit
// enters that field), not followed by a sort or repack (slots move) and not
// measuring:
//   [field(n)] [e_decide(n)] field_cand(n+1) e_emit_decide(n)
// A step whose electrons were decided that way (e_pushed) runs e_emit and
// the electron queued slots on the pushed state.
struct StepPlan {
  bool field_first;  // solve this step's field before the passes
  FieldArgs ff;
  bool measure;
  PartArgs ae;
  bool e_pushed;  // the previous step decided this step's electrons
  bool fuse;      // this step's electron emit decides the next step
  PartArgs ae_next;
  bool ion;
  PartArgs ai;
  int pend_sp;  // species of the last pass, whose queued slots run last
  bool tail;    // the next step's field is solved with those slots
  FieldArgs fn; // the next step's field (with the tail, or before the fused emit)
  int post;     // 0: nothing, 1: sort, 2: repack (both species)
  SortArgs sa[2];
};

// Plans the next step of h and advances the host-side schedule state past
// it (buffer parities, step index). field_ready: this step's field was
// solved by the previous step's tail; last: no step follows in this call.
StepPlan plan_step(pic_handle* h, bool field_ready, bool last, bool allow_fuse) {
  StepPlan q{};
  const pic_params& p = h->p;
  const int mode = field_mode(h);
  const int par = (int)(h->step & 1);
  q.ion = is_ion_step(h, h->step);
  q.field_first = !field_ready;
  if (q.field_first) q.ff = field_args(h, mode, q.ion);
  h->e_last = par;
  q.measure = h->measuring != 0;
  q.e_pushed = h->e_decided != 0;
  h->e_decided = 0;
  q.ae = particle_args(h, 0, par);
  h->cur[0] ^= 1;
  h->tsel[0] ^= 1;
  h->csel[0] ^= 1;
  q.pend_sp = 0;
  if (q.ion) {
    // the ions take this step's ionization ions with their velocities
    q.ai = particle_args(h, 1, par);
    h->cur[1] ^= 1;
    h->tsel[1] ^= 1;
    h->csel[1] ^= 1;
    h->cur_hi ^= 1;
    q.pend_sp = 1;
  }
  h->step += 1;
  q.post = 0;
  if (p.sort_interval > 0 && h->step % p.sort_interval == 0) {
    // stable sort by cell; the pool is rebuilt in the new slot order
    q.post = 1;
  } else if ((p.sort_interval == 0 || p.sort_interval > kRepackSteps) &&
             h->step % kRepackSteps == 0) {
    // pool rebuilt in slot order: drops the entries of absorbed particles
    q.post = 2;
  }
  q.fuse = allow_fuse && !last && !q.ion && q.post == 0 && !q.measure;
  q.tail = !last && !q.fuse;
  if (!last) q.fn = field_args(h, mode, is_ion_step(h, h->step));
  if (q.fuse) {
    // the next step's electron arguments, as its own plan will make them
    q.ae_next = particle_args(h, 0, (int)(h->step & 1));
    h->e_decided = 1;
    // with the next step's field, the candidacy bits of its electron slots
    // (their count is the sum of this step's output totals)
    FieldArgs& f = q.fn;
    f.cand = h->cand;
    f.cand_tcnt = q.ae.tcnt;
    f.cand_count = &h->ctl->n_e[par];
    f.cand_zero = q.ae_next.tcnt;
    f.cand_zero_n = h->max_tiles[0];
    f.cand_cap = h->p.capacity[0];
    f.cand_thr = q.ae_next.no_coll ? 0ull : q.ae_next.pcoll_thr;
    f.cand_step = q.ae_next.step;
    f.seed = h->p.seed;
    f.run = h->p.run;
  }
  for (int sp = 0; sp < 2 && q.post; ++sp) {
    q.sa[sp] = sort_args(h, sp, q.post == 1);
    if (q.post == 1) h->cur[sp] ^= 1;
    h->pcur[sp] ^= 1;
  }
  return q;
}

int launch_post(pic_handle* h, const StepPlan& q, hipStream_t s) {
  for (int sp = 0; sp < 2; ++sp) {
    if (q.post == 1) {
      const int ev = timer_begin(h);
      HIP_TRY(launch_sort(q.sa[sp], s));
      timer_end(h, PIC_TIMER_SORT, ev);
    } else if (q.post == 2) {
      HIP_TRY(launch_repack(q.sa[sp], s));
    }
  }
  return PIC_OK;
}

// One planned step on the handle's own stream, with the opt-in timers.
int launch_step(pic_handle* h, const StepPlan& q) {
  hipStream_t s = h->stream;
  if (q.field_first) {
    const int ev = timer_begin(h);
    HIP_TRY(launch_field(q.ff, s));
    timer_end(h, PIC_TIMER_FIELD, ev);
  }
  const int e_pass = timer_begin(h);
  if (!q.e_pushed) {
    const int ev = h->timing >= 2 ? timer_begin(h) : -1;
    HIP_TRY(launch_particle_kernel(0, 0, q.measure, q.ae, h->launch[0], s));
    timer_end(h, PIC_TIMER_E_DECIDE, ev);
  }
  if (q.fuse) {
    int ev = h->timing >= 2 ? timer_begin(h) : -1;
    HIP_TRY(launch_field_cand(q.fn, h->num_cu, s));
    timer_end(h, PIC_TIMER_FIELD, ev);
    ev = h->timing >= 2 ? timer_begin(h) : -1;
    HIP_TRY(launch_emit_decide(q.ae, q.ae_next, h->launch[0], s, q.e_pushed));
    timer_end(h, PIC_TIMER_E_EMIT, ev);
    timer_end(h, PIC_TIMER_ELECTRON, e_pass);
    return launch_post(h, q, s);
  }
  const int pushed = q.e_pushed ? kLaunchPushed : 0;
  {
    const int ev = h->timing >= 2 ? timer_begin(h) : -1;
    HIP_TRY(launch_particle_kernel(1, 0, q.measure, q.ae, h->launch[0], s, pushed));
    timer_end(h, PIC_TIMER_E_EMIT, ev);
  }
  int pend_pass = e_pass;
  if (q.ion) {
    const int ev = h->timing >= 2 ? timer_begin(h) : -1;
    HIP_TRY(launch_particle_kernel(2, 0, q.measure, q.ae, h->launch[0], s, pushed));
    timer_end(h, PIC_TIMER_E_RARE, ev);
    timer_end(h, PIC_TIMER_ELECTRON, e_pass);
    const int i_pass = timer_begin(h);
    for (int k = 0; k < 2; ++k) {
      const int ev2 = h->timing >= 2 ? timer_begin(h) : -1;
      HIP_TRY(launch_particle_kernel(k, 1, false, q.ai, h->launch[1], s));
      timer_end(h, k == 0 ? PIC_TIMER_I_DECIDE : PIC_TIMER_I_EMIT, ev2);
    }
    pend_pass = i_pass;
  }
  const PartArgs& pend = q.pend_sp == 0 ? q.ae : q.ai;
  const int pend_pushed = q.pend_sp == 0 ? pushed : 0;
  const int ev = h->timing >= 2 ? timer_begin(h) : -1;
  if (q.tail)
    HIP_TRY(launch_tail(q.pend_sp, q.fn, pend, kTailRareBlocks, s, pend_pushed != 0));
  else
    HIP_TRY(launch_particle_kernel(2, q.pend_sp, q.measure, pend, h->launch[q.pend_sp], s,
                                   pend_pushed));
  timer_end(h, q.pend_sp == 0 ? PIC_TIMER_E_RARE : PIC_TIMER_I_RARE, ev);
  timer_end(h, q.pend_sp == 0 ? PIC_TIMER_ELECTRON : PIC_TIMER_ION, pend_pass);
  return launch_post(h, q, s);
}

// Batched stepping: per step, the argument blocks of every discharge's
// passes go to device memory (one upload per chunk of steps, double
// buffered through pinned host memory) and each pass is one launch for all.
constexpr size_t kBatchUploadBytes = (size_t)4 << 20;  // per chunk buffer
constexpr size_t kBatchArrayAlign = 64;

size_t batch_step_bytes(int n) {
  // field blocks: this step's (first step of a call) and the next step's;
  // particle blocks: electron passes, electron passes of ion steps (their
  // queued slots run before the ions), ion passes, and the electron passes
  // whose queued slots run in the tail
  // plus the sorts of both species due after the step
  const size_t f = (size_t)n * sizeof(FieldArgs);
  const size_t a = (size_t)n * sizeof(PartArgs);
  const size_t so = (size_t)n * sizeof(SortArgs);
  auto al = [](size_t v) { return (v + kBatchArrayAlign - 1) / kBatchArrayAlign * kBatchArrayAlign; };
  return 2 * al(f) + 4 * al(a) + 2 * al(so);
}

int batch_chunk_steps(int n) {
  const size_t per = batch_step_bytes(n);
  size_t c = kBatchUploadBytes / per;
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  return (int)c;
}

int check_batch_handles(pic_handle* const* hs, int n) {
  if (!hs || n < 1 || n > kMaxBatch) return PIC_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!hs[i]) return PIC_EINVAL;
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return PIC_EINVAL;
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return PIC_EINVAL;
  }
  return PIC_OK;
}

// Replaces the particles of one species: fill(dst, pool) writes n positions
// and x-velocities to the active slot buffers and n (v_y, v_z) to the active
// pool (entry i for slot i); then the counts, pool indices and the species'
// deposit are rebuilt and the event counters and error word cleared.
// Synchronises.
template <typename Fill>
int replace_state(pic_handle* h, int species, int64_t n, int64_t step, Fill fill) {
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->e_decided = 0;
  const int old_par = (int)(h->step & 1), par = (int)(step & 1);
  if (old_par != par) {
    // keep the other species' count and (for electrons) deposit on the new parity
    if (species == 1) {
      HIP_TRY(hipMemcpyAsync(&h->ctl->n_e[par], &h->ctl->n_e[old_par], 8,
                             hipMemcpyDeviceToDevice, h->stream));
      HIP_TRY(hipMemcpyAsync(h->dep_e[par], h->dep_e[old_par], (size_t)h->nx * 8,
                             hipMemcpyDeviceToDevice, h->stream));
    } else {
      HIP_TRY(hipMemcpyAsync(&h->ctl->n_i[par], &h->ctl->n_i[old_par], 8,
                             hipMemcpyDeviceToDevice, h->stream));
    }
  }
  h->step = step;
  double* const* dst = h->part[species][h->cur[species]];
  double* const* pool = h->pool[species][h->pcur[species]];
  if (n > 0) {
    const int st = fill(dst, pool);
    if (st) return st;
  }
  int64_t nn = n;
  int64_t* cnt = species == 0 ? &h->ctl->n_e[par] : &h->ctl->n_i[par];
  HIP_TRY(hipMemcpyAsync(cnt, &nn, 8, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(&h->ctl->pool_n[species], &nn, 8, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(launch_iota(h->pid[species][h->cur[species]], cnt, h->stream));
  int64_t* dep = species == 0 ? h->dep_e[par] : h->dep_i[h->cur_hi];
  HIP_TRY(hipMemsetAsync(dep, 0, (size_t)h->nx * 8, h->stream));
  HIP_TRY(launch_deposit(dst[0], cnt, h->inv_dx, h->nx, reinterpret_cast<unsigned long long*>(dep),
                         h->stream));
  HIP_TRY(hipMemsetAsync(h->ctl->counters, 0, sizeof(h->ctl->counters), h->stream));
  HIP_TRY(hipMemsetAsync(&h->ctl->err, 0, sizeof(uint32_t), h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return PIC_OK;
}

}  // namespace

extern "C" {

const char* pic_strerror(int s) {
  switch (s) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument or parameter set";
    case PIC_EHIP: return "HIP runtime error (no GPU, or a launch failed)";
    case PIC_ECAPACITY: return "a species outgrew its capacity";
    case PIC_EUNSTABLE: return "non-finite position, velocity or field";
    case PIC_ETABLE: return "reserved";
    case PIC_ESTATE: return "call not valid in the current state";
    default: return "unknown status";
  }
}

int pic_workspace_bytes(const pic_params* p, const pic_xsec* xs, uint64_t* bytes) {
  if (!bytes) return PIC_EINVAL;
  const int v = validate(p, xs);
  if (v) return v;
  *bytes = make_layout(p, xs).total;
  return PIC_OK;
}

int pic_init(const pic_params* p, const pic_xsec* xs, void* workspace, uint64_t workspace_bytes,
             void* stream, pic_handle** out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  int v = validate(p, xs);
  if (v) return v;
  const Layout L = make_layout(p, xs);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % kAlign) != 0)
    return PIC_EINVAL;
  pic_handle* h = new (std::nothrow) pic_handle();
  if (!h) return PIC_EINVAL;
  h->p = *p;
  h->stream = (hipStream_t)stream;
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device) !=
          hipSuccess) {
    delete h;
    return PIC_EHIP;
  }

  // ---- derived constants (Sec. 2): the operation order is part of the
  // method's definition, so every side computes them the same way
  h->nx = p->n_cells + 1;
  h->L = p->gap_m;
  h->dx = p->gap_m / (double)p->n_cells;
  h->inv_dx = 1.0 / h->dx;
  h->dt = 1.0 / (p->rf_freq_hz * (double)p->steps_per_cycle);
  h->ng = p->pressure_pa / (kKb * p->gas_temp_k);
  h->mass[0] = kMe;
  h->mass[1] = 39.948 * kAmu;
  h->dts[0] = h->dt;
  h->dts[1] = (double)p->ion_subcycle * h->dt;
  h->acc[0] = (-kQe / h->mass[0]) * h->dts[0];
  h->acc[1] = (kQe / h->mass[1]) * h->dts[1];
  h->nfac32 = p->weight / (p->area_m2 * h->dx) * kInvTwo32;
  h->qfac32 = kQe * h->nfac32;
  h->kpois = h->dx * h->dx * h->qfac32 / kEps0;
  h->inv_dv[0] = 1.0 / xs->dv_e;
  h->inv_dv[1] = 1.0 / xs->dv_i;
  h->ntab = xs->n;
  h->exc_thr = xs->exc_threshold_ev;
  h->ion_thr = xs->ion_threshold_ev;
  h->ek_e = 0.5 * kMe / kQe;
  h->ve_e = 2.0 * kQe / kMe;
  h->mr_e = kMe / (kMe + h->mass[1]);
  h->mm_e = h->mass[1] / (kMe + h->mass[1]);
  h->sig_g = std::sqrt(kKb * p->gas_temp_k / h->mass[1]);
  h->sig_se = std::sqrt(p->see_temp_ev * kQe / kMe);
  h->eepf_de = p->eepf_emax_ev / (double)p->eepf_bins;
  h->inv_de = (double)p->eepf_bins / p->eepf_emax_ev;

  // cumulative collision frequencies nu_k(v) = n_g sigma_k(v) v on the table
  // speeds, and nu_max over the table (Sec. 3.5)
  std::vector<double> cum[2];
  const double* sig[2][3] = {{xs->sigma_e[0], xs->sigma_e[1], xs->sigma_e[2]},
                             {xs->sigma_i[0], xs->sigma_i[1], nullptr}};
  const int nproc[2] = {3, 2};
  const double dv[2] = {xs->dv_e, xs->dv_i};
  for (int s = 0; s < 2; ++s) {
    cum[s].assign((size_t)nproc[s] * xs->n, 0.0);
    h->numax[s] = 0.0;
    for (int i = 0; i < xs->n; ++i) {
      const double vel = (double)i * dv[s];
      double run = 0.0;
      for (int k = 0; k < nproc[s]; ++k) {
        const double nu = h->ng * sig[s][k][i] * vel;
        run = (k == 0) ? nu : run + nu;
        cum[s][(size_t)k * xs->n + i] = run;
      }
      if (run > h->numax[s]) h->numax[s] = run;
    }
    h->pcoll[s] = 1.0 - std::exp(-h->numax[s] * h->dts[s]);
  }
  h->vtab.resize(p->steps_per_cycle);
  for (int m = 0; m < p->steps_per_cycle; ++m)
    h->vtab[m] = p->rf_voltage_v * std::cos(kTwoPi * (double)m / (double)p->steps_per_cycle);
  // Thomas recurrence coefficients of the constant [1, -2, 1] matrix
  std::vector<double> th_cp(h->nx, 0.0), th_m(h->nx, 0.0);
  {
    const int n = h->nx - 2;
    th_cp[0] = 1.0 / -2.0;
    th_m[0] = -2.0;
    for (int i = 1; i < n; ++i) {
      const double m = -2.0 - 1.0 * th_cp[i - 1];
      th_m[i] = m;
      th_cp[i] = 1.0 / m;
    }
  }

  // ---- workspace
  char* w = static_cast<char*>(workspace);
  h->ctl = reinterpret_cast<DevCtl*>(w + L.ctl);
  for (int s = 0; s < 2; ++s) {
    for (int b = 0; b < 2; ++b) {
      for (int q = 0; q < 2; ++q) {
        h->part[s][b][q] = reinterpret_cast<double*>(w + L.part[s][b][q]);
        h->pool[s][b][q] = reinterpret_cast<double*>(w + L.pool[s][b][q]);
      }
      h->pid[s][b] = reinterpret_cast<uint32_t*>(w + L.pid[s][b]);
    }
    h->pcap[s] = pool_capacity(p->capacity[s]);
    for (int b = 0; b < 2; ++b) h->codes[s][b] = reinterpret_cast<uint8_t*>(w + L.codes[s][b]);
    h->csel[s] = 0;
    for (int b = 0; b < 2; ++b) h->tcnt[s][b] = reinterpret_cast<uint64_t*>(w + L.tcnt[s][b]);
    h->tsel[s] = 0;
    h->rq[s] = reinterpret_cast<uint4*>(w + L.rq[s]);
    h->max_tiles[s] = L.max_tiles[s];
    h->cum[s] = reinterpret_cast<double*>(w + L.cum[s]);
  }
  for (int b = 0; b < 2; ++b) {
    h->dep_e[b] = reinterpret_cast<int64_t*>(w + L.dep_e[b]);
    h->dep_i[b] = reinterpret_cast<int64_t*>(w + L.dep_i[b]);
  }
  h->rho = reinterpret_cast<double*>(w + L.rho);
  h->phi = reinterpret_cast<double*>(w + L.phi);
  for (int b = 0; b < 2; ++b) h->Ebuf[b] = reinterpret_cast<double*>(w + L.E[b]);
  h->e_last = 0;
  h->th_cp = reinterpret_cast<double*>(w + L.th_cp);
  h->th_m = reinterpret_cast<double*>(w + L.th_m);
  h->acc_ne = reinterpret_cast<double*>(w + L.acc_ne);
  h->acc_ni = reinterpret_cast<double*>(w + L.acc_ni);
  h->acc_w = reinterpret_cast<double*>(w + L.acc_w);
  h->acc_ew = reinterpret_cast<double*>(w + L.acc_ew);
  h->eepf = reinterpret_cast<unsigned long long*>(w + L.eepf);
  for (int sp = 0; sp < 2; ++sp) h->fedf[sp] = reinterpret_cast<unsigned long long*>(w + L.fedf[sp]);
  h->fedf_emax[0] = p->eepf_emax_ev;
  h->fedf_emax[1] = fedf_ion_emax(p->rf_voltage_v);
  h->sort_cnt = reinterpret_cast<uint32_t*>(w + L.sort_cnt);
  h->sort_seg = reinterpret_cast<uint32_t*>(w + L.sort_seg);
  h->cand = reinterpret_cast<uint32_t*>(w + L.cand);
  h->dq = reinterpret_cast<uint32_t*>(w + L.dq);
  h->sort_blocks = L.sort_blocks;
  h->step = 0;
  h->cur[0] = h->cur[1] = 0;
  h->pcur[0] = h->pcur[1] = 0;
  h->cur_hi = 0;
  h->e_decided = 0;
  h->pipeline = 1;
  h->measuring = 0;

  int st = PIC_OK;
  if (hipMemsetAsync(workspace, 0, L.total, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->cum[0], cum[0].data(), cum[0].size() * 8, hipMemcpyHostToDevice,
                     h->stream) != hipSuccess ||
      hipMemcpyAsync(h->cum[1], cum[1].data(), cum[1].size() * 8, hipMemcpyHostToDevice,
                     h->stream) != hipSuccess ||
      hipMemcpyAsync(h->th_cp, th_cp.data(), th_cp.size() * 8, hipMemcpyHostToDevice,
                     h->stream) != hipSuccess ||
      hipMemcpyAsync(h->th_m, th_m.data(), th_m.size() * 8, hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    st = PIC_EHIP;
  if (st) {
    delete h;
    return st;
  }
  for (int s = 0; s < 2; ++s)
    h->launch[s] = particle_launch_config(s, h->nx, p->eepf_bins, h->num_cu, h->max_tiles[s]);
  h->d.n_x = h->nx;
  h->d.n_tiles_max = (int32_t)(L.max_tiles[0] > L.max_tiles[1] ? L.max_tiles[0] : L.max_tiles[1]);
  h->d.dx = h->dx;
  h->d.dt = h->dt;
  h->d.gas_density = h->ng;
  for (int s = 0; s < 2; ++s) {
    h->d.nu_max[s] = h->numax[s];
    h->d.p_coll[s] = h->pcoll[s];
  }
  *out = h;
  return PIC_OK;
}

int pic_get_derived(const pic_handle* h, pic_derived* d) {
  if (!h || !d) return PIC_EINVAL;
  *d = h->d;
  return PIC_OK;
}

int pic_set_state(pic_handle* h, int species, const double* x, const double* vx, const double* vy,
                  const double* vz, int64_t n, int64_t step) {
  if (!h || species < 0 || species > 1 || n < 0 || step < 0) return PIC_EINVAL;
  if (n > 0 && (!x || !vx || !vy || !vz)) return PIC_EINVAL;
  if (n > h->p.capacity[species]) return PIC_ECAPACITY;
  return replace_state(h, species, n, step, [&](double* const* dst, double* const* pool) {
    HIP_TRY(hipMemcpyAsync(dst[0], x, (size_t)n * 8, hipMemcpyDefault, h->stream));
    HIP_TRY(hipMemcpyAsync(dst[1], vx, (size_t)n * 8, hipMemcpyDefault, h->stream));
    HIP_TRY(hipMemcpyAsync(pool[0], vy, (size_t)n * 8, hipMemcpyDefault, h->stream));
    HIP_TRY(hipMemcpyAsync(pool[1], vz, (size_t)n * 8, hipMemcpyDefault, h->stream));
    return PIC_OK;
  });
}

int pic_load_profile(pic_handle* h, int species, int64_t n, const double* dens, const double* temp_ev,
                     int npts, int64_t step) {
  if (!h || species < 0 || species > 1 || n < 0 || step < 0) return PIC_EINVAL;
  if (npts < 2 || npts > kMaxLoadPoints || (n > 0 && (!dens || !temp_ev))) return PIC_EINVAL;
  if (n > h->p.capacity[species]) return PIC_ECAPACITY;
  return replace_state(h, species, n, step, [&](double* const* dst, double* const* pool) {
    LoadArgs a{};
    a.dens = dens;
    a.temp = temp_ev;
    a.x = dst[0];
    a.vx = dst[1];
    a.vy = pool[0];
    a.vz = pool[1];
    a.n = n;
    a.L = h->L;
    a.h = h->L / (double)(npts - 1);
    a.hh = 0.5 * a.h;
    a.vfac = kQe / h->mass[species];
    a.npts = npts;
    a.species = species;
    a.seed = h->p.seed;
    a.run = h->p.run;
    HIP_TRY(launch_load_profile(a, h->stream));
    return PIC_OK;
  });
}

int pic_get_state(pic_handle* h, int species, double* x, double* vx, double* vy, double* vz,
                  int64_t cap, int64_t* n, int64_t* step) {
  if (!h || species < 0 || species > 1 || !n) return PIC_EINVAL;
  const int err = latched(h);
  const int par = (int)(h->step & 1);
  int64_t cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, species == 0 ? &h->ctl->n_e[par] : &h->ctl->n_i[par], 8,
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  *n = cnt;
  if (step) *step = h->step;
  if (err) return err;
  if (cnt > cap) return PIC_ECAPACITY;
  if (cnt > 0 && (!x || !vx || !vy || !vz)) return PIC_EINVAL;
  if (cnt > 0) {
    // v_y, v_z in slot order, gathered through the pool indices into the
    // idle pool buffer
    double* const* part = h->part[species][h->cur[species]];
    double* const* pool = h->pool[species][h->pcur[species]];
    double* const* tmp = h->pool[species][1 - h->pcur[species]];
    HIP_TRY(launch_gather(h->pid[species][h->cur[species]], pool[0], pool[1], tmp[0], tmp[1], cnt,
                          h->stream));
    HIP_TRY(hipMemcpyAsync(x, part[0], (size_t)cnt * 8, hipMemcpyDefault, h->stream));
    HIP_TRY(hipMemcpyAsync(vx, part[1], (size_t)cnt * 8, hipMemcpyDefault, h->stream));
    HIP_TRY(hipMemcpyAsync(vy, tmp[0], (size_t)cnt * 8, hipMemcpyDefault, h->stream));
    HIP_TRY(hipMemcpyAsync(vz, tmp[1], (size_t)cnt * 8, hipMemcpyDefault, h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return PIC_OK;
}

int pic_step(pic_handle* h, int64_t n_steps) {
  if (!h || n_steps < 0) return PIC_EINVAL;
  if ((h->p.flags & PIC_FLAG_FIXED_E) && !h->field_fixed_set) return PIC_ESTATE;
  bool field_ready = false;
  for (int64_t it = 0; it < n_steps; ++it) {
    const StepPlan q = plan_step(h, field_ready, it + 1 == n_steps, h->pipeline != 0);
    const int st = launch_step(h, q);
    if (st) return st;
    field_ready = q.tail || q.fuse;
    // keep the event backlog bounded
    if (h->ev_used.size() >= 4096) {
      const int c = timer_collect(h);
      if (c) return c;
    }
  }
  return PIC_OK;
}

int pic_step_many(pic_handle* const* handles, int n, int64_t n_steps, int64_t chunk) {
  if (n < 0 || n_steps < 0 || chunk < 1 || (n > 0 && !handles)) return PIC_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!handles[i]) return PIC_EINVAL;
    for (int k = 0; k < i; ++k)
      if (handles[k] == handles[i]) return PIC_EINVAL;
  }
  for (int64_t done = 0; done < n_steps; done += chunk) {
    const int64_t m = (n_steps - done < chunk) ? n_steps - done : chunk;
    for (int i = 0; i < n; ++i) {
      const int st = pic_step(handles[i], m);
      if (st) return st;
    }
  }
  return PIC_OK;
}

int pic_batch_workspace_bytes(pic_handle* const* handles, int n, uint64_t* bytes) {
  if (!bytes) return PIC_EINVAL;
  const int v = check_batch_handles(handles, n);
  if (v) return v;
  *bytes = 2 * (uint64_t)batch_chunk_steps(n) * batch_step_bytes(n);
  return PIC_OK;
}

int pic_batch_create(pic_handle* const* handles, int n, void* workspace, uint64_t workspace_bytes,
                     pic_batch** out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  const int v = check_batch_handles(handles, n);
  if (v) return v;
  const int chunk = batch_chunk_steps(n);
  const size_t per = batch_step_bytes(n);
  const size_t half = (size_t)chunk * per;
  if (!workspace || workspace_bytes < 2 * half || ((uintptr_t)workspace % kAlign) != 0)
    return PIC_EINVAL;
  pic_batch* b = new (std::nothrow) pic_batch();
  if (!b) return PIC_EINVAL;
  b->hs.assign(handles, handles + n);
  b->stream = handles[0]->stream;
  b->chunk = chunk;
  b->step_bytes = per;
  b->slot = 0;
  int nx_max = 0, nbins_max = 0;
  int64_t tiles[2] = {0, 0};
  for (pic_handle* h : b->hs) {
    nx_max = h->nx > nx_max ? h->nx : nx_max;
    nbins_max = h->p.eepf_bins > nbins_max ? h->p.eepf_bins : nbins_max;
    tiles[0] += h->max_tiles[0];
    tiles[1] += h->max_tiles[1];
  }
  b->launch = batch_launch_config(nx_max, nbins_max, handles[0]->num_cu, tiles);
  b->variants = false;
  for (pic_handle* h : b->hs)
    if (h->p.flags & (PIC_FLAG_ANISO_ELASTIC | PIC_FLAG_OPAL_SHARING)) b->variants = true;
  for (int k = 0; k < 2; ++k) {
    b->dev[k] = static_cast<unsigned char*>(workspace) + k * half;
    b->host[k] = nullptr;
    b->copied[k] = nullptr;
  }
  bool ok = true;
  for (int k = 0; k < 2 && ok; ++k) {
    ok = hipHostMalloc((void**)&b->host[k], half, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    pic_batch_free(b);
    return PIC_EHIP;
  }
  *out = b;
  return PIC_OK;
}

int pic_batch_step(pic_batch* b, int64_t n_steps) {
  if (!b || n_steps < 0) return PIC_EINVAL;
  for (pic_handle* h : b->hs)
    if ((h->p.flags & PIC_FLAG_FIXED_E) && !h->field_fixed_set) return PIC_ESTATE;
  const int n = (int)b->hs.size();
  hipStream_t s = b->stream;
  const BatchLaunch& c = b->launch;

  // one step's launches: device addresses of its argument arrays and counts
  struct StepLaunch {
    const FieldArgs* ff;
    const FieldArgs* fn;
    const PartArgs* ed;  // measuring discharges first
    const PartArgs* er;
    const PartArgs* ia;
    const PartArgs* t0;
    const SortArgs* so[2];  // sorts of each species due after the step
    int nff, nem, nion, nt0, nso;
    int64_t so_blocks;
    bool tail;
  };
  struct Post {
    int step;
    int discharge;
    StepPlan q;
  };
  std::vector<StepPlan> plans(n);
  std::vector<StepLaunch> steps;
  std::vector<Post> posts;
  bool field_ready = false;
  for (int64_t done = 0; done < n_steps;) {
    const int m = (int)((n_steps - done < b->chunk) ? n_steps - done : b->chunk);
    const int slot = b->slot;
    b->slot ^= 1;
    // the last upload from this host buffer has been read
    HIP_TRY(hipEventSynchronize(b->copied[slot]));
    unsigned char* H = b->host[slot];
    unsigned char* D = b->dev[slot];
    size_t off = 0;
    steps.clear();
    posts.clear();
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + kBatchArrayAlign - 1) / kBatchArrayAlign * kBatchArrayAlign;
      return o;
    };
    for (int k = 0; k < m; ++k) {
      const bool last = done + k + 1 == n_steps;
      for (int i = 0; i < n; ++i) plans[i] = plan_step(b->hs[i], field_ready, last, false);
      field_ready = !last;
      StepLaunch L{};
      L.tail = !last;
      const size_t o_ff = take(n * sizeof(FieldArgs)), o_fn = take(n * sizeof(FieldArgs));
      const size_t o_ed = take(n * sizeof(PartArgs)), o_er = take(n * sizeof(PartArgs));
      const size_t o_ia = take(n * sizeof(PartArgs)), o_t0 = take(n * sizeof(PartArgs));
      const size_t o_s0 = take(n * sizeof(SortArgs)), o_s1 = take(n * sizeof(SortArgs));
      SortArgs* s0 = reinterpret_cast<SortArgs*>(H + o_s0);
      SortArgs* s1 = reinterpret_cast<SortArgs*>(H + o_s1);
      FieldArgs* ff = reinterpret_cast<FieldArgs*>(H + o_ff);
      FieldArgs* fn = reinterpret_cast<FieldArgs*>(H + o_fn);
      PartArgs* ed = reinterpret_cast<PartArgs*>(H + o_ed);
      PartArgs* er = reinterpret_cast<PartArgs*>(H + o_er);
      PartArgs* ia = reinterpret_cast<PartArgs*>(H + o_ia);
      PartArgs* t0 = reinterpret_cast<PartArgs*>(H + o_t0);
      int ne = 0;
      for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < n; ++i)
          if (plans[i].measure == (pass == 0)) {
            ed[ne++] = plans[i].ae;
            if (pass == 0) L.nem += 1;
          }
      for (int i = 0; i < n; ++i) {
        const StepPlan& q = plans[i];
        if (q.field_first) ff[L.nff++] = q.ff;
        if (L.tail) fn[i] = q.fn;
        if (q.ion) {
          er[L.nion] = q.ae;
          ia[L.nion++] = q.ai;
        } else {
          t0[L.nt0++] = q.ae;
        }
        if (q.post == 1) {
          s0[L.nso] = q.sa[0];
          s1[L.nso++] = q.sa[1];
          L.so_blocks += q.sa[0].nblocks;
        } else if (q.post) {
          posts.push_back(Post{k, i, q});
        }
      }
      L.ff = reinterpret_cast<const FieldArgs*>(D + o_ff);
      L.fn = reinterpret_cast<const FieldArgs*>(D + o_fn);
      L.ed = reinterpret_cast<const PartArgs*>(D + o_ed);
      L.er = reinterpret_cast<const PartArgs*>(D + o_er);
      L.ia = reinterpret_cast<const PartArgs*>(D + o_ia);
      L.t0 = reinterpret_cast<const PartArgs*>(D + o_t0);
      L.so[0] = reinterpret_cast<const SortArgs*>(D + o_s0);
      L.so[1] = reinterpret_cast<const SortArgs*>(D + o_s1);
      steps.push_back(L);
    }
    HIP_TRY(hipMemcpyAsync(D, H, off, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(b->copied[slot], s));
    size_t pi = 0;
    for (int k = 0; k < m; ++k) {
      const StepLaunch& L = steps[k];
      if (L.nff) HIP_TRY(launch_batch_field(L.ff, L.nff, s));
      if (L.nem) HIP_TRY(launch_batch_pass(0, 0, true, L.ed, L.nem, c, s, b->variants));
      if (n > L.nem) HIP_TRY(launch_batch_pass(0, 0, false, L.ed + L.nem, n - L.nem, c, s, b->variants));
      HIP_TRY(launch_batch_pass(1, 0, false, L.ed, n, c, s, b->variants));
      if (L.nion) {
        HIP_TRY(launch_batch_pass(2, 0, false, L.er, L.nion, c, s, b->variants));
        HIP_TRY(launch_batch_pass(0, 1, false, L.ia, L.nion, c, s, b->variants));
        HIP_TRY(launch_batch_pass(1, 1, false, L.ia, L.nion, c, s, b->variants));
      }
      if (L.tail) {
        if (L.nion) {
          HIP_TRY(launch_batch_tail(1, L.fn, n, L.ia, L.nion, kTailRareBlocks, s, b->variants));
          if (L.nt0) HIP_TRY(launch_batch_pass(2, 0, false, L.t0, L.nt0, c, s, b->variants));
        } else {
          HIP_TRY(launch_batch_tail(0, L.fn, n, L.t0, L.nt0, kTailRareBlocks, s, b->variants));
        }
      } else {
        if (L.nt0) HIP_TRY(launch_batch_pass(2, 0, false, L.t0, L.nt0, c, s, b->variants));
        if (L.nion) HIP_TRY(launch_batch_pass(2, 1, false, L.ia, L.nion, c, s, b->variants));
      }
      // cell sorts: species 0 of every due discharge, then species 1 (the
      // two species of a discharge share its sort counters)
      if (L.nso) {
        HIP_TRY(launch_batch_sort(L.so[0], L.nso, L.so_blocks, c.nx_max, s));
        HIP_TRY(launch_batch_sort(L.so[1], L.nso, L.so_blocks, c.nx_max, s));
      }
      for (; pi < posts.size() && posts[pi].step == k; ++pi) {
        const int st = launch_post(b->hs[posts[pi].discharge], posts[pi].q, s);
        if (st) return st;
      }
    }
    done += m;
  }
  return PIC_OK;
}

void pic_batch_free(pic_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (int k = 0; k < 2; ++k) {
    if (b->host[k]) (void)hipHostFree(b->host[k]);
    if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
  }
  delete b;
}

int pic_sync(pic_handle* h) {
  if (!h) return PIC_EINVAL;
  return latched(h);
}

int pic_set_field(pic_handle* h, const double* E) {
  if (!h || !E) return PIC_EINVAL;
  if (!(h->p.flags & PIC_FLAG_FIXED_E)) return PIC_ESTATE;
  for (int b = 0; b < 2; ++b)
    HIP_TRY(hipMemcpyAsync(h->Ebuf[b], E, (size_t)h->nx * 8, hipMemcpyDefault, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->field_fixed_set = 1;
  return PIC_OK;
}

int pic_get_field(pic_handle* h, double* rho, double* phi, double* E, int64_t* deposit_e,
                  int64_t* deposit_i) {
  if (!h) return PIC_EINVAL;
  const size_t b = (size_t)h->nx * 8;
  const int par = (int)(h->step & 1);
  if (rho) HIP_TRY(hipMemcpyAsync(rho, h->rho, b, hipMemcpyDefault, h->stream));
  if (phi) HIP_TRY(hipMemcpyAsync(phi, h->phi, b, hipMemcpyDefault, h->stream));
  if (E) HIP_TRY(hipMemcpyAsync(E, h->Ebuf[h->e_last], b, hipMemcpyDefault, h->stream));
  if (deposit_e) HIP_TRY(hipMemcpyAsync(deposit_e, h->dep_e[par], b, hipMemcpyDefault, h->stream));
  if (deposit_i)
    HIP_TRY(hipMemcpyAsync(deposit_i, h->dep_i[h->cur_hi], b, hipMemcpyDefault, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return latched(h);
}

int pic_measure(pic_handle* h, int on) {
  if (!h) return PIC_EINVAL;
  h->measuring = on ? 1 : 0;
  return PIC_OK;
}

int pic_moments(pic_handle* h, pic_moments_out* out, int reset) {
  if (!h || !out) return PIC_EINVAL;
  const int nx = h->nx, nb = h->p.eepf_bins;
  std::vector<double> ne(nx), ni(nx), w(nx), ew(nx);
  std::vector<unsigned long long> hist(nb);
  int64_t msteps = 0;
  HIP_TRY(hipMemcpyAsync(ne.data(), h->acc_ne, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(ni.data(), h->acc_ni, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(w.data(), h->acc_w, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(ew.data(), h->acc_ew, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(hist.data(), h->eepf, nb * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(&msteps, &h->ctl->msteps, 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int j = 0; j < nx; ++j) {
    if (out->n_e) out->n_e[j] = msteps ? ne[j] / (double)msteps : 0.0;
    if (out->n_i) out->n_i[j] = msteps ? ni[j] / (double)msteps : 0.0;
    if (out->mean_energy_e) out->mean_energy_e[j] = w[j] > 0.0 ? ew[j] / w[j] : 0.0;
  }
  if (out->eepf) {
    unsigned long long tot = 0;
    for (int b = 0; b < nb; ++b) tot += hist[b];
    for (int b = 0; b < nb; ++b) {
      const double eb = ((double)b + 0.5) * h->eepf_de;
      out->eepf[b] = tot ? (double)hist[b] / ((double)tot * std::sqrt(eb) * h->eepf_de) : 0.0;
    }
  }
  out->steps_averaged = msteps;
  if (reset) {
    HIP_TRY(hipMemsetAsync(h->acc_ne, 0, nx * 8, h->stream));
    HIP_TRY(hipMemsetAsync(h->acc_ni, 0, nx * 8, h->stream));
    HIP_TRY(hipMemsetAsync(h->acc_w, 0, nx * 8, h->stream));
    HIP_TRY(hipMemsetAsync(h->acc_ew, 0, nx * 8, h->stream));
    HIP_TRY(hipMemsetAsync(h->eepf, 0, nb * 8, h->stream));
    for (int sp = 0; sp < 2; ++sp) HIP_TRY(hipMemsetAsync(h->fedf[sp], 0, (size_t)2 * nb * 8, h->stream));
    HIP_TRY(hipMemsetAsync(h->ctl->wall_hits, 0,
                           sizeof(h->ctl->wall_hits) + sizeof(h->ctl->wall_absorbed) +
                               sizeof(h->ctl->wall_esum) + sizeof(h->ctl->ioniz_meas),
                           h->stream));
    HIP_TRY(hipMemsetAsync(&h->ctl->msteps, 0, 8, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return latched(h);
}

int pic_wall_moments(pic_handle* h, pic_wall_out* out) {
  if (!h || !out) return PIC_EINVAL;
  const int nb = h->p.eepf_bins;
  std::vector<unsigned long long> hist[2];
  unsigned long long hits[2][2], absd[2][2], ioniz = 0;
  double esum[2][2];
  int64_t msteps = 0;
  for (int sp = 0; sp < 2; ++sp) {
    hist[sp].resize((size_t)2 * nb);
    HIP_TRY(hipMemcpyAsync(hist[sp].data(), h->fedf[sp], (size_t)2 * nb * 8, hipMemcpyDeviceToHost,
                           h->stream));
  }
  HIP_TRY(hipMemcpyAsync(hits, h->ctl->wall_hits, sizeof(hits), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(absd, h->ctl->wall_absorbed, sizeof(absd), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(esum, h->ctl->wall_esum, sizeof(esum), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(&ioniz, &h->ctl->ioniz_meas, 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(&msteps, &h->ctl->msteps, 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  // particles per m^2 per s over the measured time msteps * dt
  const double per = msteps ? h->p.weight / (h->p.area_m2 * (double)msteps * h->dt) : 0.0;
  for (int sp = 0; sp < 2; ++sp) {
    const double de = h->fedf_emax[sp] / (double)nb;
    out->fedf_emax_ev[sp] = h->fedf_emax[sp];
    for (int w = 0; w < 2; ++w) {
      out->arrivals[sp][w] = (int64_t)hits[sp][w];
      out->absorbed[sp][w] = (int64_t)absd[sp][w];
      out->flux[sp][w] = per * (double)hits[sp][w];
      out->absorbed_flux[sp][w] = per * (double)absd[sp][w];
      out->mean_energy_ev[sp][w] = hits[sp][w] ? esum[sp][w] / (double)hits[sp][w] : 0.0;
      double* f = out->fedf[sp][w];
      if (!f) continue;
      unsigned long long tot = 0;
      for (int b = 0; b < nb; ++b) tot += hist[sp][(size_t)w * nb + b];
      for (int b = 0; b < nb; ++b)
        f[b] = tot ? (double)hist[sp][(size_t)w * nb + b] / ((double)tot * de) : 0.0;
    }
  }
  out->fedf_bins = nb;
  out->ionizations = (int64_t)ioniz;
  out->ionization_rate = per * (double)ioniz;
  out->steps_averaged = msteps;
  return latched(h);
}

int pic_get_monitors(pic_handle* h, pic_monitors* out) {
  if (!h || !out) return PIC_EINVAL;
  const int nx = h->nx;
  std::vector<double> ne(nx), w(nx), ew(nx);
  int64_t msteps = 0;
  HIP_TRY(hipMemcpyAsync(ne.data(), h->acc_ne, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(w.data(), h->acc_w, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(ew.data(), h->acc_ew, nx * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(&msteps, &h->ctl->msteps, 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  out->steps_averaged = msteps;
  out->p_coll[0] = h->pcoll[0];
  out->p_coll[1] = h->pcoll[1];
  double nmax = 0.0;
  for (int j = 0; j < nx; ++j) {
    ne[j] = msteps ? ne[j] / (double)msteps : 0.0;
    nmax = ne[j] > nmax ? ne[j] : nmax;
  }
  // centre values: the middle node, or the mean of the two middle nodes
  const int j0 = (nx - 1) / 2, j1 = nx / 2;
  const double nc = 0.5 * (ne[j0] + ne[j1]);
  const double e0 = w[j0] > 0.0 ? ew[j0] / w[j0] : 0.0;
  const double e1 = w[j1] > 0.0 ? ew[j1] / w[j1] : 0.0;
  const double ec = 0.5 * (e0 + e1);
  out->n_e_max = nmax;
  out->n_e_center = nc;
  out->mean_energy_center_ev = ec;
  out->omega_pe_dt = std::sqrt(nmax * kQe * kQe / (kEps0 * kMe)) * h->dt;
  const double te = (2.0 / 3.0) * ec;  // eV
  out->lambda_d_m = nc > 0.0 ? std::sqrt(kEps0 * te / (kQe * nc)) : 0.0;
  out->dx_over_lambda_d = out->lambda_d_m > 0.0 ? h->dx / out->lambda_d_m : 0.0;
  out->n_d = nc * h->p.area_m2 * out->lambda_d_m / h->p.weight;
  return latched(h);
}

int pic_get_counters(pic_handle* h, int64_t* counters) {
  if (!h || !counters) return PIC_EINVAL;
  unsigned long long c[kCounterSlots][NCOUNTERS];
  HIP_TRY(hipMemcpyAsync(c, h->ctl->counters, sizeof(c), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int i = 0; i < NCOUNTERS; ++i) {
    unsigned long long t = 0;
    for (int k = 0; k < kCounterSlots; ++k) t += c[k][i];
    counters[i] = (int64_t)t;
  }
  return latched(h);
}

int pic_get_decisions(pic_handle* h, int species, uint8_t* codes, int64_t cap, int64_t* n) {
  if (!h || species < 0 || species > 1 || !n) return PIC_EINVAL;
  if (!(h->p.flags & PIC_FLAG_RECORD)) return PIC_ESTATE;
  int64_t cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, &h->ctl->ncodes[species], 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  *n = cnt;
  if (cnt > cap) return PIC_ECAPACITY;
  if (cnt > 0) {
    if (!codes) return PIC_EINVAL;
    HIP_TRY(hipMemcpyAsync(codes, h->codes[species][h->csel[species] ^ 1], (size_t)cnt,
                           hipMemcpyDefault, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return latched(h);
}

int pic_set_launch(pic_handle* h, int decide_wg_per_cu, int emit_wg_per_cu) {
  if (!h || decide_wg_per_cu < 1 || emit_wg_per_cu < 1) return PIC_EINVAL;
  for (int s = 0; s < 2; ++s) particle_launch_set(h->launch[s], h->num_cu, decide_wg_per_cu, emit_wg_per_cu);
  return PIC_OK;
}

int pic_set_decide_block(pic_handle* h, int threads) {
  if (!h || (threads != kDecideBlocks[0] && threads != kDecideBlocks[1])) return PIC_EINVAL;
  for (int s = 0; s < 2; ++s)
    if (!particle_launch_block(h->launch[s], h->num_cu, threads)) return PIC_EINVAL;
  return PIC_OK;
}

int pic_set_pipeline(pic_handle* h, int on) {
  if (!h || on < 0 || on > 1) return PIC_EINVAL;
  h->pipeline = on;
  return PIC_OK;
}

int pic_tune(pic_handle* h, int64_t steps_per_trial, int* decide_wg_per_cu, int* emit_wg_per_cu) {
  if (!h || steps_per_trial < 1) return PIC_EINVAL;
  // time one kernel of the electron pass over steps_per_trial steps with
  // events around every particle kernel, without disturbing the caller's
  // accumulated timers
  const int level = h->timing;
  auto trial = [&](int timer, double* us) -> int {
    int st = timer_collect(h);
    if (st) return st;
    const double ms0 = h->t_ms[timer];
    const int64_t n0 = h->t_n[timer];
    h->timing = 2;
    st = pic_step(h, steps_per_trial);
    if (!st) st = timer_collect(h);
    h->timing = level;
    if (st) return st;
    const int64_t n = h->t_n[timer] - n0;
    *us = n ? 1e3 * (h->t_ms[timer] - ms0) / (double)n : 0.0;
    h->t_ms[timer] = ms0;
    h->t_n[timer] = n0;
    return PIC_OK;
  };
  const PartLaunch& c = h->launch[0];
  int kd = c.bpc_decide[0], ke = c.bpc_emit;
  double best = -1.0;
  for (int k = 1; k <= c.bpc_decide[0]; ++k) {
    pic_set_launch(h, k, ke);
    double us = 0.0;
    const int st = trial(PIC_TIMER_E_DECIDE, &us);
    if (st) return st;
    if (best < 0.0 || us < best) {
      best = us;
      kd = k;
    }
  }
  best = -1.0;
  for (int k = 1; k <= c.bpc_emit; ++k) {
    pic_set_launch(h, kd, k);
    double us = 0.0;
    const int st = trial(PIC_TIMER_E_EMIT, &us);
    if (st) return st;
    if (best < 0.0 || us < best) {
      best = us;
      ke = k;
    }
  }
  pic_set_launch(h, kd, ke);
  if (decide_wg_per_cu) *decide_wg_per_cu = kd;
  if (emit_wg_per_cu) *emit_wg_per_cu = ke;
  return latched(h);
}

int pic_tune_pass(pic_handle* h, int64_t steps_per_trial, pic_pass_trial* trials, int max_trials,
                  int* n_trials, int* best) {
  if (!h || steps_per_trial < 1 || max_trials < 0 || (max_trials > 0 && !trials)) return PIC_EINVAL;
  // the particle passes' time per step over steps_per_trial ordinary steps,
  // with events around each pass (timing level 1), without disturbing the
  // caller's accumulated timers
  const int level = h->timing;
  const int pipeline0 = h->pipeline;
  auto trial = [&](double* us) -> int {
    int st = timer_collect(h);
    if (st) return st;
    double ms0[2];
    int64_t n0[2];
    const int tm[2] = {PIC_TIMER_ELECTRON, PIC_TIMER_ION};
    for (int k = 0; k < 2; ++k) {
      ms0[k] = h->t_ms[tm[k]];
      n0[k] = h->t_n[tm[k]];
    }
    h->timing = 1;
    st = pic_step(h, steps_per_trial);
    if (!st) st = timer_collect(h);
    h->timing = level;
    if (st) return st;
    double ms = 0.0;
    for (int k = 0; k < 2; ++k) {
      ms += h->t_ms[tm[k]] - ms0[k];
      h->t_ms[tm[k]] = ms0[k];
      h->t_n[tm[k]] = n0[k];
    }
    *us = 1e3 * ms / (double)steps_per_trial;
    return PIC_OK;
  };
  const PartLaunch& c = h->launch[0];
  const int db0 = c.decide_block;
  int n = 0, ib = -1;
  pic_pass_trial bestt{};
  auto run = [&](int pipe, int db, int kd, int ke, double* us) -> int {
    h->pipeline = pipe;
    int st = pic_set_decide_block(h, db);
    if (!st) st = pic_set_launch(h, kd, ke);
    if (st) return st;
    pic_pass_trial t{pipe, db, kd, ke, 0.0};
    st = trial(&t.us_per_step);
    if (st) return st;
    if (n < max_trials) trials[n] = t;
    if (ib < 0 || t.us_per_step < bestt.us_per_step) {
      ib = n;
      bestt = t;
    }
    ++n;
    *us = t.us_per_step;
    return PIC_OK;
  };
  int st = PIC_OK;
  double us = 0.0;
  // pipelined: the fused emit's workgroups per CU (its decide pass runs only
  // on the steps that cannot be pipelined, at the default size and the most
  // workgroups that fit)
  const int kd_max = c.bpc_decide_by[0][0];
  for (int k = 1; k <= c.bpc_emit_decide && !st; ++k) st = run(1, kDecideBlocks[0], kd_max, k, &us);
  // unpipelined: each compiled decide size at each of its shapes, then each
  // emit shape at the best decide
  int db_best = kDecideBlocks[0], kd_best = kd_max;
  double kd_us = -1.0;
  for (int b = 0; b < 2 && !st; ++b) {
    for (int k = 1; k <= c.bpc_decide_by[b][0] && !st; ++k) {
      st = run(0, kDecideBlocks[b], k, c.bpc_emit, &us);
      if (!st && (kd_us < 0.0 || us < kd_us)) {
        kd_us = us;
        db_best = kDecideBlocks[b];
        kd_best = k;
      }
    }
  }
  for (int k = 1; k < c.bpc_emit && !st; ++k) st = run(0, db_best, kd_best, k, &us);
  if (st) {
    h->pipeline = pipeline0;
    (void)pic_set_decide_block(h, db0);
    return st;
  }
  h->pipeline = bestt.pipeline;
  pic_set_decide_block(h, bestt.decide_block);
  pic_set_launch(h, bestt.decide_wg_per_cu, bestt.emit_wg_per_cu);
  if (n_trials) *n_trials = n;
  if (best) *best = ib;
  return latched(h);
}

int pic_timing(pic_handle* h, int level) {
  if (!h || level < 0 || level > 2) return PIC_EINVAL;
  h->timing = level;
  return PIC_OK;
}

int pic_get_timing(pic_handle* h, double* ms, int64_t* launches, int reset) {
  if (!h) return PIC_EINVAL;
  const int st = timer_collect(h);
  if (st) return st;
  for (int i = 0; i < PIC_NTIMERS; ++i) {
    if (ms) ms[i] = h->t_ms[i];
    if (launches) launches[i] = h->t_n[i];
    if (reset) {
      h->t_ms[i] = 0.0;
      h->t_n[i] = 0;
    }
  }
  return PIC_OK;
}

void pic_free(pic_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
}

int pic_selftest_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n,
                        void* stream) {
  if (n < 0 || !key || (n > 0 && (!ctr || !out))) return PIC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_selftest_philox(ctr, key[0], key[1], out, n, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PIC_OK;
}

int pic_selftest_sqrt(const double* in, double* out, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!in || !out))) return PIC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_selftest_sqrt(in, out, n, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PIC_OK;
}

int pic_selftest_copy(const double* in, double* out, int64_t n, void* stream) {
  if (n < 0 || (n & 1) || (n > 0 && (!in || !out))) return PIC_EINVAL;
  if (((uintptr_t)in | (uintptr_t)out) & 15) return PIC_EINVAL;
  HIP_TRY(launch_selftest_copy(in, out, n, (hipStream_t)stream));
  return PIC_OK;
}

}  // extern "C"
