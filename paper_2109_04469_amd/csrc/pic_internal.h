// Internal declarations of libpic: kernel argument blocks (shared by the
// device code and the host launchers) and the host-side handle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/pic.h"
#include "pic_dev.h"

namespace pic {

constexpr double kQe = 1.602176634e-19;     // CODATA 2018
constexpr double kMe = 9.1093837015e-31;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKb = 1.380649e-23;

enum FieldMode { FIELD_EXACT = 0, FIELD_ZERO = 1, FIELD_FIXED = 2, FIELD_THOMAS = 3 };

struct FieldArgs {
  const int64_t* dep_e;
  const int64_t* dep_i;
  int64_t* zero_a;  // deposit buffers cleared for this step's particle kernels
  int64_t* zero_b;
  double* rho;
  double* phi;
  double* E;
  const double* th_cp;  // Thomas recurrence coefficients (FIELD_THOMAS)
  const double* th_m;
  double* acc_ne;
  double* acc_ni;
  double* acc_w;
  DevCtl* ctl;
  double V;
  double dx;
  double qfac32;  // e W / (A dx) 2^-32
  double nfac32;  // W / (A dx) 2^-32
  double kpois;   // dx^2 qfac32 / eps0
  int nx;
  int mode;
  int measuring;
  int parity;
  // pipelined steps: candidacy bits of the next step's electron slots,
  // drawn by the other workgroups of k_field_cand (null otherwise)
  uint32_t* cand;
  const uint64_t* cand_tcnt;  // the deciding pass's tile totals (their outputs are the slots)
  const int64_t* cand_count;  // the deciding pass's slot count
  uint64_t* cand_zero;        // the tile totals the fused pass adds into, zeroed here
  int64_t cand_zero_n;
  int64_t cand_cap;
  uint64_t cand_thr;
  uint32_t cand_step;
  uint32_t seed;
  uint32_t run;
};

// Particle state of a species: x, v_x and a 4-byte pool index per slot in
// ping-pong buffers, and v_y, v_z in a velocity pool at that index. A pass
// moves (x, v_x, id); v_y and v_z stay in place unless a collision changes
// them, and newborns take fresh pool entries.
struct PartArgs {
  const double* xin;
  const double* vxin;
  const uint32_t* idin;
  double* xout;
  double* vxout;
  uint32_t* idout;
  double* pvy;  // this species' velocity pool
  double* pvz;
  // births of the other species are appended here
  double* bx;
  double* bvx;
  uint32_t* bid;
  double* bpvy;  // the other species' velocity pool
  double* bpvz;
  const double* E;
  unsigned long long* dep_own;    // deposit of this kernel's outputs
  unsigned long long* dep_other;  // deposit of the other species' births
  const double* cum;              // cumulative nu tables, nproc x ntab
  DevCtl* ctl;
  uint64_t* tcnt;   // per tile: outputs | births << 16 | queued slots << 32
  uint64_t* tcnt_next;  // the other totals buffer: zeroed here for the next pass
  uint4* rq;        // queued slots: (slot, code, output slot, birth rank)
  uint8_t* codes;
  const uint32_t* cand;          // candidacy bit per slot (electrons, pipelined steps)
  uint32_t* dq;                  // output slots whose next-step decision is deferred
  double* acc_ew;                // CIC-weighted energy (electrons, measuring)
  unsigned long long* eepf;     // EEPF histogram (electrons, measuring)
  unsigned long long* fedf;     // this species' arrivals per energy bin, [wall][nbins]
  double ek_s;                  // m_s / (2 e): eV per (m/s)^2, this species
  double fedf_inv_de;           // energy bins per eV of the arrival histogram
  int measure_walls;            // accumulate electrode arrivals (measuring)
  int64_t cap;                  // capacity of the output arrays
  int64_t bcap;                 // capacity of the birth target arrays
  int64_t pcap;                 // capacity of this species' pool
  int64_t bpcap;                // capacity of the other species' pool
  int64_t max_tiles;
  double inv_dx;
  double L;
  double acc;      // (q/m) dt_s
  double dts;
  double p_wall;   // R (electrons) or gamma (ions)
  double pcoll;
  uint64_t pcoll_thr;  // u01(r) < pcoll exactly when r < pcoll_thr (r a 32-bit word)
  double numax;
  double inv_dv;
  double mr;       // m/(m+M) (electron elastic)
  double mm;       // M/(m+M)
  double ek;       // 1/2 m / e  (J -> eV factor times m/2)
  double ve;       // 2 e / m
  double exc_thr;
  double ion_thr;
  double sig_g;    // sqrt(k T_g / M)
  double sig_se;   // sqrt(e T_se / m_e)
  double half;     // L/2
  double eepf_hw;
  double inv_de;
  int nx;
  int ntab;
  int nbins;
  int parity;
  uint32_t step;
  uint32_t seed;
  uint32_t run;
  int no_coll;
  int record;
  int model;  // kModelAniso | kModelOpal
};
constexpr int kModelAniso = 1;  // anisotropic electron elastic scattering
constexpr int kModelOpal = 2;   // Opal energy sharing in ionization
constexpr double kOpalW = 10.0;  // eV, argon

struct SortArgs {
  const double* sx;  // input: x, v_x, pool index, pool
  const double* svx;
  const uint32_t* sid;
  const double* spvy;
  const double* spvz;
  double* dx;        // output in cell order, pool repacked in slot order
  double* dvx;
  uint32_t* did;
  double* dpvy;
  double* dpvz;
  int64_t* pool_n;       // set to the count
  const int64_t* count;  // device count of the species
  int64_t cap;           // capacity of src/dst
  uint32_t* cnt;         // [nkeys][nblocks]
  uint32_t* seg;         // scan segment sums (256)
  double inv_dx;
  int nx;
  int nblocks;
};

// host launchers
hipError_t launch_field(const FieldArgs& a, hipStream_t s);
// the field (workgroup 0) and the candidacy bits a.cand of the next step's
// electron slots (the other workgroups)
hipError_t launch_field_cand(const FieldArgs& a, int num_cu, hipStream_t s);
// grid and LDS bytes of one species' two particle kernels
// Compiled workgroup sizes of k_decide, the default first.
constexpr int kDecideBlocks[2] = {512, 256};

struct PartLaunch {
  int grid_decide[2];  // [measuring]
  size_t lds_decide[2];
  int grid_emit;
  size_t lds_emit;
  int grid_emit_decide;  // the electron emit fused with the next step's decisions
  size_t lds_emit_decide;
  int grid_emit_decide3;  // the same on input that still needs its push
  int bpc_emit_decide3;
  int grid_rare;
  int bpc_decide[2];   // resident workgroups per CU at these LDS sizes (occupancy)
  int decide_block;    // k_decide's threads per workgroup: one of its compiled sizes
  int bpc_decide_by[2][2];  // [default size, other size][measuring]: occupancy of each
  int bpc_emit;
  int bpc_emit_decide;
  int64_t max_tiles;
};
PartLaunch particle_launch_config(int species, int nx, int nbins, int num_cu, int64_t max_tiles);
// the same with k_decide at kd and k_emit at ke workgroups per CU (clamped
// to [1, occupancy] and to the tile count)
void particle_launch_set(PartLaunch& c, int num_cu, int kd, int ke);
// k_decide compiled for `threads` per workgroup (512 or 256), at the most
// workgroups per CU that fit; false (nothing changed) for any other size
bool particle_launch_block(PartLaunch& c, int num_cu, int threads);
// kernel 0: k_decide, 1: k_emit, 2: k_rare (launched in this order).
// flags (electrons only): kLaunchPushed, the emit and rare kernels take an
// input that holds the pushed state (the previous step's fused emit decided
// this step and stored it), with no second push.
constexpr int kLaunchPushed = 2;
hipError_t launch_particle_kernel(int kernel, int species, bool measure, const PartArgs& a,
                                  const PartLaunch& c, hipStream_t s, int flags = 0);
// field of the next step (one workgroup) together with the queued slots of
// this step's last particle pass of `species` (rare_blocks workgroups);
// pushed: electron slots whose input holds the pushed state
hipError_t launch_tail(int species, const FieldArgs& f, const PartArgs& a, int rare_blocks,
                       hipStream_t s, bool pushed = false);
// Electron pass a fused with the decisions of the next step b: the emit,
// the queued slots of a with their outputs decided for b, and the outputs
// whose decisions the streaming part deferred. pushed: a's input holds the
// pushed state (the previous pipelined step left it); otherwise it is pushed
// again here.
hipError_t launch_emit_decide(const PartArgs& a, const PartArgs& b, const PartLaunch& c,
                              hipStream_t s, bool pushed);
// Batched launches over n discharges (n <= kMaxBatch): args and f are
// arrays of argument blocks in device memory, one per discharge.
constexpr int kMaxBatch = 256;
struct BatchLaunch {
  int grid_decide[2][2];  // [species][measuring]
  size_t lds_decide[2][2];
  int grid_emit[2];
  size_t lds_emit;
  int grid_rare;
  int nx_max;
  int nbins_max;
};
// max_tiles: the largest number of tiles a pass of each species can have,
// summed over the discharges
BatchLaunch batch_launch_config(int nx_max, int nbins_max, int num_cu, const int64_t max_tiles[2]);
// variants: some discharge of the list uses a method variant (model != 0)
hipError_t launch_batch_pass(int kernel, int species, bool measure, const PartArgs* args, int n,
                             const BatchLaunch& c, hipStream_t s, bool variants);
hipError_t launch_batch_tail(int species, const FieldArgs* f, int nf, const PartArgs* args, int n,
                             int rare_blocks, hipStream_t s, bool variants);
hipError_t launch_batch_field(const FieldArgs* f, int n, hipStream_t s);
hipError_t launch_sort(const SortArgs& a, hipStream_t s);
// n independent sorts (args in device memory, each with its own counters);
// total_blocks = the sum of their nblocks, nx_max the largest nx
hipError_t launch_batch_sort(const SortArgs* args, int n, int64_t total_blocks, int nx_max,
                             hipStream_t s);
// pool repacked in slot order (no reordering of the slots)
hipError_t launch_repack(const SortArgs& a, hipStream_t s);
// id[i] = i for i < *count
hipError_t launch_iota(uint32_t* id, const int64_t* count, hipStream_t s);
// out_y[i] = vy[id[i]], out_z[i] = vz[id[i]] for i < n
hipError_t launch_gather(const uint32_t* id, const double* vy, const double* vz, double* out_y,
                         double* out_z, int64_t n, hipStream_t s);
hipError_t launch_deposit(const double* x, const int64_t* count, double inv_dx, int nx,
                          unsigned long long* dep, hipStream_t s);
// particles drawn from density and temperature profiles (pic_load_profile)
constexpr uint32_t kLoadStep = 0xFFFFFFFEu;  // counter word 0 of the loader's draws
constexpr int kMaxLoadPoints = 8192;
struct LoadArgs {
  const double* dens;  // npts points on [0, L], device
  const double* temp;  // temperature in eV at the same points, device
  double* x;
  double* vx;
  double* vy;
  double* vz;
  int64_t n;
  double L;
  double h;    // L / (npts - 1)
  double hh;   // h / 2
  double vfac; // e / m
  int npts;
  int species;
  uint32_t seed;
  uint32_t run;
};
hipError_t launch_load_profile(const LoadArgs& a, hipStream_t s);
hipError_t launch_selftest_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                                  int64_t n, hipStream_t s);
hipError_t launch_selftest_sqrt(const double* in, double* out, int64_t n, hipStream_t s);
hipError_t launch_selftest_copy(const double* in, double* out, int64_t n, hipStream_t s);

}  // namespace pic

struct pic_handle {
  pic_params p;
  pic_derived d;
  hipStream_t stream;
  int device;
  int num_cu;
  // derived constants
  int nx;
  double L, dx, inv_dx, dt, ng;
  double dts[2], acc[2], mass[2];
  double nfac32, qfac32, kpois;
  double inv_dv[2], numax[2], pcoll[2];
  double ek_e, ve_e, mr_e, mm_e, sig_g, sig_se, inv_de, eepf_de;
  double exc_thr, ion_thr;
  int ntab;
  std::vector<double> vtab;
  // device memory (carved from the caller's workspace)
  pic::DevCtl* ctl;
  double* part[2][2][2];  // [species][buffer][x, vx]
  uint32_t* pid[2][2];    // [species][buffer] pool index per slot
  double* pool[2][2][2];  // [species][buffer][vy, vz]
  int64_t pcap[2];        // pool entries per buffer
  uint8_t* codes[2][2];  // per species, two buffers used by alternate passes
  int csel[2];           // the code buffer of the next pass of each species
  uint64_t* tcnt[2][2];  // per species, two buffers used by alternate passes
  int tsel[2];           // the buffer the next pass of each species adds into
  uint4* rq[2];
  int64_t max_tiles[2];
  int64_t* dep_e[2];
  int64_t* dep_i[2];
  double* rho;
  double* phi;
  double* Ebuf[2];  // E of even and odd steps
  int e_last;       // buffer of the last field solved
  double* cum[2];
  double* th_cp;
  double* th_m;
  double* acc_ne;
  double* acc_ni;
  double* acc_w;
  double* acc_ew;
  unsigned long long* eepf;
  unsigned long long* fedf[2];  // [species]: [wall][eepf_bins] arrivals per energy bin
  double fedf_emax[2];          // upper edge of the arrival energy bins, eV
  uint32_t* sort_cnt;
  uint32_t* sort_seg;
  uint32_t* cand;  // candidacy bits of a pipelined step's electron slots
  uint32_t* dq;    // slots of a pipelined step whose decisions are deferred
  int sort_blocks;
  // host-side schedule state
  int64_t step;
  int cur[2];
  int pcur[2];  // active pool buffer per species
  int cur_hi;
  int e_decided;  // the last step decided the next step's electrons (pipelined)
  int pipeline;   // pipelined electron steps allowed (pic_set_pipeline)
  int measuring;
  int field_fixed_set;
  pic::PartLaunch launch[2];  // [species]
  // opt-in kernel timing: event pairs recorded around launches
  int timing;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;  // (timer, index of start event)
  size_t ev_next = 0;                        // event pairs handed out since the last fold
  double t_ms[PIC_NTIMERS];
  int64_t t_n[PIC_NTIMERS];
};
