/*
 * libpic — explicit 1D3V electrostatic PIC/MCC of an RF capacitively coupled
 * argon discharge on one MI355X (gfx950), behind a plain C ABI.
 *
 * The method is the six-step cycle of Vass, Palla & Hartmann,
 * "Revisiting the numerical stability/accuracy conditions of explicit
 * PIC/MCC simulations of low-temperature gas discharges" (arXiv:2109.04469),
 * Sec. 2 (computational method) with the surface model of Sec. 2 step 5 and
 * the collision step of Sec. 2 step 6; the problem parameters are those of
 * Sec. 3, Table 1.
 *
 * Conventions for every entry point below
 *  - Return value: int32 status, PIC_OK (0) or one of the negative PIC_E*
 *    codes. No C++ exception or longjmp crosses this boundary.
 *  - Memory: libpic never allocates or frees device memory. The caller
 *    allocates ONE device workspace of the size pic_workspace_bytes() reports
 *    and keeps it alive until pic_free(). Host metadata (the handle) is
 *    malloc'd by pic_init and released by pic_free.
 *  - Streams: every device operation is enqueued on the hipStream_t given to
 *    pic_init (NULL = the legacy default stream). pic_step is asynchronous;
 *    the calls documented as "synchronises" wait for that stream.
 *  - Errors found on the device (non-finite state, capacity overflow) are
 *    latched in a device error word and
 *    returned by the next synchronising call. After a latched error the
 *    particle state is unspecified; recover with pic_set_state.
 *  - A handle may be used by one host thread at a time.
 *  - Units: SI unless the name says otherwise (_ev = electronvolt).
 */
#ifndef LIBPIC_PIC_H
#define LIBPIC_PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PIC_OK          0
#define PIC_EINVAL     -1 /* bad argument or parameter set                    */
#define PIC_EHIP       -2 /* a HIP runtime call failed (no GPU, launch error) */
#define PIC_ECAPACITY  -3 /* a species outgrew its capacity                   */
#define PIC_EUNSTABLE  -4 /* a non-finite position, velocity or field value   */
#define PIC_ETABLE     -5 /* reserved (speeds beyond a table are counted, see
                             PIC_CNT_BEYOND_TABLE)                            */
#define PIC_ESTATE     -6 /* call not valid in the handle's current state     */

/* ---- species ----------------------------------------------------------- */
#define PIC_ELECTRON 0
#define PIC_ION      1 /* Ar+ */

/* ---- test-mode flags (pic_params.flags) --------------------------------- */
#define PIC_FLAG_NO_FIELD       (1u << 0) /* E = 0 everywhere, no Poisson solve */
#define PIC_FLAG_FIXED_E        (1u << 1) /* E held at the array of pic_set_field */
#define PIC_FLAG_NO_COLL        (1u << 2) /* skip the collision step            */
#define PIC_FLAG_IMMOBILE_IONS  (1u << 3) /* ions never pushed nor collided     */
#define PIC_FLAG_RECORD         (1u << 4) /* keep per-slot decision codes       */
#define PIC_FLAG_THOMAS         (1u << 5) /* solve Poisson with the serial Thomas
                                             recurrence instead of the exact
                                             integer prefix-sum form           */
/* method variants (not in the paper, whose scattering is isotropic and whose
 * ionization shares the energy uniformly): */
#define PIC_FLAG_ANISO_ELASTIC  (1u << 6) /* electron elastic scattering with the
   screened-Coulomb angular distribution of Vahedi & Surendra (1995):
   cos chi = (2 + eps - 2 (1 + eps)^u) / eps, eps the electron energy in eV,
   about the incident direction, azimuth uniform, in the two-body frame   */
#define PIC_FLAG_OPAL_SHARING   (1u << 7) /* ionization energy shared as in Opal,
   Peterson & Beaty (1971): the ejected electron takes
   eps_ej = w tan(u atan(eps' / (2 w))), w = 10 eV (argon), eps' the energy
   above threshold; the scattered one the rest                            */

/* ---- event counters (pic_get_counters), accumulated since pic_set_state --- */
enum {
  PIC_CNT_STEPS = 0,
  PIC_CNT_E_PUSHED,      /* electron particle-steps                          */
  PIC_CNT_I_PUSHED,      /* ion particle-steps (sub-cycled steps only)       */
  PIC_CNT_E_ABSORBED,
  PIC_CNT_E_REFLECTED,
  PIC_CNT_I_ABSORBED,
  PIC_CNT_SE_EMITTED,
  PIC_CNT_E_CANDIDATES,  /* null-collision candidates                        */
  PIC_CNT_E_ELASTIC,
  PIC_CNT_E_EXCITATION,
  PIC_CNT_E_IONIZATION,
  PIC_CNT_I_CANDIDATES,
  PIC_CNT_I_ISOTROPIC,
  PIC_CNT_I_BACKWARD,
  PIC_CNT_REFLECT_LOST,  /* reflected but still outside: removed             */
  PIC_CNT_BEYOND_TABLE,  /* candidates faster than the last table speed: the
                            last table entry is used                        */
  PIC_NCOUNTERS
};

/* ---- per-slot decision code (pic_get_decisions), one byte per slot ------
 * bits 0..2  wall outcome: 0 inside, 1 absorbed, 2 reflected,
 *            3 absorbed and emitted a secondary electron, 4 reflected but
 *            still outside (removed)
 * bits 3..5  collision: 0 not a candidate, 1 null, 2 first process
 *            (e: elastic, Ar+: isotropic), 3 second (e: excitation,
 *            Ar+: backward), 4 third (e: ionization)
 * bit  7     slot was pushed this step                                      */

typedef struct pic_params {
  /* discharge (Sec. 2 and Table 1) */
  double   gap_m;            /* L, electrode gap                               */
  double   pressure_pa;      /* p                                              */
  double   gas_temp_k;       /* T_g                                            */
  double   rf_voltage_v;     /* phi_0: V(t) = phi_0 cos(2 pi f t) on x = 0     */
  double   rf_freq_hz;       /* f                                              */
  int32_t  steps_per_cycle;  /* N_t: dt = 1/(f N_t)                            */
  int32_t  n_cells;          /* N_x - 1: dx = L/n_cells, N_x grid points       */
  double   weight;           /* W, real particles per superparticle            */
  double   area_m2;          /* nominal electrode area (1 cm^2 in the paper)   */
  double   reflection;       /* R, electron reflection probability            */
  double   gamma_see;        /* gamma, secondary emission yield per ion impact */
  double   see_temp_ev;      /* temperature of emitted secondary electrons     */
  /* capacities and schedule */
  int64_t  capacity[2];      /* max superparticles per species (e, Ar+)        */
  int32_t  ion_subcycle;     /* k >= 1: ions advance on steps n % k == 0 with k dt */
  int32_t  sort_interval;    /* cell sort after every K-th step (0 = never)    */
  /* counter-based random streams: key = (seed, run) */
  uint32_t seed;
  uint32_t run;
  /* diagnostics (Sec. 3.1: EEPF at the discharge centre) */
  int32_t  eepf_bins;        /* >= 1                                           */
  double   eepf_emax_ev;     /* histogram covers [0, eepf_emax_ev)             */
  double   eepf_halfwidth_m; /* electrons with |x - L/2| <= halfwidth count    */
  uint32_t flags;            /* PIC_FLAG_*                                     */
} pic_params;

/* Collision cross sections (Sec. 2 step 6), host arrays in m^2, tabulated at
 * the speeds v_k = k * dv for k = 0..n-1. Electron tables are indexed by the
 * electron speed, ion tables by the ion-atom relative speed (lab energy
 * 1/2 M g^2). Copied at pic_init; the caller keeps ownership. */
typedef struct pic_xsec {
  int32_t        n;                 /* entries per table, >= 2               */
  double         dv_e;              /* electron table speed step, m/s        */
  double         dv_i;              /* ion table speed step, m/s             */
  const double*  sigma_e[3];        /* elastic, excitation, ionization       */
  const double*  sigma_i[2];        /* isotropic elastic, backward (charge transfer) */
  double         exc_threshold_ev;  /* energy lost in excitation             */
  double         ion_threshold_ev;  /* energy lost in ionization             */
} pic_xsec;

/* Quantities derived at pic_init (host), for inspection. */
typedef struct pic_derived {
  int32_t n_x;          /* grid points                                      */
  int32_t n_tiles_max;  /* particle tiles at full capacity (largest species) */
  double  dx;           /* L/(N_x - 1)                                      */
  double  dt;           /* 1/(f N_t)                                        */
  double  gas_density;  /* p/(k_B T_g)                                      */
  double  nu_max[2];    /* max total collision frequency per species, 1/s   */
  double  p_coll[2];    /* 1 - exp(-nu_max dt_s), Sec. 3.5                  */
} pic_derived;

/* Time-averaged moments (Sec. 3.1). Host arrays owned by the caller; any
 * pointer may be NULL to skip that output. */
typedef struct pic_moments_out {
  double*  n_e;           /* [N_x] electron density, m^-3                   */
  double*  n_i;           /* [N_x] ion density, m^-3                        */
  double*  mean_energy_e; /* [N_x] CIC-weighted mean electron energy, eV    */
  double*  eepf;          /* [eepf_bins] EEPF at L/2, eV^-3/2, normalised so
                             that sum_b sqrt(eps_b) f_b d(eps) = 1          */
  int64_t  steps_averaged;
} pic_moments_out;

/* Electrode diagnostics over the measured steps (Sec. 3.3: the mean ion
 * flux to the electrodes and the flux-energy distributions of electrons and
 * ions arriving there). Index [s][w]: species s (0 e-, 1 Ar+), electrode w
 * (0: x = 0, driven; 1: x = L, grounded). An arrival is a particle that
 * leaves the gap through the electrode in a push; electrons that are then
 * reflected count as arrivals but not as absorbed. Its impact energy is
 * (m/2)|v|^2 with the pushed velocity. fedf[s][w]: caller-owned host arrays
 * of fedf_bins values (or NULL), f(eps) in eV^-1 normalised so that the sum
 * over bins of f d(eps) is 1 (arrivals above fedf_emax_ev count in the
 * fluxes and mean energies but not in f); bins of width fedf_emax_ev[s] /
 * fedf_bins, fedf_emax_ev = eepf_emax_ev for electrons and
 * max(1.25 phi_0, 10 eV) for ions, fedf_bins = eepf_bins. */
typedef struct pic_wall_out {
  int64_t  arrivals[2][2];
  int64_t  absorbed[2][2];
  double   flux[2][2];            /* arrivals per m^2 per s                    */
  double   absorbed_flux[2][2];   /* absorptions per m^2 per s                 */
  double   mean_energy_ev[2][2];  /* mean impact energy                        */
  double*  fedf[2][2];
  double   fedf_emax_ev[2];
  int32_t  fedf_bins;
  int64_t  ionizations;           /* electron-impact ionizations, same steps   */
  double   ionization_rate;       /* per m^2 per s: in a steady state it equals
                                     the ion flux absorbed at both electrodes  */
  int64_t  steps_averaged;
} pic_wall_out;

/* Stability and accuracy monitors of Sec. 3.5 from the time averages. */
typedef struct pic_monitors {
  double  omega_pe_dt;           /* sqrt(e^2 n_max / (eps0 m_e)) dt, n_max the
                                    largest time-averaged electron density     */
  double  p_coll[2];             /* 1 - exp(-nu_max dt_s) per species          */
  double  n_e_max;
  double  n_e_center;            /* time-averaged n_e at L/2, m^-3             */
  double  mean_energy_center_ev; /* CIC-weighted mean electron energy at L/2   */
  double  lambda_d_m;            /* sqrt(eps0 T_e / (e n_e)) at L/2,
                                    T_e = (2/3) <eps> in eV                    */
  double  dx_over_lambda_d;
  double  n_d;                   /* superparticles per Debye length at L/2:
                                    n_e A lambda_D / W                         */
  int64_t steps_averaged;
} pic_monitors;

typedef struct pic_handle pic_handle;

/* Size of the single device workspace for parameter set *p (capacities, grid,
 * tables). Returns PIC_EINVAL for an invalid parameter set. */
int pic_workspace_bytes(const pic_params* p, const pic_xsec* xs, uint64_t* bytes);

/* Validates *p and *xs, derives dx, dt, gas density, the cumulative
 * collision-frequency tables and P_coll per species (Sec. 2, Sec. 3.5),
 * builds the RF voltage table V_n = phi_0 cos(2 pi n / N_t), lays out the
 * caller's device workspace (at least pic_workspace_bytes, 256-byte aligned)
 * and zeroes it. Both species start empty at step 0. stream is a
 * hipStream_t. Synchronises. On success *out owns host metadata only. */
int pic_init(const pic_params* p, const pic_xsec* xs, void* workspace,
             uint64_t workspace_bytes, void* stream, pic_handle** out);

/* Replaces the particles of one species with n superparticles: positions x
 * in [0, L] and velocities (vx, vy, vz) taken as v at the half step before
 * `step` (leap-frog staggering, Sec. 2 step 4). Arrays are SoA of n doubles,
 * host or device pointers (the copy direction is inferred). Sets the step
 * counter of the handle to `step` for both species, clears the event
 * counters and latched errors, and recomputes the charge deposit of both
 * species. Synchronises. PIC_ECAPACITY if n > capacity. */
int pic_set_state(pic_handle* h, int species, const double* x, const double* vx,
                  const double* vy, const double* vz, int64_t n, int64_t step);

/* Copies the current particles of one species into caller arrays of
 * `cap` doubles each (host or device). *n receives the count; if the count
 * exceeds cap nothing is copied and PIC_ECAPACITY is returned. *step (may be
 * NULL) receives the step counter. Synchronises and reports latched errors. */
int pic_get_state(pic_handle* h, int species, double* x, double* vx, double* vy,
                  double* vz, int64_t cap, int64_t* n, int64_t* step);

/* Enqueues n_steps steps of the cycle of Sec. 2: deposit (1), Poisson with
 * Dirichlet walls phi(0) = V(t), phi(L) = 0 and field (2), gather (3),
 * leap-frog push (4), wall absorption / reflection / secondary emission (5),
 * null-collision MCC (6); survivors compacted in slot order, births appended;
 * cell sort every sort_interval steps. Asynchronous: returns after enqueueing;
 * errors of earlier steps are reported by the next synchronising call. */
int pic_step(pic_handle* h, int64_t n_steps);

/* Waits for the stream and returns the first latched device error, if any. */
int pic_sync(pic_handle* h);

/* Sets the field used by PIC_FLAG_FIXED_E runs: N_x doubles (host or
 * device), V/m. Synchronises. PIC_ESTATE if the flag is not set. */
int pic_set_field(pic_handle* h, const double* E);

/* Copies the charge density rho, potential phi and field E of the most
 * recent field solve (N_x doubles each, host or device; NULL skips; under
 * PIC_FLAG_NO_FIELD or PIC_FLAG_FIXED_E phi is 0) and the integer CIC
 * deposits of the current particles of both species, i.e. the input of the
 * next solve (N_x int64 each, units of 2^-32 superparticle; NULL skips).
 * Synchronises. */
int pic_get_field(pic_handle* h, double* rho, double* phi, double* E,
                  int64_t* deposit_e, int64_t* deposit_i);

/* Starts (on != 0) or stops accumulation of the time-averaged moments. Each
 * step taken while on contributes its densities at the start of the step and
 * the electron energies from the half-step velocities. */
int pic_measure(pic_handle* h, int on);

/* Reads the time-averaged moments; reset != 0 clears the accumulators
 * afterwards. Synchronises. */
int pic_moments(pic_handle* h, pic_moments_out* out, int reset);

/* Electrode fluxes, impact energies and flux-energy distributions over the
 * steps measured since the last pic_moments reset (which clears these too).
 * Synchronises. */
int pic_wall_moments(pic_handle* h, pic_wall_out* out);

/* omega_pe dt, P_coll, Debye length, dx / lambda_D and the superparticles
 * per Debye length (Sec. 3.5) from the current time averages. At the centre
 * L/2: the middle grid point, or the mean of the two middle points for an
 * even number of points. Synchronises. */
int pic_get_monitors(pic_handle* h, pic_monitors* out);

/* Copies the PIC_NCOUNTERS event counters (host int64 array). Synchronises. */
int pic_get_counters(pic_handle* h, int64_t* counters);

/* With PIC_FLAG_RECORD: copies the decision codes of the last step for the
 * slots that existed at its start (host or device buffer of `cap` bytes).
 * *n receives the number of slots. Synchronises. */
int pic_get_decisions(pic_handle* h, int species, uint8_t* codes, int64_t cap, int64_t* n);

/* Advances n independent discharges by n_steps each. Each handle's steps
 * are enqueued on its own stream (the one given to pic_init) in chunks of
 * `chunk` steps (chunk >= 1), round robin over the handles, so that
 * discharges on different streams run concurrently on the GPU: a parameter
 * sweep of the kind of Sec. 3 (N_t, N_x, W, R, gamma, pressure, voltage)
 * advanced as one batch. Every discharge computes exactly what pic_step on
 * it alone computes. Does not synchronise; errors of one handle stop the
 * enqueueing and are returned. Handles must be distinct. */
int pic_step_many(pic_handle* const* handles, int n, int64_t n_steps, int64_t chunk);

/* ---- batched launches --------------------------------------------------
 * A batch advances n independent discharges (1 <= n <= 256, the same sweep
 * as above) in lockstep with ONE launch per particle pass, field solve and
 * tail for all of them: the kernels lay the discharges' particle tiles end
 * to end, so that small discharges fill the GPU together instead of one at
 * a time, and the launch count per step does not grow with n. The cell
 * sorts stay per discharge.
 *  - Handles: distinct, created on the same device with the same stream;
 *    the batch enqueues everything on that stream. While a batch is in use
 *    the handles may still be used one at a time (pic_step, pic_get_state,
 *    ...); the batch only borrows them during pic_batch_step.
 *  - Memory: the caller allocates a device workspace of
 *    pic_batch_workspace_bytes() (256-byte aligned), where the per-step
 *    kernel argument blocks go; the batch itself allocates two pinned host
 *    staging buffers of half that size (released by pic_batch_free) and no
 *    device memory.
 *  - Results: every discharge computes exactly what pic_step on it alone
 *    computes (bitwise). Device errors are latched per handle and returned
 *    by pic_sync on that handle. Event timers (pic_timing) cover the sorts
 *    only when stepping through a batch. */
typedef struct pic_batch pic_batch;

/* Workspace bytes of a batch of these handles. */
int pic_batch_workspace_bytes(pic_handle* const* handles, int n, uint64_t* bytes);

/* Creates a batch over the handles (borrowed, not owned: free the batch
 * before the handles). PIC_EINVAL on a bad handle list or workspace. */
int pic_batch_create(pic_handle* const* handles, int n, void* workspace, uint64_t workspace_bytes,
                     pic_batch** out);

/* Advances every discharge of the batch by n_steps. Asynchronous on the
 * batch's stream, except that it waits for the GPU to have read the argument
 * blocks of the previous chunk of steps (64 steps or fewer per chunk) before
 * reusing their host buffer. */
int pic_batch_step(pic_batch* b, int64_t n_steps);

/* Synchronises the batch's stream and releases its host memory. */
void pic_batch_free(pic_batch* b);

/* Launch shape of the particle kernels: decide_wg_per_cu and
 * emit_wg_per_cu workgroups per compute unit for the decide and emit
 * kernels of both species (clamped to [1, what fits on a CU] and to the tile
 * count; the default is the most that fits). Results do not depend on it:
 * the tiles and every per-slot decision are the same for any grid. */
int pic_set_launch(pic_handle* h, int decide_wg_per_cu, int emit_wg_per_cu);

/* Pipelined electron steps on (1, the default) or off (0). On, within one
 * pic_step call the electron emit of a step also takes the next step's
 * electron decisions (push, candidacy, walls, collision process, deposit),
 * so that step has no decide pass of its own; this applies to steps that
 * are not the last of the call, not ion steps, not followed by a cell sort
 * or pool repack and not measuring. The arithmetic is the same: results are
 * identical bit for bit either way (Sec. 2 defines one step; the pipeline
 * only regroups its work across kernels). */
int pic_set_pipeline(pic_handle* h, int on);

/* Workgroup size of the decide kernels (both species): one of the compiled
 * sizes, 512 threads (the default) or 256 threads; each takes the same tiles
 * of 2048 slots, in runs of four consecutive slots per thread, so results do
 * not depend on it. The decide workgroups per CU return to the most that
 * fit at that size (pic_set_launch changes them). PIC_EINVAL for any other
 * size. Steps taken through a batch (pic_batch_step) use the
 * batched kernels, whose size is fixed at 512. */
int pic_set_decide_block(pic_handle* h, int threads);

/* Picks the launch shape by measurement: advances the discharge by
 * steps_per_trial steps per candidate (every decide shape, then every emit
 * shape), timing the electron decide and emit kernels with events, and keeps
 * the fastest; the chosen shape is returned through the pointers (may be
 * NULL). The steps are ordinary steps of the discharge. Synchronises. */
int pic_tune(pic_handle* h, int64_t steps_per_trial, int* decide_wg_per_cu, int* emit_wg_per_cu);

/* One candidate configuration of the particle passes that pic_tune_pass
 * timed: the electron schedule (pic_set_pipeline), the decide kernels'
 * compiled workgroup size (pic_set_decide_block), the launch shape
 * (pic_set_launch) and the measured time of the particle passes (electron
 * and ion passes with their kernels back to back, PIC_TIMER_ELECTRON +
 * PIC_TIMER_ION) per step, microseconds. */
typedef struct {
  int pipeline;
  int decide_block;
  int decide_wg_per_cu;
  int emit_wg_per_cu;
  double us_per_step;
} pic_pass_trial;

/* Chooses the particle passes' compiled kernels and launch shape by
 * measurement on the discharge itself: pipelined electron steps (the fused
 * emit-and-decide kernel) at each of its workgroups per CU, then unpipelined
 * steps (separate decide and emit kernels) with the decide kernel at each
 * compiled workgroup size (512 and 256 threads) and each of its shapes, then
 * each emit shape at the best decide. Each candidate advances the
 * discharge by steps_per_trial ordinary steps with events around the
 * passes; the fastest is kept (pic_set_pipeline, pic_set_decide_block,
 * pic_set_launch). trials: a
 * caller-owned host array of max_trials entries (NULL with max_trials 0)
 * that receives the candidates in the order timed; n_trials: their count;
 * best: the index of the chosen one (both may be NULL). Results do not
 * depend on the choice: every candidate computes the same steps bit for bit
 * (Sec. 2 defines one step; the candidates regroup its work). Synchronises;
 * on an error the schedule is left as it was. */
int pic_tune_pass(pic_handle* h, int64_t steps_per_trial, pic_pass_trial* trials, int max_trials,
                  int* n_trials, int* best);

/* Kernel timing with HIP events recorded on the handle's stream
 * (measurement surface). level 0: off. level 1: two event records around
 * the field kernel, each species' particle pass (PIC_TIMER_ELECTRON,
 * PIC_TIMER_ION: its decide, emit and rare kernels back to back, the gaps
 * between them included) and each species' cell sort (PIC_TIMER_SORT).
 * level 2: also around every single particle kernel (the _DECIDE, _EMIT and
 * _RARE timers); the extra records delay the launches they separate, so the
 * pass timers of level 2 read high. */
enum {
  PIC_TIMER_FIELD = 0,
  PIC_TIMER_ELECTRON,
  PIC_TIMER_ION,
  PIC_TIMER_SORT,
  PIC_TIMER_E_DECIDE,
  PIC_TIMER_E_EMIT,
  PIC_TIMER_E_RARE,
  PIC_TIMER_I_DECIDE,
  PIC_TIMER_I_EMIT,
  PIC_TIMER_I_RARE,
  PIC_NTIMERS
};
int pic_timing(pic_handle* h, int level);

/* Synchronises and returns, per timer, the summed kernel time in ms
 * (ms[PIC_NTIMERS]) and the number of timed launches (launches[PIC_NTIMERS]);
 * reset != 0 clears them. */
int pic_get_timing(pic_handle* h, double* ms, int64_t* launches, int reset);

/* Copies the derived quantities of pic_init (host). */
int pic_get_derived(const pic_handle* h, pic_derived* d);

/* Releases host metadata. The workspace stays the caller's. Waits for the
 * stream first. NULL is ignored. */
void pic_free(pic_handle* h);

/* Static string describing a status code. */
const char* pic_strerror(int status);

/* ---- self-checks of device arithmetic (test surface) ---------------------
 * Philox4x32-10 (Salmon et al., SC'11) evaluated on the device for n
 * counters: ctr and out are device arrays of 4n uint32, key is 2 host
 * uint32. The method's random decisions (Sec. 2 steps 5 and 6) draw from
 * this generator keyed by (seed, run) with counter (step, slot,
 * 16*species + purpose, 0); the collision-candidacy uniform of slot i is
 * word i mod 4 of the block (step, i / 4, 16*species + 4, 0). Runs on
 * `stream` (a hipStream_t) and synchronises it. */
int pic_selftest_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n,
                        void* stream);

/* FP64 square root of n device doubles on the device (the wall and
 * collision decisions rely on it being correctly rounded). Synchronises. */
int pic_selftest_sqrt(const double* in, double* out, int64_t n, void* stream);

/* Plain device-to-device copy of n doubles (n even, both arrays 16-byte
 * aligned, not overlapping): the reference streaming kernel against which
 * the particle kernels' bandwidth and HBM traffic counters are read. Only
 * enqueued on `stream`; does not synchronise. */
int pic_selftest_copy(const double* in, double* out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBPIC_PIC_H */
