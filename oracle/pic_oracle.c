/*
 * Plain CPU oracle of the explicit 1D3V electrostatic PIC/MCC cycle for an
 * RF capacitively coupled argon discharge: Vass, Palla, Hartmann,
 * arXiv:2109.04469, Sec. 2 (the six steps executed in order every time
 * step), with the parameters of Sec. 3 / Table 1.
 *
 * TEST INFRASTRUCTURE ONLY. This library is loaded by the tests, the smoke
 * check and the benchmark's CPU-baseline leg, never by the simulation
 * library. It is single-threaded FP64 (IEEE round to nearest, built with
 * -ffp-contract=off) and runs each step of the method as a plain loop in the
 * order the paper lists them. Where the paper leaves a choice open, the
 * reading taken is stated next to the code (the design notes list them all).
 *
 * Random numbers: Philox4x32-10 keyed by (seed, run) with counter
 * (step, slot, 16*species + purpose, 0); u32 r -> (r + 1/2) 2^-32. The
 * collision-candidacy uniform, the one draw every particle needs every step,
 * is word (slot mod 4) of the block with counter (step, slot / 4,
 * 16*species + 4, 0), so one block serves four consecutive slots. The paper
 * draws from MT19937 (Sec. 2 step 5); a counter-based stream keyed by slot
 * gives every particle-step its own draws independent of execution order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* CODATA 2018 */
#define Q_E 1.602176634e-19
#define MASS_E 9.1093837015e-31
#define AMU 1.66053906660e-27
#define EPS0 8.8541878128e-12
#define K_B 1.380649e-23
#define TWO_PI 6.283185307179586
#define TWO32 4294967296.0
#define INV_TWO32 2.3283064365386963e-10 /* 2^-32 */

/* status codes, same numbering as the library's */
#define ORA_OK 0
#define ORA_EINVAL -1
#define ORA_ECAPACITY -3
#define ORA_EUNSTABLE -4

/* flags */
#define F_NO_FIELD 1u
#define F_FIXED_E 2u
#define F_NO_COLL 4u
#define F_IMMOBILE_IONS 8u
#define F_RECORD 16u
#define F_ANISO 64u /* screened-Coulomb electron elastic scattering (variant) */
#define F_OPAL 128u /* Opal et al. ionization energy sharing (variant) */
#define OPAL_W 10.0 /* eV, argon */

enum { C_STEPS = 0, C_E_PUSHED, C_I_PUSHED, C_E_ABSORBED, C_E_REFLECTED, C_I_ABSORBED,
       C_SE_EMITTED, C_E_CAND, C_E_ELASTIC, C_E_EXC, C_E_ION, C_I_CAND, C_I_ISO, C_I_BACK,
       C_REFLECT_LOST, C_BEYOND, NCOUNT };

typedef struct {
  double gap_m, pressure_pa, gas_temp_k, rf_voltage_v, rf_freq_hz;
  int32_t steps_per_cycle, n_cells;
  double weight, area_m2, reflection, gamma_see, see_temp_ev;
  int64_t capacity[2];
  int32_t ion_subcycle, sort_interval;
  uint32_t seed, run;
  int32_t eepf_bins;
  double eepf_emax_ev, eepf_halfwidth_m;
  uint32_t flags;
  int32_t ntab;
  double dv_e, dv_i;
  double exc_threshold_ev, ion_threshold_ev;
} ora_params;

typedef struct {
  int64_t n, cap;
  double *x, *vx, *vy, *vz;
} ora_species;

typedef struct {
  ora_params p;
  /* derived (Sec. 2) */
  int32_t nx;
  double L, dx, inv_dx, dt, ng, mass[2], dts[2], acc[2];
  double nfac32, qfac32;
  double inv_dv[2], numax[2], pcoll[2];
  double *cum[2][3]; /* cumulative collision frequency tables */
  int nproc[2];
  double *vtab;
  double ek_e, ve_e, mr_e, mm_e, sig_g, sig_se, inv_de, eepf_de;
  /* state */
  ora_species sp[2];
  int64_t step;
  int64_t *dep[2];
  double *rho, *phi, *E;
  /* diagnostics */
  int measuring;
  int64_t msteps;
  double *acc_ne, *acc_ni, *acc_ew, *acc_w;
  int64_t *eepf_h;
  /* electrode arrivals while measuring, [species][wall], wall 0 at x = 0 */
  int64_t wall_hits[2][2], wall_abs[2][2], ioniz_meas;
  double wall_esum[2][2];
  int64_t *fedf[2];  /* [wall][eepf_bins] per species */
  double fedf_emax[2], ek[2];
  int64_t counters[NCOUNT];
  uint8_t *codes[2];
  int64_t ncodes[2];
  int err;
} ora_sim;

/* ------------------------------------------------------------------------ */
/* random numbers                                                           */

static void draw(const ora_sim* s, int64_t slot, int species, int purpose, uint32_t r[4]) {
  uint32_t ctr[4] = {(uint32_t)s->step, (uint32_t)slot, (uint32_t)(16 * species + purpose), 0u};
  uint32_t key[2] = {s->p.seed, s->p.run};
  ora_philox4x32_10(ctr, key, r);
}

static double u01(uint32_t r) { return ((double)r + 0.5) * INV_TWO32; }

/* collision-candidacy word of a slot (purpose 4, shared by four slots) */
static uint32_t candidacy_word(const ora_sim* s, int64_t slot, int species) {
  uint32_t ctr[4] = {(uint32_t)s->step, (uint32_t)(slot >> 2), (uint32_t)(16 * species + 4), 0u};
  uint32_t key[2] = {s->p.seed, s->p.run};
  uint32_t r[4];
  ora_philox4x32_10(ctr, key, r);
  return r[slot & 3];
}

/* Box-Muller: two standard normals from two uniforms in (0, 1). */
static void box_muller(double u1, double u2, double* a, double* b) {
  double rad = sqrt(-2.0 * log(u1));
  double th = TWO_PI * u2;
  *a = rad * cos(th);
  *b = rad * sin(th);
}

/* Isotropic unit vector: cos(chi) uniform on (-1, 1), azimuth uniform. */
static void iso_dir(double ua, double ub, double* nx, double* ny, double* nz) {
  double cth = 1.0 - 2.0 * ua;
  double sth = 2.0 * sqrt(ua * (1.0 - ua));
  double ph = TWO_PI * ub;
  *nx = cth;
  *ny = sth * cos(ph);
  *nz = sth * sin(ph);
}

/* Variant of the electron elastic scattering direction (Vahedi & Surendra,
 * 1995): deflection chi from the incident direction e (unit vector) with
 * cos chi = (2 + eps - 2 (1 + eps)^u) / eps for energy eps in eV (uniform
 * in (-1, 1) at eps = 0), azimuth phi = 2 pi w measured in the plane normal
 * to e from b1 = unit(e x a) towards b2 = e x b1, where a is the x axis, or
 * the y axis when |e_x| >= 0.9. */
static void deflect(double ex, double ey, double ez, double eps, double u, double w, double* nx,
                    double* ny, double* nz) {
  double c;
  if (eps > 0.0)
    c = (2.0 + eps - 2.0 * pow(1.0 + eps, u)) / eps;
  else
    c = 1.0 - 2.0 * u;
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  double s2 = 1.0 - c * c;
  double sn = sqrt(s2 > 0.0 ? s2 : 0.0);
  double ph = TWO_PI * w;
  double b1[3];
  if (fabs(ex) < 0.9) {
    double r = sqrt(ey * ey + ez * ez);
    b1[0] = 0.0;
    b1[1] = ez / r;
    b1[2] = -ey / r;
  } else {
    double r = sqrt(ez * ez + ex * ex);
    b1[0] = -ez / r;
    b1[1] = 0.0;
    b1[2] = ex / r;
  }
  double b2[3] = {ey * b1[2] - ez * b1[1], ez * b1[0] - ex * b1[2], ex * b1[1] - ey * b1[0]};
  double cp = cos(ph), sp = sin(ph);
  *nx = c * ex + sn * (cp * b1[0] + sp * b2[0]);
  *ny = c * ey + sn * (cp * b1[1] + sp * b2[1]);
  *nz = c * ez + sn * (cp * b1[2] + sp * b2[2]);
}

/* ------------------------------------------------------------------------ */
/* grid helpers: linear shape of total width 2 dx (Sec. 2 step 1)           */

/* Cell index j in [0, N_x - 2] and the fixed-point weight w1 (units of
 * 2^-32) of node j+1; node j receives 2^32 - w1. */
void ora_cell(int32_t nx, double inv_dx, double x, int64_t* j_out, double* f_out, int64_t* w1_out) {
  double t = x * inv_dx;
  int64_t j = (int64_t)t;
  if (j > nx - 2) j = nx - 2;
  if (j < 0) j = 0;
  double f = t - (double)j;
  int64_t w1 = (int64_t)floor(f * TWO32 + 0.5);
  if (w1 < 0) w1 = 0;
  if (w1 > (int64_t)4294967296LL) w1 = (int64_t)4294967296LL;
  *j_out = j;
  *f_out = f;
  *w1_out = w1;
}

/* Step 1: charge assignment. dep[j] = sum over particles of their weight at
 * node j in units of 2^-32 superparticle (exact integer sums). */
void ora_deposit_array(int32_t nx, double inv_dx, int64_t n, const double* x, int64_t* dep) {
  memset(dep, 0, sizeof(int64_t) * (size_t)nx);
  /* integer sums: any order (threads of an OpenMP build) gives the same */
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : dep[:nx])
#endif
  for (int64_t i = 0; i < n; i++) {
    int64_t j, w1;
    double f;
    ora_cell(nx, inv_dx, x[i], &j, &f, &w1);
    dep[j] += (int64_t)4294967296LL - w1;
    dep[j + 1] += w1;
  }
}

/* Textbook Thomas algorithm for a_i y_{i-1} + b_i y_i + c_i y_{i+1} = d_i,
 * i = 0..n-1 (a_0 and c_{n-1} unused): forward elimination, back
 * substitution. */
void ora_thomas(int64_t n, const double* a, const double* b, const double* c, const double* d,
                double* y) {
  if (n <= 0) return;
  double* cp = (double*)malloc(sizeof(double) * (size_t)n);
  double* dp = (double*)malloc(sizeof(double) * (size_t)n);
  cp[0] = c[0] / b[0];
  dp[0] = d[0] / b[0];
  for (int64_t i = 1; i < n; i++) {
    double m = b[i] - a[i] * cp[i - 1];
    cp[i] = c[i] / m;
    dp[i] = (d[i] - a[i] * dp[i - 1]) / m;
  }
  y[n - 1] = dp[n - 1];
  for (int64_t i = n - 2; i >= 0; i--) y[i] = dp[i] - cp[i] * y[i + 1];
  free(cp);
  free(dp);
}

/* Step 2: Poisson's equation phi'' = -rho/eps0 by second-order finite
 * differences on N_x points with Dirichlet values phi_0 = V and
 * phi_{N_x-1} = 0, solved with the Thomas algorithm. */
void ora_poisson(int32_t nx, double dx, double V, const double* rho, double* phi) {
  int64_t n = nx - 2;
  phi[0] = V;
  phi[nx - 1] = 0.0;
  if (n <= 0) return;
  double* a = (double*)malloc(sizeof(double) * (size_t)n);
  double* b = (double*)malloc(sizeof(double) * (size_t)n);
  double* c = (double*)malloc(sizeof(double) * (size_t)n);
  double* d = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    a[i] = 1.0;
    b[i] = -2.0;
    c[i] = 1.0;
    d[i] = -(dx * dx) * rho[i + 1] / EPS0;
  }
  d[0] = d[0] - phi[0];
  d[n - 1] = d[n - 1] - phi[nx - 1];
  ora_thomas(n, a, b, c, d, phi + 1);
  free(a);
  free(b);
  free(c);
  free(d);
}

/* Step 2, field: E = -dphi/dx by central differences inside; at the walls
 * Gauss's law over the half cell next to the electrode. */
void ora_efield(int32_t nx, double dx, const double* rho, const double* phi, double* E) {
  for (int32_t j = 1; j < nx - 1; j++) E[j] = (phi[j - 1] - phi[j + 1]) / (2.0 * dx);
  E[0] = (phi[0] - phi[1]) / dx - rho[0] * dx / (2.0 * EPS0);
  E[nx - 1] = (phi[nx - 2] - phi[nx - 1]) / dx + rho[nx - 1] * dx / (2.0 * EPS0);
}

/* Stable counting sort of one species by clamped cell index. */
static void sort_species(ora_sim* s, ora_species* q) {
  int64_t n = q->n;
  if (n <= 1) return;
  int32_t nk = s->nx - 1;
  int64_t* cnt = (int64_t*)calloc((size_t)nk + 1, sizeof(int64_t));
  int64_t* key = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    int64_t j, w1;
    double f;
    ora_cell(s->nx, s->inv_dx, q->x[i], &j, &f, &w1);
    key[i] = j;
    cnt[j + 1]++;
  }
  for (int32_t k = 0; k < nk; k++) cnt[k + 1] += cnt[k];
  double* t[4];
  double* src[4] = {q->x, q->vx, q->vy, q->vz};
  for (int a = 0; a < 4; a++) t[a] = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    int64_t d = cnt[key[i]]++;
    for (int a = 0; a < 4; a++) t[a][d] = src[a][i];
  }
  for (int a = 0; a < 4; a++) {
    memcpy(src[a], t[a], sizeof(double) * (size_t)n);
    free(t[a]);
  }
  free(cnt);
  free(key);
}

/* ------------------------------------------------------------------------ */
/* construction                                                             */

void ora_free(ora_sim* s);

static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

ora_sim* ora_create(const ora_params* p, const double* sig_e0, const double* sig_e1,
                    const double* sig_e2, const double* sig_i0, const double* sig_i1) {
  if (!p || p->n_cells < 2 || p->steps_per_cycle < 1 || p->gap_m <= 0.0 || p->rf_freq_hz <= 0.0 ||
      p->ntab < 2 || p->dv_e <= 0.0 || p->dv_i <= 0.0 || p->ion_subcycle < 1 || p->eepf_bins < 1 ||
      p->capacity[0] < 0 || p->capacity[1] < 0 || p->area_m2 <= 0.0 || p->weight <= 0.0 ||
      p->gas_temp_k <= 0.0 || p->pressure_pa < 0.0)
    return NULL;
  ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
  s->p = *p;
  s->nx = p->n_cells + 1;
  s->L = p->gap_m;
  s->dx = p->gap_m / (double)p->n_cells;
  s->inv_dx = 1.0 / s->dx;
  s->dt = 1.0 / (p->rf_freq_hz * (double)p->steps_per_cycle);
  s->ng = p->pressure_pa / (K_B * p->gas_temp_k);
  s->mass[0] = MASS_E;
  s->mass[1] = 39.948 * AMU;
  s->dts[0] = s->dt;
  s->dts[1] = (double)p->ion_subcycle * s->dt;
  s->acc[0] = (-Q_E / s->mass[0]) * s->dts[0];
  s->acc[1] = (Q_E / s->mass[1]) * s->dts[1];
  s->nfac32 = p->weight / (p->area_m2 * s->dx) * INV_TWO32;
  s->qfac32 = Q_E * s->nfac32;
  s->inv_dv[0] = 1.0 / p->dv_e;
  s->inv_dv[1] = 1.0 / p->dv_i;
  s->nproc[0] = 3;
  s->nproc[1] = 2;
  const double* sig[2][3] = {{sig_e0, sig_e1, sig_e2}, {sig_i0, sig_i1, NULL}};
  double dvs[2] = {p->dv_e, p->dv_i};
  for (int sp = 0; sp < 2; sp++) {
    for (int k = 0; k < s->nproc[sp]; k++) s->cum[sp][k] = dalloc(p->ntab);
    s->numax[sp] = 0.0;
    for (int32_t i = 0; i < p->ntab; i++) {
      double v = (double)i * dvs[sp];
      double run = 0.0;
      for (int k = 0; k < s->nproc[sp]; k++) {
        double nu = s->ng * sig[sp][k][i] * v;
        run = (k == 0) ? nu : run + nu;
        s->cum[sp][k][i] = run;
      }
      if (run > s->numax[sp]) s->numax[sp] = run;
    }
    s->pcoll[sp] = 1.0 - exp(-s->numax[sp] * s->dts[sp]);
  }
  s->vtab = dalloc(p->steps_per_cycle);
  for (int32_t m = 0; m < p->steps_per_cycle; m++)
    s->vtab[m] = p->rf_voltage_v * cos(TWO_PI * (double)m / (double)p->steps_per_cycle);
  s->ek_e = 0.5 * MASS_E / Q_E;
  s->ve_e = 2.0 * Q_E / MASS_E;
  s->mr_e = MASS_E / (MASS_E + s->mass[1]);
  s->mm_e = s->mass[1] / (MASS_E + s->mass[1]);
  s->sig_g = sqrt(K_B * p->gas_temp_k / s->mass[1]);
  s->sig_se = sqrt(p->see_temp_ev * Q_E / MASS_E);
  s->eepf_de = p->eepf_emax_ev / (double)p->eepf_bins;
  s->inv_de = (double)p->eepf_bins / p->eepf_emax_ev;
  for (int sp = 0; sp < 2; sp++) {
    ora_species* q = &s->sp[sp];
    q->cap = p->capacity[sp];
    q->n = 0;
    q->x = dalloc(q->cap);
    q->vx = dalloc(q->cap);
    q->vy = dalloc(q->cap);
    q->vz = dalloc(q->cap);
    s->dep[sp] = (int64_t*)calloc((size_t)s->nx, sizeof(int64_t));
    s->codes[sp] = (uint8_t*)calloc((size_t)(q->cap > 0 ? q->cap : 1), 1);
  }
  s->rho = dalloc(s->nx);
  s->phi = dalloc(s->nx);
  s->E = dalloc(s->nx);
  s->acc_ne = dalloc(s->nx);
  s->acc_ni = dalloc(s->nx);
  s->acc_ew = dalloc(s->nx);
  s->acc_w = dalloc(s->nx);
  s->eepf_h = (int64_t*)calloc((size_t)p->eepf_bins, sizeof(int64_t));
  /* arrival energy bins: the EEPF range for electrons; ions gain at most
   * about the peak sheath voltage: 1.25 phi_0, at least 10 eV */
  s->fedf_emax[0] = p->eepf_emax_ev;
  s->fedf_emax[1] = 1.25 * p->rf_voltage_v > 10.0 ? 1.25 * p->rf_voltage_v : 10.0;
  for (int k = 0; k < 2; k++) {
    s->fedf[k] = (int64_t*)calloc((size_t)(2 * p->eepf_bins), sizeof(int64_t));
    s->ek[k] = 0.5 * s->mass[k] / Q_E;
  }
  return s;
}

void ora_free(ora_sim* s) {
  if (!s) return;
  for (int sp = 0; sp < 2; sp++) {
    for (int k = 0; k < 3; k++) free(s->cum[sp][k]);
    free(s->sp[sp].x);
    free(s->sp[sp].vx);
    free(s->sp[sp].vy);
    free(s->sp[sp].vz);
    free(s->dep[sp]);
    free(s->codes[sp]);
  }
  free(s->vtab);
  free(s->rho);
  free(s->phi);
  free(s->E);
  free(s->acc_ne);
  free(s->acc_ni);
  free(s->acc_ew);
  free(s->acc_w);
  free(s->eepf_h);
  free(s->fedf[0]);
  free(s->fedf[1]);
  free(s);
}

int ora_set_state(ora_sim* s, int species, const double* x, const double* vx, const double* vy,
                  const double* vz, int64_t n, int64_t step) {
  if (species < 0 || species > 1 || n < 0) return ORA_EINVAL;
  ora_species* q = &s->sp[species];
  if (n > q->cap) return ORA_ECAPACITY;
  memcpy(q->x, x, sizeof(double) * (size_t)n);
  memcpy(q->vx, vx, sizeof(double) * (size_t)n);
  memcpy(q->vy, vy, sizeof(double) * (size_t)n);
  memcpy(q->vz, vz, sizeof(double) * (size_t)n);
  q->n = n;
  s->step = step;
  memset(s->counters, 0, sizeof(s->counters));
  s->err = 0;
  return ORA_OK;
}

int64_t ora_get_count(const ora_sim* s, int species) { return s->sp[species].n; }
int64_t ora_get_step(const ora_sim* s) { return s->step; }

/* Threads a particle pass runs on: 1 in the plain build, the OpenMP
 * thread count in a build with -fopenmp. */
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_get_state(const ora_sim* s, int species, double* x, double* vx, double* vy, double* vz) {
  const ora_species* q = &s->sp[species];
  memcpy(x, q->x, sizeof(double) * (size_t)q->n);
  memcpy(vx, q->vx, sizeof(double) * (size_t)q->n);
  memcpy(vy, q->vy, sizeof(double) * (size_t)q->n);
  memcpy(vz, q->vz, sizeof(double) * (size_t)q->n);
}

void ora_set_field(ora_sim* s, const double* E) { memcpy(s->E, E, sizeof(double) * (size_t)s->nx); }

void ora_get_field(const ora_sim* s, double* rho, double* phi, double* E, int64_t* de, int64_t* di) {
  size_t b = sizeof(double) * (size_t)s->nx;
  if (rho) memcpy(rho, s->rho, b);
  if (phi) memcpy(phi, s->phi, b);
  if (E) memcpy(E, s->E, b);
  if (de) memcpy(de, s->dep[0], sizeof(int64_t) * (size_t)s->nx);
  if (di) memcpy(di, s->dep[1], sizeof(int64_t) * (size_t)s->nx);
}

void ora_get_counters(const ora_sim* s, int64_t* c) { memcpy(c, s->counters, sizeof(s->counters)); }

int64_t ora_get_decisions(const ora_sim* s, int species, uint8_t* codes) {
  memcpy(codes, s->codes[species], (size_t)s->ncodes[species]);
  return s->ncodes[species];
}

/* dx, dt, ng, numax_e, numax_i, pcoll_e, pcoll_i, nx */
void ora_get_derived(const ora_sim* s, double* out) {
  out[0] = s->dx;
  out[1] = s->dt;
  out[2] = s->ng;
  out[3] = s->numax[0];
  out[4] = s->numax[1];
  out[5] = s->pcoll[0];
  out[6] = s->pcoll[1];
  out[7] = (double)s->nx;
}

void ora_measure(ora_sim* s, int on) { s->measuring = on; }

/* Time averages (Sec. 3.1): densities, CIC-weighted mean electron energy
 * and the EEPF at the centre, normalised so that the sum over bins of
 * sqrt(eps_b) f_b d(eps) is 1. */
void ora_moments(ora_sim* s, double* ne, double* ni, double* emean, double* eepf, int64_t* steps,
                 int reset) {
  int32_t nx = s->nx;
  for (int32_t j = 0; j < nx; j++) {
    if (ne) ne[j] = s->msteps ? s->acc_ne[j] / (double)s->msteps : 0.0;
    if (ni) ni[j] = s->msteps ? s->acc_ni[j] / (double)s->msteps : 0.0;
    if (emean) emean[j] = s->acc_w[j] > 0.0 ? s->acc_ew[j] / s->acc_w[j] : 0.0;
  }
  if (eepf) {
    int64_t tot = 0;
    for (int32_t b = 0; b < s->p.eepf_bins; b++) tot += s->eepf_h[b];
    for (int32_t b = 0; b < s->p.eepf_bins; b++) {
      double eb = ((double)b + 0.5) * s->eepf_de;
      eepf[b] = tot ? (double)s->eepf_h[b] / ((double)tot * sqrt(eb) * s->eepf_de) : 0.0;
    }
  }
  if (steps) *steps = s->msteps;
  if (reset) {
    s->msteps = 0;
    memset(s->acc_ne, 0, sizeof(double) * (size_t)nx);
    memset(s->acc_ni, 0, sizeof(double) * (size_t)nx);
    memset(s->acc_ew, 0, sizeof(double) * (size_t)nx);
    memset(s->acc_w, 0, sizeof(double) * (size_t)nx);
    memset(s->eepf_h, 0, sizeof(int64_t) * (size_t)s->p.eepf_bins);
    for (int k = 0; k < 2; k++) memset(s->fedf[k], 0, sizeof(int64_t) * (size_t)(2 * s->p.eepf_bins));
    memset(s->wall_hits, 0, sizeof(s->wall_hits));
    memset(s->wall_abs, 0, sizeof(s->wall_abs));
    memset(s->wall_esum, 0, sizeof(s->wall_esum));
    s->ioniz_meas = 0;
  }
}

/* Electrode diagnostics since the last reset: arrivals, absorptions and
 * impact-energy sums [species][wall] (flattened 2 x 2), the raw arrival
 * histograms [species][wall][eepf_bins], the ionizations and the measured
 * steps. */
void ora_wall_raw(const ora_sim* s, int64_t* hits, int64_t* absorbed, double* esum, int64_t* hist,
                  int64_t* ioniz, int64_t* steps, double* emax) {
  for (int k = 0; k < 2; k++)
    for (int w = 0; w < 2; w++) {
      hits[2 * k + w] = s->wall_hits[k][w];
      absorbed[2 * k + w] = s->wall_abs[k][w];
      esum[2 * k + w] = s->wall_esum[k][w];
    }
  for (int k = 0; k < 2; k++)
    memcpy(hist + (size_t)k * 2 * s->p.eepf_bins, s->fedf[k], sizeof(int64_t) * (size_t)(2 * s->p.eepf_bins));
  *ioniz = s->ioniz_meas;
  *steps = s->msteps;
  emax[0] = s->fedf_emax[0];
  emax[1] = s->fedf_emax[1];
}

/* ------------------------------------------------------------------------ */
/* one time step                                                            */

typedef struct {
  int64_t n, cap;
  double *x, *vx, *vy, *vz;
} plist;

static void plist_init(plist* l, int64_t cap) {
  l->n = 0;
  l->cap = cap;
  l->x = dalloc(cap);
  l->vx = dalloc(cap);
  l->vy = dalloc(cap);
  l->vz = dalloc(cap);
}
static void plist_free(plist* l) {
  free(l->x);
  free(l->vx);
  free(l->vy);
  free(l->vz);
}
static void plist_push(plist* l, double x, double vx, double vy, double vz) {
  if (l->n < l->cap) {
    l->x[l->n] = x;
    l->vx[l->n] = vx;
    l->vy[l->n] = vy;
    l->vz[l->n] = vz;
  }
  l->n++;
}
static void plist_append(plist* l, const plist* m) {
  for (int64_t k = 0; k < m->n; k++) plist_push(l, m->x[k], m->vx[k], m->vy[k], m->vz[k]);
}

/* Linear interpolation of a cumulative collision-frequency table at speed v.
 * Beyond the last table speed the last entry is used (a constant frequency,
 * still bounded by nu_max); the function then returns 1 so the event can be
 * counted. */
static int table_lookup(const ora_sim* s, int sp, double v, double* nu) {
  double tv = v * s->inv_dv[sp];
  if (!(tv < (double)(s->p.ntab - 1))) {
    for (int q = 0; q < s->nproc[sp]; q++) nu[q] = s->cum[sp][q][s->p.ntab - 1];
    return 1;
  }
  int64_t k = (int64_t)tv;
  double t = tv - (double)k;
  for (int q = 0; q < s->nproc[sp]; q++) nu[q] = (1.0 - t) * s->cum[sp][q][k] + t * s->cum[sp][q][k + 1];
  return 0;
}

/* Outputs of one run of consecutive slots of a particle pass, in slot
 * order: the species' survivors (an ionization electron right after its
 * parent), the ions born from electron impact ionization and the secondary
 * electrons emitted by ion impacts, with the run's event counts and
 * electrode diagnostics. A pass is one run in the plain build; an OpenMP
 * build splits it into one run per thread and joins the runs in slot order,
 * which gives the same lists and integer counts. */
typedef struct {
  plist out, ibirth, se;
  int64_t counters[NCOUNT];
  int64_t wall_hits[2][2], wall_abs[2][2], ioniz_meas;
  double wall_esum[2][2];
  int64_t* fedf[2];
  int err;
} ora_run;

/* Steps (3)-(6) of Sec. 2 for slot i of species sp: field at the particle,
 * leap-frog push, the walls and the null-collision Monte Carlo step; the
 * outputs go to run c. */
static void step_slot(ora_sim* s, int sp, int64_t i, ora_run* c) {
  const ora_params* p = &s->p;
  const int32_t nx = s->nx;
  const double L = s->L;
  const ora_species* q = &s->sp[sp];
  const double dts = s->dts[sp];
  double x = q->x[i], vx = q->vx[i], vy = q->vy[i], vz = q->vz[i];
  uint8_t code = 0x80;
  /* (3) field at the particle: linear interpolation */
  int64_t j, w1;
  double f;
  ora_cell(nx, s->inv_dx, x, &j, &f, &w1);
  double Ep = (1.0 - f) * s->E[j] + f * s->E[j + 1];
  /* (4) leap-frog: v(n+1/2) = v(n-1/2) + (q/m) E dt, x(n+1) = x(n) + v dt */
  vx = vx + s->acc[sp] * Ep;
  x = x + vx * dts;
  uint32_t r0[4];
  draw(s, i, sp, 0, r0);
  int alive = 1;
  /* (5) boundaries */
  if (!isfinite(x) || !isfinite(vx)) {
    c->err = c->err ? c->err : ORA_EUNSTABLE;
    alive = 0;
    code |= 1;
  } else if (x < 0.0 || x > L) {
    /* arrival at an electrode: count it, its impact energy and its
     * energy bin (Sec. 3.3); absorption is added below */
    int wall = x < 0.0 ? 0 : 1;
    if (s->measuring) {
      double eps = s->ek[sp] * (vx * vx + vy * vy + vz * vz);
      c->wall_hits[sp][wall]++;
      c->wall_esum[sp][wall] += eps;
      int64_t b = (int64_t)(eps * ((double)p->eepf_bins / s->fedf_emax[sp]));
      if (b >= 0 && b < p->eepf_bins) c->fedf[sp][(int64_t)wall * p->eepf_bins + b]++;
    }
    double ub = u01(r0[0]);
    if (sp == 0) {
      if (ub < p->reflection) {
        /* elastic (specular) reflection */
        x = (x < 0.0) ? -x : (L + L) - x;
        vx = -vx;
        if (x < 0.0 || x > L) {
          alive = 0;
          code |= 4;
          c->counters[C_REFLECT_LOST]++;
        } else {
          code |= 2;
          c->counters[C_E_REFLECTED]++;
        }
      } else {
        alive = 0;
        code |= 1;
        c->counters[C_E_ABSORBED]++;
      }
    } else {
      alive = 0;
      c->counters[C_I_ABSORBED]++;
      if (ub < p->gamma_see) {
        /* ion-induced secondary electron, emitted from the hit wall
         * with a half-Maxwellian velocity at see_temp_ev */
        uint32_t r3[4];
        draw(s, i, 1, 3, r3);
        double n1, n2, n3, dummy;
        box_muller(u01(r3[0]), u01(r3[1]), &n1, &n2);
        box_muller(u01(r3[2]), u01(r3[3]), &n3, &dummy);
        double xw = (x < 0.0) ? 0.0 : L;
        double vxs = s->sig_se * fabs(n1);
        if (x > L) vxs = -vxs;
        plist_push(&c->se, xw, vxs, s->sig_se * n2, s->sig_se * n3);
        code |= 3;
        c->counters[C_SE_EMITTED]++;
      } else {
        code |= 1;
      }
    }
    if (s->measuring && !alive) c->wall_abs[sp][wall]++;
  }
  /* (6) null-collision Monte Carlo */
  int child = 0;
  double cx = 0, cvx = 0, cvy = 0, cvz = 0;
  if (alive && !(p->flags & F_NO_COLL) && u01(candidacy_word(s, i, sp)) < s->pcoll[sp]) {
    double nu[3];
    if (sp == 0) {
      c->counters[C_E_CAND]++;
      double v2 = vx * vx + vy * vy + vz * vz;
      double speed = sqrt(v2);
      if (table_lookup(s, 0, speed, nu) != 0) c->counters[C_BEYOND]++;
      {
        double r = u01(r0[2]) * s->numax[0];
        uint32_t r1[4];
        if (r < nu[0]) {
          /* elastic: two-body kinematics, atom at rest, isotropic in
           * the centre-of-mass frame */
          draw(s, i, 0, 1, r1);
          double nx_, ny_, nz_;
          if ((p->flags & F_ANISO) && speed > 0.0)
            deflect(vx / speed, vy / speed, vz / speed, s->ek_e * v2, u01(r1[0]), u01(r1[1]),
                    &nx_, &ny_, &nz_);
          else
            iso_dir(u01(r1[0]), u01(r1[1]), &nx_, &ny_, &nz_);
          double g = s->mm_e * speed;
          vx = s->mr_e * vx + g * nx_;
          vy = s->mr_e * vy + g * ny_;
          vz = s->mr_e * vz + g * nz_;
          code |= 2 << 3;
          c->counters[C_E_ELASTIC]++;
        } else if (r < nu[1]) {
          /* excitation: threshold energy lost, new direction isotropic */
          draw(s, i, 0, 1, r1);
          double eps = s->ek_e * v2 - p->exc_threshold_ev;
          if (eps < 0.0) eps = 0.0;
          double sp1 = sqrt(eps * s->ve_e);
          double nx_, ny_, nz_;
          iso_dir(u01(r1[0]), u01(r1[1]), &nx_, &ny_, &nz_);
          vx = sp1 * nx_;
          vy = sp1 * ny_;
          vz = sp1 * nz_;
          code |= 3 << 3;
          c->counters[C_E_EXC]++;
        } else if (r < nu[2]) {
          /* ionization: the energy above threshold is shared
           * uniformly between the scattered and the ejected electron,
           * both isotropic; the new ion is thermal */
          draw(s, i, 0, 1, r1);
          uint32_t r2[4], r3[4];
          draw(s, i, 0, 2, r2);
          draw(s, i, 0, 3, r3);
          double eps = s->ek_e * v2 - p->ion_threshold_ev;
          if (eps < 0.0) eps = 0.0;
          /* uniform sharing, or (variant) the Opal et al. form whose
           * cumulative distribution on [0, eps/2] is
           * atan(e / w) / atan(eps / (2 w)) */
          double e_ej = (p->flags & F_OPAL) ? OPAL_W * tan(u01(r2[0]) * atan(eps / (2.0 * OPAL_W)))
                                            : u01(r2[0]) * eps;
          double e_sc = eps - e_ej;
          double s_sc = sqrt(e_sc * s->ve_e);
          double s_ej = sqrt(e_ej * s->ve_e);
          double ax, ay, az, bx, by, bz;
          iso_dir(u01(r1[0]), u01(r1[1]), &ax, &ay, &az);
          iso_dir(u01(r1[2]), u01(r1[3]), &bx, &by, &bz);
          vx = s_sc * ax;
          vy = s_sc * ay;
          vz = s_sc * az;
          child = 1;
          cx = x;
          cvx = s_ej * bx;
          cvy = s_ej * by;
          cvz = s_ej * bz;
          double n1, n2, n3, dummy;
          box_muller(u01(r3[0]), u01(r3[1]), &n1, &n2);
          box_muller(u01(r3[2]), u01(r3[3]), &n3, &dummy);
          plist_push(&c->ibirth, x, s->sig_g * n1, s->sig_g * n2, s->sig_g * n3);
          code |= 4 << 3;
          c->counters[C_E_ION]++;
          if (s->measuring) c->ioniz_meas++;
        } else {
          code |= 1 << 3;
        }
      }
    } else {
      /* Ar+ on a thermal Ar atom drawn for the candidate */
      c->counters[C_I_CAND]++;
      uint32_t r1[4];
      draw(s, i, 1, 1, r1);
      double n1, n2, n3, dummy;
      box_muller(u01(r1[0]), u01(r1[1]), &n1, &n2);
      box_muller(u01(r1[2]), u01(r1[3]), &n3, &dummy);
      double ax = s->sig_g * n1, ay = s->sig_g * n2, az = s->sig_g * n3;
      double gx = vx - ax, gy = vy - ay, gz = vz - az;
      double g = sqrt(gx * gx + gy * gy + gz * gz);
      if (table_lookup(s, 1, g, nu) != 0) c->counters[C_BEYOND]++;
      {
        double r = u01(r0[2]) * s->numax[1];
        if (r < nu[0]) {
          /* isotropic elastic in the centre-of-mass frame (equal masses) */
          uint32_t r2[4];
          draw(s, i, 1, 2, r2);
          double ux, uy, uz;
          iso_dir(u01(r2[0]), u01(r2[1]), &ux, &uy, &uz);
          double hg = 0.5 * g;
          vx = 0.5 * (vx + ax) + hg * ux;
          vy = 0.5 * (vy + ay) + hg * uy;
          vz = 0.5 * (vz + az) + hg * uz;
          code |= 2 << 3;
          c->counters[C_I_ISO]++;
        } else if (r < nu[1]) {
          /* backward scattering = symmetric charge transfer: the ion
           * leaves with the atom's velocity */
          vx = ax;
          vy = ay;
          vz = az;
          code |= 3 << 3;
          c->counters[C_I_BACK]++;
        } else {
          code |= 1 << 3;
        }
      }
    }
  }
  if (p->flags & F_RECORD) s->codes[sp][i] = code;
  if (alive) {
    plist* out = &c->out;
    plist_push(out, x, vx, vy, vz);
    if (child) plist_push(out, cx, cvx, cvy, cvz);
  }
}

int ora_step(ora_sim* s, int64_t nsteps) {
  const ora_params* p = &s->p;
  const int32_t nx = s->nx;
  const double L = s->L;
  for (int64_t it = 0; it < nsteps; it++) {
    const int64_t step = s->step;
    /* (1) densities */
    ora_deposit_array(nx, s->inv_dx, s->sp[0].n, s->sp[0].x, s->dep[0]);
    ora_deposit_array(nx, s->inv_dx, s->sp[1].n, s->sp[1].x, s->dep[1]);
    for (int32_t j = 0; j < nx; j++) {
      double r = (double)(s->dep[1][j] - s->dep[0][j]) * s->qfac32;
      if (j == 0 || j == nx - 1) r = 2.0 * r; /* half-cell volume at the walls */
      s->rho[j] = r;
    }
    /* (2) potential and field */
    if (p->flags & F_NO_FIELD) {
      for (int32_t j = 0; j < nx; j++) {
        s->phi[j] = 0.0;
        s->E[j] = 0.0;
      }
    } else if (p->flags & F_FIXED_E) {
      for (int32_t j = 0; j < nx; j++) s->phi[j] = 0.0;
    } else {
      double V = s->vtab[step % p->steps_per_cycle];
      ora_poisson(nx, s->dx, V, s->rho, s->phi);
      ora_efield(nx, s->dx, s->rho, s->phi, s->E);
    }
    for (int32_t j = 0; j < nx; j++) {
      if (!isfinite(s->E[j])) s->err = s->err ? s->err : ORA_EUNSTABLE;
    }
    /* time averages at the start of the step */
    if (s->measuring) {
      for (int32_t j = 0; j < nx; j++) {
        double ne = (double)s->dep[0][j] * s->nfac32;
        double ni = (double)s->dep[1][j] * s->nfac32;
        if (j == 0 || j == nx - 1) {
          ne = 2.0 * ne;
          ni = 2.0 * ni;
        }
        s->acc_ne[j] += ne;
        s->acc_ni[j] += ni;
        s->acc_w[j] += (double)s->dep[0][j] * INV_TWO32;
      }
      const ora_species* q = &s->sp[0];
      const double half = 0.5 * L;
      for (int64_t i = 0; i < q->n; i++) {
        double v2 = q->vx[i] * q->vx[i] + q->vy[i] * q->vy[i] + q->vz[i] * q->vz[i];
        double eps = s->ek_e * v2;
        int64_t j, w1;
        double f;
        ora_cell(nx, s->inv_dx, q->x[i], &j, &f, &w1);
        s->acc_ew[j] += ((double)((int64_t)4294967296LL - w1) * INV_TWO32) * eps;
        s->acc_ew[j + 1] += ((double)w1 * INV_TWO32) * eps;
        if (fabs(q->x[i] - half) <= p->eepf_halfwidth_m) {
          int64_t b = (int64_t)(eps * s->inv_de);
          if (b < p->eepf_bins) s->eepf_h[b]++;
        }
      }
      s->msteps++;
    }

    /* (3)-(6) for the electrons, then for the ions on their sub-cycled steps */
    const int ion_step = !(p->flags & F_IMMOBILE_IONS) && (step % p->ion_subcycle == 0);
    plist eout, iout, ibirth, se;
    plist_init(&eout, 2 * s->sp[0].n + 1);
    plist_init(&ibirth, s->sp[0].n + 1);
    plist_init(&iout, s->sp[1].n + 1);
    plist_init(&se, s->sp[1].n + 1);
    s->ncodes[0] = s->sp[0].n;
    s->ncodes[1] = ion_step ? s->sp[1].n : 0;

    for (int sp = 0; sp < 2; sp++) {
      if (sp == 1 && !ion_step) break;
      const ora_species* q = &s->sp[sp];
      s->counters[sp == 0 ? C_E_PUSHED : C_I_PUSHED] += q->n;
      const int64_t n = q->n;
      int nrun = 1;
#ifdef _OPENMP
      nrun = omp_get_max_threads();
      if ((int64_t)nrun > n) nrun = n > 0 ? (int)n : 1;
#endif
      ora_run* runs = (ora_run*)calloc((size_t)nrun, sizeof(ora_run));
      for (int k = 0; k < nrun; k++) {
        int64_t len = n * (k + 1) / nrun - n * k / nrun;
        plist_init(&runs[k].out, 2 * len + 1);
        plist_init(&runs[k].ibirth, len + 1);
        plist_init(&runs[k].se, len + 1);
        for (int w = 0; w < 2; w++)
          runs[k].fedf[w] = (int64_t*)calloc((size_t)(2 * p->eepf_bins), sizeof(int64_t));
      }
#ifdef _OPENMP
#pragma omp parallel for schedule(static, 1)
#endif
      for (int k = 0; k < nrun; k++)
        for (int64_t i = n * k / nrun; i < n * (k + 1) / nrun; i++) step_slot(s, sp, i, &runs[k]);
      /* join the runs in slot order */
      for (int k = 0; k < nrun; k++) {
        ora_run* c = &runs[k];
        plist_append((sp == 0) ? &eout : &iout, &c->out);
        plist_append(&ibirth, &c->ibirth);
        plist_append(&se, &c->se);
        for (int m = 0; m < NCOUNT; m++) s->counters[m] += c->counters[m];
        for (int a = 0; a < 2; a++)
          for (int w = 0; w < 2; w++) {
            s->wall_hits[a][w] += c->wall_hits[a][w];
            s->wall_abs[a][w] += c->wall_abs[a][w];
            s->wall_esum[a][w] += c->wall_esum[a][w];
          }
        for (int w = 0; w < 2; w++)
          for (int64_t b = 0; b < 2 * (int64_t)p->eepf_bins; b++) s->fedf[w][b] += c->fedf[w][b];
        s->ioniz_meas += c->ioniz_meas;
        if (c->err && !s->err) s->err = c->err;
        plist_free(&c->out);
        plist_free(&c->ibirth);
        plist_free(&c->se);
        free(c->fedf[0]);
        free(c->fedf[1]);
      }
      free(runs);
    }

    /* rebuild: e = [survivors with ionization electrons after their parent]
     * ++ [secondary electrons]; Ar+ = [survivors or the unmoved ions] ++
     * [ionization ions], each list in parent-slot order */
    ora_species* qe = &s->sp[0];
    ora_species* qi = &s->sp[1];
    int64_t ne_new = eout.n + se.n;
    int64_t ni_old = ion_step ? iout.n : qi->n;
    int64_t ni_new = ni_old + ibirth.n;
    int status = 0;
    if (ne_new > qe->cap || ni_new > qi->cap) {
      status = ORA_ECAPACITY;
    } else {
      memcpy(qe->x, eout.x, sizeof(double) * (size_t)eout.n);
      memcpy(qe->vx, eout.vx, sizeof(double) * (size_t)eout.n);
      memcpy(qe->vy, eout.vy, sizeof(double) * (size_t)eout.n);
      memcpy(qe->vz, eout.vz, sizeof(double) * (size_t)eout.n);
      memcpy(qe->x + eout.n, se.x, sizeof(double) * (size_t)se.n);
      memcpy(qe->vx + eout.n, se.vx, sizeof(double) * (size_t)se.n);
      memcpy(qe->vy + eout.n, se.vy, sizeof(double) * (size_t)se.n);
      memcpy(qe->vz + eout.n, se.vz, sizeof(double) * (size_t)se.n);
      qe->n = ne_new;
      if (ion_step) {
        memcpy(qi->x, iout.x, sizeof(double) * (size_t)iout.n);
        memcpy(qi->vx, iout.vx, sizeof(double) * (size_t)iout.n);
        memcpy(qi->vy, iout.vy, sizeof(double) * (size_t)iout.n);
        memcpy(qi->vz, iout.vz, sizeof(double) * (size_t)iout.n);
      }
      memcpy(qi->x + ni_old, ibirth.x, sizeof(double) * (size_t)ibirth.n);
      memcpy(qi->vx + ni_old, ibirth.vx, sizeof(double) * (size_t)ibirth.n);
      memcpy(qi->vy + ni_old, ibirth.vy, sizeof(double) * (size_t)ibirth.n);
      memcpy(qi->vz + ni_old, ibirth.vz, sizeof(double) * (size_t)ibirth.n);
      qi->n = ni_new;
    }
    plist_free(&eout);
    plist_free(&iout);
    plist_free(&ibirth);
    plist_free(&se);
    if (status) return status;
    s->step++;
    s->counters[C_STEPS]++;
    if (p->sort_interval > 0 && s->step % p->sort_interval == 0) {
      sort_species(s, qe);
      sort_species(s, qi);
    }
    if (s->err) return s->err;
  }
  /* deposit and field of the final state, for inspection */
  ora_deposit_array(nx, s->inv_dx, s->sp[0].n, s->sp[0].x, s->dep[0]);
  ora_deposit_array(nx, s->inv_dx, s->sp[1].n, s->sp[1].x, s->dep[1]);
  return s->err;
}

/* Deposit of the current state (both species), without stepping. */
void ora_deposit(ora_sim* s) {
  ora_deposit_array(s->nx, s->inv_dx, s->sp[0].n, s->sp[0].x, s->dep[0]);
  ora_deposit_array(s->nx, s->inv_dx, s->sp[1].n, s->sp[1].x, s->dep[1]);
}

/* Field solve of the current state at its step (Sec. 2 steps 1-2). */
void ora_solve_field(ora_sim* s) {
  ora_deposit(s);
  for (int32_t j = 0; j < s->nx; j++) {
    double r = (double)(s->dep[1][j] - s->dep[0][j]) * s->qfac32;
    if (j == 0 || j == s->nx - 1) r = 2.0 * r;
    s->rho[j] = r;
  }
  double V = s->vtab[s->step % s->p.steps_per_cycle];
  ora_poisson(s->nx, s->dx, V, s->rho, s->phi);
  ora_efield(s->nx, s->dx, s->rho, s->phi, s->E);
}
