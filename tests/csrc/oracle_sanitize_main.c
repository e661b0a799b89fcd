/* Drives the CPU oracle through a short discharge with every diagnostic on,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer: walls
 * with reflection and emission, all collision processes, births, cell sorts,
 * time averages, electrode histograms, the field solvers and the profile
 * loader. Exit status 0 when every call succeeded; the sanitizers abort on
 * the first finding. Test infrastructure only. */
#include "../../oracle/pic_oracle.c"

#include <stdio.h>

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int ora_load_profile(const double* dens, const double* temp_ev, int npts, double L, double vfac,
                     uint32_t seed, uint32_t run, int species, int64_t n, double* x, double* vx,
                     double* vy, double* vz);

static double uniform(uint64_t* s) {
  *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
  return ((double)(*s >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

int main(void) {
  ora_params p;
  memset(&p, 0, sizeof(p));
  p.gap_m = 0.025;
  p.pressure_pa = 60.0;
  p.gas_temp_k = 300.0;
  p.rf_voltage_v = 250.0;
  p.rf_freq_hz = 13.56e6;
  p.steps_per_cycle = 400;
  p.n_cells = 64;
  p.weight = 1e6;
  p.area_m2 = 1e-4;
  p.reflection = 0.4;
  p.gamma_see = 0.3;
  p.see_temp_ev = 1.0;
  p.capacity[0] = p.capacity[1] = 40000;
  p.ion_subcycle = 3;
  p.sort_interval = 7;
  p.seed = 5;
  p.run = 9;
  p.eepf_bins = 64;
  p.eepf_emax_ev = 30.0;
  p.eepf_halfwidth_m = 0.0025;
  p.flags = 16; /* record decisions */
  p.ntab = 257;
  p.dv_e = 1.2e7 / 256.0; /* speeds beyond the table occur too */
  p.dv_i = 2e4 / 256.0;
  p.exc_threshold_ev = 11.5;
  p.ion_threshold_ev = 15.8;
  double se[3][257], si[2][257];
  for (int k = 0; k < 257; k++) {
    se[0][k] = 5e-20;
    se[1][k] = 2e-20;
    se[2][k] = 3e-20;
    si[0][k] = 4e-19;
    si[1][k] = 3e-19;
  }
  ora_sim* s = ora_create(&p, se[0], se[1], se[2], si[0], si[1]);
  if (!s) return 2;
  int64_t n = 3000;
  double *x = malloc(8 * n), *vx = malloc(8 * n), *vy = malloc(8 * n), *vz = malloc(8 * n);
  uint64_t st = 42;
  for (int sp = 0; sp < 2; sp++) {
    double v = sp == 0 ? 2.5e6 : 3e3;
    for (int64_t i = 0; i < n; i++) {
      x[i] = p.gap_m * uniform(&st);
      vx[i] = v * (2.0 * uniform(&st) - 1.0);
      vy[i] = v * (2.0 * uniform(&st) - 1.0);
      vz[i] = v * (2.0 * uniform(&st) - 1.0);
    }
    if (ora_set_state(s, sp, x, vx, vy, vz, n, 0)) return 3;
  }
  if (ora_step(s, 40)) return 4;
  ora_measure(s, 1);
  if (ora_step(s, 60)) return 5;
  int32_t nx = p.n_cells + 1;
  double *ne = malloc(8 * nx), *ni = malloc(8 * nx), *em = malloc(8 * nx), *ep = malloc(8 * 64);
  int64_t steps = 0;
  int64_t hits[4], absd[4], hist[4 * 64], ion, mst;
  double esum[4], emax[2];
  ora_wall_raw(s, hits, absd, esum, hist, &ion, &mst, emax);
  ora_moments(s, ne, ni, em, ep, &steps, 1);
  int64_t cnt[16];
  ora_get_counters(s, cnt);
  uint8_t* codes = malloc((size_t)p.capacity[0]);
  ora_get_decisions(s, 0, codes);
  ora_solve_field(s);
  /* fixed field and no field modes on the same state */
  double* E = calloc((size_t)nx, 8);
  ora_set_field(s, E);
  double *rho = malloc(8 * nx), *phi = malloc(8 * nx);
  int64_t *de = malloc(8 * nx), *di = malloc(8 * nx);
  ora_get_field(s, rho, phi, E, de, di);
  /* profile loader */
  double dens[33], temp[33];
  for (int k = 0; k < 33; k++) {
    dens[k] = 1e15 * (1.0 + k % 5);
    temp[k] = 1.0 + 0.1 * k;
  }
  if (ora_load_profile(dens, temp, 33, p.gap_m, Q_E / MASS_E, 3, 4, 0, n, x, vx, vy, vz)) return 6;
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
  ora_philox4x32_10(ctr, key, out);
  printf("steps %lld e %lld i %lld hits %lld collisions %lld ionizations %lld\n", (long long)steps,
         (long long)ora_get_count(s, 0), (long long)ora_get_count(s, 1),
         (long long)(hits[0] + hits[1] + hits[2] + hits[3]), (long long)(cnt[8] + cnt[9] + cnt[10]),
         (long long)cnt[10]);
  ora_free(s);
  free(x), free(vx), free(vy), free(vz), free(ne), free(ni), free(em), free(ep), free(codes);
  free(E), free(rho), free(phi), free(de), free(di);
  return 0;
}
