/*
 * Oracle of the warm-start particle loader (TEST INFRASTRUCTURE ONLY).
 *
 * Particles are drawn from a density profile given at npts equally spaced
 * points on [0, L] and taken linear between them. The cumulative density is
 * then quadratic inside each interval; slot i's position is where it reaches
 * u_i times its total, u_i the slot's position uniform. Its velocity
 * components are normal with variance e T(x) / m for a temperature profile
 * (eV) linear between the same points. Written from that definition, in
 * plain sequential C: the interval masses are summed from the left, the
 * interval is found by scanning, and the quadratic is solved in the form
 * t = 2 r / (a + sqrt(a^2 + 2 (b - a) r / h)), which is the root in [0, h]
 * of a t + (b - a) t^2 / (2 h) = r and avoids cancellation when b ~ a.
 * Draws: Philox4x32-10 keyed (seed, run), counter (0xFFFFFFFE, slot,
 * 16 species + purpose, 0); purpose 0 word 0 -> u_i, purpose 1 -> three
 * normals by Box-Muller from words (0, 1) and (2, 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#define LOAD_STEP 0xFFFFFFFEu
static const double INV_2_32 = 2.3283064365386963e-10;
static const double TWO_PI_W = 6.283185307179586;

static double unit(uint32_t r) { return ((double)r + 0.5) * INV_2_32; }

static void normals(double u1, double u2, double* a, double* b) {
  double rad = sqrt(-2.0 * log(u1));
  double th = TWO_PI_W * u2;
  *a = rad * cos(th);
  *b = rad * sin(th);
}

static double nonneg(double v) { return v > 0.0 ? v : 0.0; }

int ora_load_profile(const double* dens, const double* temp_ev, int npts, double L, double vfac,
                     uint32_t seed, uint32_t run, int species, int64_t n, double* x, double* vx,
                     double* vy, double* vz) {
  if (npts < 2) return -1;
  double h = L / (double)(npts - 1);
  double hh = 0.5 * h;
  double* cum = (double*)malloc(sizeof(double) * (size_t)npts);
  if (!cum) return -1;
  cum[0] = 0.0;
  for (int k = 0; k + 1 < npts; ++k) cum[k + 1] = cum[k] + (nonneg(dens[k]) + nonneg(dens[k + 1])) * hh;
  double total = cum[npts - 1];
  uint32_t key[2] = {seed, run};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t c0[4] = {LOAD_STEP, (uint32_t)i, (uint32_t)(16 * species), 0u}, r0[4];
    ora_philox4x32_10(c0, key, r0);
    double r = unit(r0[0]) * total;
    int k = 0;
    while (k + 1 <= npts - 2 && cum[k + 1] <= r) ++k;
    double rp = r - cum[k];
    double a = nonneg(dens[k]), b = nonneg(dens[k + 1]);
    double disc = a * a + 2.0 * (b - a) * rp / h;
    double den = a + sqrt(disc > 0.0 ? disc : 0.0);
    double t = den > 0.0 ? 2.0 * rp / den : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > h) t = h;
    double xi = (double)k * h + t;
    if (xi > L) xi = L;
    double T = temp_ev[k] + (temp_ev[k + 1] - temp_ev[k]) * (t / h);
    if (T < 0.0) T = 0.0;
    double sig = sqrt(T * vfac);
    uint32_t c1[4] = {LOAD_STEP, (uint32_t)i, (uint32_t)(16 * species + 1), 0u}, r1[4];
    ora_philox4x32_10(c1, key, r1);
    double n1, n2, n3, n4;
    normals(unit(r1[0]), unit(r1[1]), &n1, &n2);
    normals(unit(r1[2]), unit(r1[3]), &n3, &n4);
    x[i] = xi;
    vx[i] = sig * n1;
    vy[i] = sig * n2;
    vz[i] = sig * n3;
  }
  free(cum);
  return 0;
}
