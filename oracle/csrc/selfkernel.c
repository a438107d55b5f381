/* Oracle helper (test infrastructure only): cell integrals of the
 * non-replicating spectral self kernel K(n, t), by direct quadrature of its
 * defining psi-integral (Section 2.3.1, eq. "non_replicant_kernel").
 *
 *   cs t <  L : K = (1/2pi) int_0^{2pi} cos^2(psi) cos(x sin psi) dpsi
 *               (periodic integrand: trapezoid rule, exponentially convergent)
 *   cs t >= L : K = (2/pi) int_0^{asin(L/(cs t))} cos^2(psi) cos(x sin psi) dpsi
 *               (composite Gauss-Legendre, one panel per half oscillation)
 *   x = n pi cs t / L
 *
 * The cell integral over [t0, t1] is Gauss-Legendre in t, split at t = L/cs;
 * on the part after L/cs the substitution t = L/cs + (t1 - L/cs) s^2 removes
 * the (t - L/cs)^{3/2} endpoint behaviour of K.
 *
 * Built with plain gcc by the build step; loaded through ctypes from
 * oracle/selfterm.py.  Shares nothing with the HIP library.
 */
#include <math.h>
#include <stdint.h>

#define NGL 20
static double gl_x[NGL], gl_w[NGL];
static int gl_ready = 0;

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton on P_n. */
static void gl_init(void) {
  if (gl_ready) return;
  const int n = NGL;
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double z1 = z;
      z = z1 - p1 / pp;
      if (fabs(z - z1) < 1e-16) break;
    }
    gl_x[i] = z;
    gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
  gl_ready = 1;
}

static double k_early(double x) {
  /* (1/2pi) int_0^{2pi} cos^2 psi cos(x sin psi) dpsi, trapezoid with m points;
   * the aliasing error is of the size of J_m(x), negligible once m exceeds x by
   * many widths x^(1/3) of the Bessel transition region */
  double ax = fabs(x);
  int m = 4 * (int)ceil((ax + 20.0 * cbrt(ax) + 48.0) / 4.0);
  double s = 0.0;
  for (int k = 0; k < m; ++k) {
    double p = 2.0 * M_PI * k / m;
    double c = cos(p);
    s += c * c * cos(x * sin(p));
  }
  return s / m;
}

static double k_late(double x, double psim, int n) {
  /* (2/pi) int_0^{psim} cos^2 psi cos(x sin psi) dpsi */
  int panels = n / 2 + 4;
  double h = psim / panels, s = 0.0;
  for (int p = 0; p < panels; ++p) {
    double a = p * h, mid = a + 0.5 * h;
    for (int i = 0; i < NGL; ++i) {
      double psi = mid + 0.5 * h * gl_x[i];
      double c = cos(psi);
      s += gl_w[i] * 0.5 * h * c * c * cos(x * sin(psi));
    }
  }
  return 2.0 / M_PI * s;
}

double oracle_K_mode(int n, double t, double L, double cs) {
  gl_init();
  double x = n * M_PI * cs * t / L;
  if (cs * t < L) return k_early(x);
  return k_late(x, asin(L / (cs * t)), n);
}

static double cell(int n, double t0, double t1, double L, double cs) {
  double tl = L / cs, s = 0.0;
  if (t0 < tl) { /* early part [t0, min(t1, tl)] */
    double b = t1 < tl ? t1 : tl, h = b - t0, mid = 0.5 * (t0 + b);
    for (int i = 0; i < NGL; ++i) s += gl_w[i] * 0.5 * h * oracle_K_mode(n, mid + 0.5 * h * gl_x[i], L, cs);
  }
  if (t1 > tl) { /* late part [max(t0, tl), t1] */
    double a = t0 > tl ? t0 : tl;
    if (a > tl) {
      double h = t1 - a, mid = 0.5 * (a + t1);
      for (int i = 0; i < NGL; ++i) s += gl_w[i] * 0.5 * h * oracle_K_mode(n, mid + 0.5 * h * gl_x[i], L, cs);
    } else { /* t = tl + D s^2, s in [0, 1] */
      double D = t1 - tl;
      for (int i = 0; i < NGL; ++i) {
        double sn = 0.5 * (1.0 + gl_x[i]);
        s += gl_w[i] * 0.5 * 2.0 * D * sn * oracle_K_mode(n, tl + D * sn * sn, L, cs);
      }
    }
  }
  return s;
}

/* out[T] = int over the centred cell [max(0,(T-1/2)dt), (T+1/2)dt] of K(n,t) dt,
 * for T = 0..W (the |k_n| factor is applied by the caller). */
void oracle_K_cells(int n, int W, double dt, double L, double cs, double* out) {
  gl_init();
  for (int T = 0; T <= W; ++T) {
    double t0 = (T - 0.5) * dt;
    if (t0 < 0) t0 = 0;
    out[T] = cell(n, t0, (T + 0.5) * dt, L, cs);
  }
}

/* Many modes at once (OpenMP over modes): modes[i], windows W[i], out at offs[i]. */
void oracle_K_table(int nm, const int32_t* modes, const int32_t* W, const int64_t* offs,
                    double dt, double L, double cs, double* out) {
  gl_init();
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nm; ++i) oracle_K_cells(modes[i], W[i], dt, L, cs, out + offs[i]);
}
