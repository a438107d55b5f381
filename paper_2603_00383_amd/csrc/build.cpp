// Host-side operator build: geometry, causality windows, closed-form kernel
// entries, fault-wise H-matrix partition, per-lag adaptive cross approximation,
// packing into device work items, spectral self-kernel tables.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <numeric>

#include "internal.hpp"

namespace seas {

// ============================================================== primitives
// Weighted sum n1' I_31 + n2' I_32 of the antiplane primitives (Section 2.3.2,
// eq. "primitives") at one corner (r1, r2) and ct = cs t. H(0) = 0, sgn(0) = 0.
// Inside the cone ct > r: sqrt((ct/r)^2 - 1) = Q / r with Q^2 = (ct - r)(ct + r),
// and arccos(|r1| / sqrt(ct^2 - r2^2)) = atan2(Q, |r1|).
static inline double corner(double r1, double r2, double ct, double n1, double n2) {
  const double ar2 = std::fabs(r2);
  if (!(ct > ar2)) return 0.0;  // before the plane front: both terms vanish (ct <= |r2| <= r)
  double v = 0.0;
  if (r1 > 0.0) v += n2;         // plane-wave term H(r1) H(t - |r2|/cs)
  if (!(ct > std::fabs(r1))) return v;  // ct <= |r1| <= r: outside the cylindrical front
  const double r = std::hypot(r1, r2);
  if (ct > r) {
    const double Q = std::sqrt((ct - r) * (ct + r));
    const double rr = r * r;
    v -= n1 * r2 * Q / (M_PI * rr);
    if (r1 != 0.0) {
      const double a1 = std::fabs(r1);
      const double sg = r1 > 0.0 ? 1.0 : -1.0;
      v += n2 * sg * (a1 * Q / rr - std::atan2(Q, a1)) / M_PI;
    }
  }
  return v;
}

struct PairFrame {  // receiver a, source b
  double n1, n2, h;
};

static inline PairFrame frame(const Fault& A, const Fault& B) {
  return {A.nx * B.tx + A.ny * B.ty, A.nx * B.nx + A.ny * B.ny, 0.5 * B.dx};
}

static inline void offsets(const Fault& A, int i, const Fault& B, int j, double& r1, double& r2) {
  const double dx = A.midx(i) - B.midx(j), dy = A.midy(i) - B.midy(j);
  r1 = dx * B.tx + dy * B.ty;
  r2 = dx * B.nx + dy * B.ny;
}

// K^T of eq. "kernel_interactions": space-time difference over the source element.
double kernel_entry(const Fault& A, int i, const Fault& B, int j, int T, double dt, double cs) {
  double r1, r2;
  offsets(A, i, B, j, r1, r2);
  const PairFrame fr = frame(A, B);
  const double c1 = cs * ((T + 1) * dt), c0 = cs * (T * dt);
  return (corner(r1 + fr.h, r2, c1, fr.n1, fr.n2) - corner(r1 - fr.h, r2, c1, fr.n1, fr.n2)) -
         (corner(r1 + fr.h, r2, c0, fr.n1, fr.n2) - corner(r1 - fr.h, r2, c0, fr.n1, fr.n2));
}

// Static stress at receiver i per unit slip of source element j (late-time limit
// of -mu/(2cs) K^T / dt): two screw dislocations at the element ends.
double static_stress(const Fault& A, int i, const Fault& B, int j, double mu) {
  double r1, r2;
  offsets(A, i, B, j, r1, r2);
  const PairFrame fr = frame(A, B);
  const double p1 = r1 + fr.h, m1 = r1 - fr.h;
  const double pp = p1 * p1 + r2 * r2, mm = m1 * m1 + r2 * r2;
  const double c = mu / (2.0 * M_PI);
  return fr.n1 * c * r2 * (1.0 / pp - 1.0 / mm) - fr.n2 * c * (p1 / pp - m1 / mm);
}

// ============================================================== self kernel
// Gauss-Legendre rule on [-1, 1] from the three-term recurrence, by Newton from
// Tricomi's initial guesses.
struct GL {
  std::vector<double> x, w;
  explicit GL(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) *
                 std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
      double dp = 1.0;
      for (int it = 0; it < 60; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (p0 - z * p1) / (1.0 - z * z);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-17) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

// Integral of K(n, t) over [t0, t1] (eq. "non_replicant_kernel"), with the order
// of integration exchanged: K is (2/pi) times the integral of cos^2(psi) cos(a t
// sin psi) over psi in [0, pi/2] restricted to t <= L / (cs sin psi) (this one
// region covers both branches of the definition, a = n pi cs / L). The t-integral
// is then elementary, leaving one smooth psi-integral split where the restriction
// starts to cut the cell: sin psi1 = L/(cs t1), sin psi0 = L/(cs t0).
void self_cells(int n, int W, double dt, double L, double cs, double* out) {
  static const GL g(16);
  const double a = n * M_PI * cs / L;
  auto piece = [&](double lo, double hi, int panels, const std::function<double(double)>& f) {
    if (hi <= lo) return 0.0;
    const double h = (hi - lo) / panels;
    double s = 0.0;
    for (int p = 0; p < panels; ++p) {
      const double m = lo + (p + 0.5) * h;
      double acc = 0.0;
      for (size_t k = 0; k < g.x.size(); ++k) acc += g.w[k] * f(m + 0.5 * h * g.x[k]);
      s += 0.5 * h * acc;
    }
    return s;
  };
  for (int T = 0; T <= W; ++T) {
    const double t0 = std::max(0.0, (T - 0.5) * dt), t1 = (T + 0.5) * dt;
    const double s1 = L / (cs * t1);
    const double psi1 = s1 >= 1.0 ? 0.5 * M_PI : std::asin(s1);
    double psi0 = 0.5 * M_PI;
    if (t0 > 0.0) {
      const double s0 = L / (cs * t0);
      psi0 = s0 >= 1.0 ? 0.5 * M_PI : std::asin(s0);
    }
    const int pan1 = 4 + (int)std::ceil(a * t1 * std::sin(psi1) / M_PI);
    const int pan2 = 4 + (int)std::ceil(a * t0 * (std::sin(psi0) - std::sin(psi1)) / M_PI);
    // full cell: int_t0^t1 cos(a s t) dt = 2 cos(a s (t0+t1)/2) sin(a s (t1-t0)/2) / (a s)
    const double tm = 0.5 * (t0 + t1), th = 0.5 * (t1 - t0);
    const double full = piece(0.0, psi1, pan1, [&](double psi) {
      const double s = std::sin(psi), c = std::cos(psi);
      const double as = a * s;
      const double v = as * th < 1e-8 ? 2.0 * th * std::cos(as * tm)
                                      : 2.0 * std::cos(as * tm) * std::sin(as * th) / as;
      return c * c * v;
    });
    // cut cell: int_t0^{L/(cs s)} cos(a s t) dt = (sin(n pi) - sin(a s t0)) / (a s), sin(n pi) = 0
    const double cut = piece(psi1, psi0, pan2, [&](double psi) {
      const double s = std::sin(psi), c = std::cos(psi);
      return -c * c * std::sin(a * s * t0) / (a * s);
    });
    out[T] = 2.0 / M_PI * (full + cut);
  }
}

// Integral of K(n, t) over t >= t0: the static tail a window ending at t0 drops.
// Over [t0, tb], tb = 64 max(t0, L/cs), the exchanged order of self_cells: the
// full piece psi in [0, psi_b] (sin psi_b = L/(cs tb)) integrates cos(a s t) over
// the whole range, the cut piece psi in [psi_b, psi_0] up to t = L/(cs s). The
// oscillation in psi is at most n pi there, whatever tb is. Beyond tb, the late
// branch K = (2/pi) int_0^{s0} sqrt(1 - s^2) cos(a t s) ds (s0 = L/(cs t),
// a t s0 = n pi) expands in powers of 1/(a t): K = (2/pi) sum_m c_m J_m
// (a t)^-(2m+1), c_m the coefficients of sqrt(1 - y), J_m = int_0^{n pi} u^{2m}
// cos u du (J_0 = 0), and each term integrates in closed form; the ratio of
// successive terms is about (L/(cs tb))^2 = 1/4096.
double self_tail_integral(int n, double t0, double L, double cs) {
  static const GL g(16);
  const double a = n * M_PI * cs / L;
  const double tl = L / cs;
  const double tb = 64.0 * std::max(t0, tl);
  auto piece = [&](double lo, double hi, int panels, const std::function<double(double)>& f) {
    if (hi <= lo) return 0.0;
    const double h = (hi - lo) / panels;
    double acc = 0.0;
    for (int p = 0; p < panels; ++p) {
      const double m = lo + (p + 0.5) * h;
      double q = 0.0;
      for (size_t k = 0; k < g.x.size(); ++k) q += g.w[k] * f(m + 0.5 * h * g.x[k]);
      acc += 0.5 * h * q;
    }
    return acc;
  };
  const double psib = std::asin(L / (cs * tb));
  const double psi0 = t0 <= tl ? 0.5 * M_PI : std::asin(L / (cs * t0));
  const int pan = 8 + 2 * n;
  // int_t0^tb cos(a s t) dt = (sin(a s tb) - sin(a s t0)) / (a s)
  const double full = piece(0.0, psib, pan, [&](double psi) {
    const double s = std::sin(psi), c = std::cos(psi);
    const double as = a * s;
    const double v = as * tb < 1e-6 ? tb - t0 : (std::sin(as * tb) - std::sin(as * t0)) / as;
    return c * c * v;
  });
  // int_t0^{L/(cs s)} cos(a s t) dt = (sin(n pi) - sin(a s t0)) / (a s), sin(n pi) = 0
  const double cut = piece(psib, psi0, pan, [&](double psi) {
    const double s = std::sin(psi), c = std::cos(psi);
    return -c * c * std::sin(a * s * t0) / (a * s);
  });
  // closed-form terms past tb: int_tb^inf (a t)^-(2m+1) dt = 1 / (2m a^(2m+1) tb^(2m))
  const double X = n * M_PI, cosX = (n & 1) ? -1.0 : 1.0;
  double C[10], S[10];  // int_0^X u^k cos u du and int_0^X u^k sin u du (sin X = 0)
  C[0] = 0.0;
  S[0] = 1.0 - cosX;
  for (int k = 1; k < 10; ++k) {
    C[k] = -k * S[k - 1];
    S[k] = -std::pow(X, k) * cosX + k * C[k - 1];
  }
  const double cm[5] = {1.0, -0.5, -0.125, -0.0625, -5.0 / 128.0};
  double far = 0.0;
  for (int m = 1; m <= 4; ++m) far += cm[m] * C[2 * m] / (2.0 * m * std::pow(a, 2 * m + 1) * std::pow(tb, 2 * m));
  return 2.0 / M_PI * (full + cut + far);
}

// ============================================================== partition
struct Node {
  int lo, hi, kid0 = -1, kid1 = -1;
  double cx, cy, r;
};

static void build_tree(const Fault& f, int leaf, std::vector<Node>& nodes) {
  std::function<int(int, int)> rec = [&](int lo, int hi) -> int {
    Node nd;
    nd.lo = lo;
    nd.hi = hi;
    const double s = -0.5 * f.L + 0.5 * (lo + hi) * f.dx;  // closed-form bounding circle
    nd.cx = f.cx + s * f.tx;
    nd.cy = f.cy + s * f.ty;
    nd.r = 0.5 * (hi - lo) * f.dx;
    const int id = (int)nodes.size();
    nodes.push_back(nd);
    if (hi - lo > leaf) {
      const int mid = lo + (hi - lo) / 2;
      const int k0 = rec(lo, mid);
      const int k1 = rec(mid, hi);
      nodes[id].kid0 = k0;
      nodes[id].kid1 = k1;
    }
    return id;
  };
  rec(0, f.Np);
}

static void traverse(const std::vector<Node>& to, const std::vector<Node>& ts, double eta_H, int pair,
                     int a, int b, std::vector<BlockDesc>& out) {
  std::function<void(int, int)> rec = [&](int o, int s) {
    const Node &O = to[o], &S = ts[s];
    const double d = std::hypot(O.cx - S.cx, O.cy - S.cy);
    const bool oleaf = O.kid0 < 0, sleaf = S.kid0 < 0;
    if (d > eta_H * (O.r + S.r)) {
      out.push_back({pair, a, b, O.lo, O.hi, S.lo, S.hi, 1, 0, 0});
      return;
    }
    if (oleaf && sleaf) {
      out.push_back({pair, a, b, O.lo, O.hi, S.lo, S.hi, 0, 0, 0});
      return;
    }
    bool split_o;
    if (O.r > S.r) split_o = !oleaf;
    else if (S.r > O.r) split_o = sleaf;
    else split_o = !oleaf;
    if (split_o) {
      rec(O.kid0, s);
      rec(O.kid1, s);
    } else {
      rec(o, S.kid0);
      rec(o, S.kid1);
    }
  };
  rec(0, 0);
}

// ============================================================== compression
// Adaptive cross approximation with full pivoting on the evaluated block:
// A ~= sum_l u_l w_l^T, stopping when the residual's Frobenius norm is at most
// tol times that of A. Returns the rank, or -1 when the rank reaches
// kmax (the factors would not be smaller than the block: store it dense).
static int aca_full(const double* A, int p, int q, double tol, int kmax, std::vector<double>& U,
                    std::vector<double>& Wf, std::vector<double>& R) {
  const size_t n = (size_t)p * q;
  R.assign(A, A + n);
  double nrm2 = 0.0, amax = 0.0;
  size_t imax = 0;
  for (size_t e = 0; e < n; ++e) {
    nrm2 += R[e] * R[e];
    if (std::fabs(R[e]) > amax) {
      amax = std::fabs(R[e]);
      imax = e;
    }
  }
  U.clear();
  Wf.clear();
  if (nrm2 == 0.0) return 0;
  const double thr2 = tol * tol * nrm2;
  int k = 0;
  std::vector<double> u(p), w(q);
  while (true) {
    if (k >= kmax) return -1;
    const int is = (int)(imax / q), js = (int)(imax % q);
    const double piv = R[imax];
    if (piv == 0.0) break;
    for (int i = 0; i < p; ++i) u[i] = R[(size_t)i * q + js];
    for (int j = 0; j < q; ++j) w[j] = R[(size_t)is * q + j] / piv;
    U.insert(U.end(), u.begin(), u.end());
    Wf.insert(Wf.end(), w.begin(), w.end());
    ++k;
    double r2 = 0.0;
    amax = 0.0;
    imax = 0;
    for (int i = 0; i < p; ++i) {
      double* row = &R[(size_t)i * q];
      const double ui = u[i];
      for (int j = 0; j < q; ++j) {
        const double v = row[j] - ui * w[j];
        row[j] = v;
        r2 += v * v;
        if (std::fabs(v) > amax) {
          amax = std::fabs(v);
          imax = (size_t)i * q + j;
        }
      }
    }
    if (r2 <= thr2) break;
  }
  if (k >= kmax) return -1;
  return k;
}

// Adaptive cross approximation with partial pivoting (Bebendorf's construction):
// the block is never formed; row(i, r) and col(j, c) evaluate one row or column,
// and the residual of the rank-k approximation there is that minus the crosses
// so far. Each cross takes the residual row's largest entry as pivot; the next
// row is the largest entry of the new residual column among rows not yet used.
// A cross with |u| |w| <= tol ||S_k||_F (S_k the approximation, its norm updated
// exactly) proposes convergence; residual rows and columns away from the pivots,
// spread over the block, then estimate ||A - S_k||_F, and the worst of those rows
// is the next pivot unless the estimate is within tol ||S_k||_F. Same factor
// layout and return values as aca_full (0: every row evaluated and zero).
template <class Row, class Col>
static int aca_partial(int p, int q, double tol, int kmax, Row&& row, Col&& col, std::vector<double>& U,
                       std::vector<double>& Wf) {
  U.clear();
  Wf.clear();
  std::vector<char> used(p, 0), usedc(q, 0);
  std::vector<double> r(q), c(p), w(q), rc(q), cc(p);
  int k = 0;
  double s2 = 0.0;
  auto residual_row = [&](int ii, double* out) {
    row(ii, out);
    for (int l = 0; l < k; ++l) {
      const double ul = U[(size_t)l * p + ii];
      const double* wl = &Wf[(size_t)l * q];
      for (int j = 0; j < q; ++j) out[j] -= ul * wl[j];
    }
  };
  auto residual_col = [&](int jj, double* out) {
    col(jj, out);
    for (int l = 0; l < k; ++l) {
      const double wl = Wf[(size_t)l * q + jj];
      const double* ul = &U[(size_t)l * p];
      for (int ii = 0; ii < p; ++ii) out[ii] -= wl * ul[ii];
    }
  };
  auto free_from = [](const std::vector<char>& u, int at) {  // first unused index from at, cyclically
    const int n = (int)u.size();
    for (int d = 0; d < n; ++d)
      if (!u[(at + d) % n]) return (at + d) % n;
    return -1;
  };
  const int nchk = std::min(4, std::min(p, q));
  int i = p / 2;
  while (i >= 0) {
    used[i] = 1;
    residual_row(i, r.data());
    int js = 0;
    for (int j = 1; j < q; ++j)
      if (std::fabs(r[j]) > std::fabs(r[js])) js = j;
    if (r[js] == 0.0) {  // row reproduced exactly: take the next unused one
      i = free_from(used, i);
      continue;
    }
    if (k >= kmax) return -1;
    const double piv = r[js];
    for (int j = 0; j < q; ++j) w[j] = r[j] / piv;
    residual_col(js, c.data());
    usedc[js] = 1;
    double cross = 0.0, uu = 0.0, ww = 0.0;
    for (int l = 0; l < k; ++l) {
      double du = 0.0, dw = 0.0;
      for (int ii = 0; ii < p; ++ii) du += U[(size_t)l * p + ii] * c[ii];
      for (int j = 0; j < q; ++j) dw += Wf[(size_t)l * q + j] * w[j];
      cross += du * dw;
    }
    for (int ii = 0; ii < p; ++ii) uu += c[ii] * c[ii];
    for (int j = 0; j < q; ++j) ww += w[j] * w[j];
    s2 += 2.0 * cross + uu * ww;
    U.insert(U.end(), c.begin(), c.end());
    Wf.insert(Wf.end(), w.begin(), w.end());
    ++k;
    int in = -1;
    for (int ii = 0; ii < p; ++ii)
      if (!used[ii] && (in < 0 || std::fabs(c[ii]) > std::fabs(c[in]))) in = ii;
    if (uu * ww <= tol * tol * s2 || in < 0) {
      double er = 0.0, ec = 0.0, worst = -1.0;
      int nr = 0, ncl = 0, iw = -1;
      for (int m = 0; m < nchk; ++m) {
        const int ii = free_from(used, (int)(((2 * m + 1) * (int64_t)p) / (2 * nchk)));
        if (ii >= 0) {
          residual_row(ii, rc.data());
          double e = 0.0;
          for (int j = 0; j < q; ++j) e += rc[j] * rc[j];
          er += e;
          ++nr;
          if (e > worst) {
            worst = e;
            iw = ii;
          }
        }
        const int jj = free_from(usedc, (int)(((2 * m + 1) * (int64_t)q) / (2 * nchk)));
        if (jj >= 0) {
          residual_col(jj, cc.data());
          for (int i2 = 0; i2 < p; ++i2) ec += cc[i2] * cc[i2];
          ++ncl;
        }
      }
      const double est = std::max(nr ? er * p / nr : 0.0, ncl ? ec * q / ncl : 0.0);
      if (est <= tol * tol * s2 || iw < 0) break;
      in = iw;
    }
    i = in;
  }
  if (k >= kmax) return -1;
  return k;  // 0: every row was zero
}

// Orthonormalise the k columns of length n of X in place (Gram-Schmidt, twice);
// R (k x k, row-major, upper triangular) gets X = Q R. A column that vanishes
// against the earlier ones is set to zero with a zero diagonal.
static void thin_qr(std::vector<double>& X, int n, int k, std::vector<double>& R) {
  R.assign((size_t)k * k, 0.0);
  for (int c = 0; c < k; ++c) {
    double* x = &X[(size_t)c * n];
    double n0 = 0.0;
    for (int i = 0; i < n; ++i) n0 += x[i] * x[i];
    for (int pass = 0; pass < 2; ++pass)
      for (int l = 0; l < c; ++l) {
        const double* ql = &X[(size_t)l * n];
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += ql[i] * x[i];
        for (int i = 0; i < n; ++i) x[i] -= d * ql[i];
        R[(size_t)l * k + c] += d;
      }
    double nn = 0.0;
    for (int i = 0; i < n; ++i) nn += x[i] * x[i];
    if (!(nn > 1e-28 * n0)) {
      for (int i = 0; i < n; ++i) x[i] = 0.0;
      continue;
    }
    const double s = std::sqrt(nn);
    R[(size_t)c * k + c] = s;
    for (int i = 0; i < n; ++i) x[i] /= s;
  }
}

// Truncate S = U W^T (rank k, the layout of aca_full) by its singular values:
// U = Qu Ru, W = Qw Rw, Ru Rw^T = X Sigma Y^T by one-sided Jacobi rotations,
// then U <- Qu X_r Sigma_r and W <- Qw Y_r with the smallest r whose dropped
// singular values have a root sum of squares of at most tol ||S||_F. Returns r.
static int svd_truncate(std::vector<double>& U, std::vector<double>& Wf, int p, int q, int k, double tol) {
  std::vector<double> Ru, Rw;
  thin_qr(U, p, k, Ru);
  thin_qr(Wf, q, k, Rw);
  // M = Ru Rw^T, stored by columns: M[c][r] = sum_l Ru[r][l] Rw[c][l]
  std::vector<double> M((size_t)k * k, 0.0), Y((size_t)k * k, 0.0);
  for (int c = 0; c < k; ++c)
    for (int r = 0; r < k; ++r) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += Ru[(size_t)r * k + l] * Rw[(size_t)c * k + l];
      M[(size_t)c * k + r] = s;
    }
  for (int c = 0; c < k; ++c) Y[(size_t)c * k + c] = 1.0;
  // columns of M rotated pairwise until orthogonal: M Y' = X Sigma
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
    for (int a = 0; a < k - 1; ++a)
      for (int b = a + 1; b < k; ++b) {
        double* ma = &M[(size_t)a * k];
        double* mb = &M[(size_t)b * k];
        double aa = 0.0, bb = 0.0, ab = 0.0;
        for (int r = 0; r < k; ++r) {
          aa += ma[r] * ma[r];
          bb += mb[r] * mb[r];
          ab += ma[r] * mb[r];
        }
        if (!(std::fabs(ab) > 1e-15 * std::sqrt(aa * bb))) continue;
        rotated = true;
        const double zeta = (bb - aa) / (2.0 * ab);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cn = 1.0 / std::sqrt(1.0 + t * t), sn = cn * t;
        double* ya = &Y[(size_t)a * k];
        double* yb = &Y[(size_t)b * k];
        for (int r = 0; r < k; ++r) {
          const double x = ma[r], y = mb[r];
          ma[r] = cn * x - sn * y;
          mb[r] = sn * x + cn * y;
          const double u = ya[r], v = yb[r];
          ya[r] = cn * u - sn * v;
          yb[r] = sn * u + cn * v;
        }
      }
    if (!rotated) break;
  }
  std::vector<double> sig(k);
  std::vector<int> ord(k);
  double tot = 0.0;
  for (int c = 0; c < k; ++c) {
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += M[(size_t)c * k + r] * M[(size_t)c * k + r];
    sig[c] = std::sqrt(s);
    tot += s;
    ord[c] = c;
  }
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return sig[x] > sig[y]; });
  int r = k;
  double drop = 0.0;
  while (r > 0 && drop + sig[ord[r - 1]] * sig[ord[r - 1]] <= tol * tol * tot) {
    drop += sig[ord[r - 1]] * sig[ord[r - 1]];
    --r;
  }
  std::vector<double> U2((size_t)r * p, 0.0), W2((size_t)r * q, 0.0);
  for (int l = 0; l < r; ++l) {
    const int c = ord[l];
    const double* m = &M[(size_t)c * k];  // sigma x_c: U' column l = Qu m
    const double* y = &Y[(size_t)c * k];  // W' column l = Qw y_c
    double* u2 = &U2[(size_t)l * p];
    double* w2 = &W2[(size_t)l * q];
    for (int j = 0; j < k; ++j) {
      const double* qu = &U[(size_t)j * p];
      const double* qw = &Wf[(size_t)j * q];
      for (int i = 0; i < p; ++i) u2[i] += qu[i] * m[j];
      for (int i = 0; i < q; ++i) w2[i] += qw[i] * y[j];
    }
  }
  U.swap(U2);
  Wf.swap(W2);
  return r;
}

// ============================================================== 16-bit storage
// Round to nearest even. BF16 keeps the FP32 exponent and 8 significand bits;
// FP16 is IEEE binary16 (values here are scaled into [-1, 1] first).
uint16_t to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float from_bf16(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}
uint16_t to_f16(float x) {
  const _Float16 h = (_Float16)x;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
float from_f16(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (float)h;
}

// power of two >= m (1 for m = 0): values divided by it lie in [-1, 1] exactly scaled
static double pow2_at_least(double m) {
  if (!(m > 0.0)) return 1.0;
  int e;
  const double f = std::frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
  (void)f;
  return std::ldexp(1.0, e);
}

// ============================================================== per-block build
struct LagFactor {
  int T;        // lag (-1 = static tail)
  int rank;     // > 0 low rank, 0 dense
  std::vector<double> U, W, D;  // U: k x p (col l = U[l*p..]), W: k x q, D: p x q row-major
};

// Items of one block for the two evaluation passes: list 0 ("far") is applied
// once per time block of S steps to S history windows at a time; list 1 ("near")
// holds the lags 1..S-1 and the static tail, applied every step. With S = 1 every
// lag and the tail are in list 0.
struct BlockOut {
  std::vector<Item> items[4];
  std::vector<int32_t> lagT[4], lagCol[4];
  std::vector<double> d64;
  std::vector<float> d32;
  std::vector<uint16_t> d16;
  std::vector<float> s32;  // FP32 segment far list
  int64_t stored = 0, dense = 0;
};

// Pack a run of lag factors of one (sub-)block into items of list `L` whose
// kernel evaluates S steps: the history span T_last - T_first + S rows of q
// values, the low-rank columns (times S) and the lag count must fit the LDS
// buffers of the kernel.
static void pack_list(int r0, int r1, int s0, int s1, const Fault& A, const Fault& B,
                      std::vector<LagFactor*>& lags, bool f32, int tail_off, int S, int L, BlockOut& out) {
  const int p = r1 - r0, q = s1 - s0;
  const int64_t target = f32 ? 65536 : 32768;  // elements per item
  auto push = [&](double v) {
    if (f32) out.d32.push_back((float)v);
    else out.d64.push_back(v);
  };
  auto cur_size = [&]() -> int64_t { return f32 ? (int64_t)out.d32.size() : (int64_t)out.d64.size(); };
  size_t i = 0;
  while (i < lags.size()) {
    const bool lr = lags[i]->rank > 0;
    const bool tail = lags[i]->T < 0;
    size_t j = i;
    int64_t elems = 0;
    int ncol = 0;
    while (j < lags.size() && (lags[j]->rank > 0) == lr && (lags[j]->T < 0) == tail) {
      const int nl = (int)(j - i) + 1;
      const int64_t e = lr ? (int64_t)lags[j]->rank * (p + q) : (int64_t)p * q;
      if (j > i) {
        if (tail) break;
        if (lags[j]->T != lags[j - 1]->T + 1) break;  // an item's lags are consecutive
        if (S > 1 && lags[j]->T == 2 * S) break;      // block-start items hold lags below 2S only
        const int span = lags[j]->T - lags[i]->T + S;
        if ((int64_t)span * q > kHistMax) break;
        if (nl > kColMax) break;
        if (lr && (ncol + lags[j]->rank > kColMax || (int64_t)(ncol + lags[j]->rank) * S > kZMax)) break;
        if (elems + e > target) break;
      }
      elems += e;
      if (lr) ncol += lags[j]->rank;
      ++j;
    }
    Item it{};
    it.data = cur_size();  // block-local, rebased later
    it.kind = lr ? 0 : 1;
    it.src = tail ? 1 : 0;
    it.p = p;
    it.q = q;
    it.row0 = A.off + r0;
    it.col0 = B.off + s0;
    it.nlag = (int)(j - i);
    it.lag_off = (int)out.lagT[L].size();
    it.ncol = ncol;
    it.tail_off = tail ? tail_off + s0 : 0;
    for (size_t l = i; l < j; ++l) out.lagT[L].push_back(lags[l]->T);
    out.lagCol[L].push_back(0);
    if (lr) {
      int c = 0;
      for (size_t l = i; l < j; ++l) {
        c += lags[l]->rank;
        out.lagCol[L].push_back(c);
      }
      for (int jj = 0; jj < q; ++jj)  // W panel [q][ncol]
        for (size_t l = i; l < j; ++l)
          for (int r = 0; r < lags[l]->rank; ++r) push(lags[l]->W[(size_t)r * q + jj]);
      for (size_t l = i; l < j; ++l)  // U panel [ncol][p]
        for (int r = 0; r < lags[l]->rank; ++r)
          for (int ii = 0; ii < p; ++ii) push(lags[l]->U[(size_t)r * p + ii]);
    } else {
      for (int l = 0; l < it.nlag; ++l) out.lagCol[L].push_back(0);
      for (size_t l = i; l < j; ++l)  // [nlag][q][p]
        for (int jj = 0; jj < q; ++jj)
          for (int ii = 0; ii < p; ++ii) push(lags[l]->D[(size_t)ii * q + jj]);
    }
    out.stored += elems;
    out.items[L].push_back(it);
    for (size_t l = i; l < j; ++l) {  // release
      std::vector<double>().swap(lags[l]->U);
      std::vector<double>().swap(lags[l]->W);
      std::vector<double>().swap(lags[l]->D);
    }
    i = j;
  }
}

// Pack a run of lag factors of one (sub-)block into items of the segment far
// list for the matrix-core kernel, whose products have ncols = S * nv columns (S
// history windows of nv variants). Values are BF16 / FP16 (dtype) or FP32.
// Layout (rows padded with zeros to q8 / ncol8 values so that every 8-value group
// is one aligned 16- or 32-byte load):
//   dense:    [p][nlag * q8]   row i holds lag 0's q8 values, then lag 1's, ...
//   low rank: W [ncol][q8]     projection rows, lag after lag
//             U [p][ncol8]     expansion rows
// 16-bit values are the factors divided by a power-of-two item scale (dense: the
// item's max |D|; low rank: max |W| times max |U|, each panel scaled on its own),
// so they lie in [-1, 1]; FP32 values are the factors (scale 1). Limits: staged
// history (span * nv * q8 values), the projected panel (ncol8 * ncols values) and
// the lag count.
static void pack_seg(int r0, int r1, int s0, int s1, const Fault& A, const Fault& B,
                     std::vector<LagFactor*>& lags, int dtype, int tail_off, int S, int nv, BlockOut& out,
                     int L = 0) {
  const int p = r1 - r0, q = s1 - s0, q8 = round8(q);
  const int ncols = S * nv;
  const bool f32 = dtype == SEAS_F32;
  const int eb = f32 ? 4 : 2;
  // stored values per item: 1 MiB of factors, so that the fixed cost of an item in
  // the kernel (a barrier and the staging of its history panel, most of which the
  // previous item of the block staged too) is small next to its stream of factors
  const int64_t target = f32 ? 262144 : 524288;
  auto put = [&](double v) {
    if (f32) out.s32.push_back((float)v);
    else out.d16.push_back(dtype == SEAS_BF16 ? to_bf16((float)v) : to_f16((float)v));
  };
  size_t i = 0;
  while (i < lags.size()) {
    const bool lr = lags[i]->rank > 0;
    const bool tail = lags[i]->T < 0;
    size_t j = i;
    int64_t elems = 0;
    int ncol = 0;
    while (j < lags.size() && (lags[j]->rank > 0) == lr && (lags[j]->T < 0) == tail) {
      const int nl = (int)(j - i) + 1;
      const int64_t e = lr ? (int64_t)lags[j]->rank * (p + q) : (int64_t)p * q;
      if (j > i) {
        if (tail) break;
        if (lags[j]->T != lags[j - 1]->T + 1) break;
        if (S > 1 && lags[j]->T == 2 * S) break;  // block-start items hold lags below 2S only
        const int span = lags[j]->T - lags[i]->T + S;
        if ((int64_t)span * nv * seg_ld(q8, eb) > seg_hist_limit(ncols, eb, nv)) break;
        if (nl > kColMax) break;
        if (lr && (int64_t)seg_ld(round8(ncol + lags[j]->rank), eb) * ncols > seg_z_limit(ncols, eb, nv)) break;
        if (elems + e > target) break;
      }
      elems += e;
      if (lr) ncol += lags[j]->rank;
      ++j;
    }
    Item it{};
    it.data = f32 ? (int64_t)out.s32.size() : (int64_t)out.d16.size();  // block-local, rebased later
    it.kind = lr ? 0 : 1;
    it.src = tail ? 1 : 0;
    it.p = p;
    it.q = q;
    it.row0 = A.off + r0;
    it.col0 = B.off + s0;
    it.nlag = (int)(j - i);
    it.lag_off = (int)out.lagT[L].size();
    it.ncol = ncol;
    it.tail_off = tail ? tail_off + s0 : 0;
    for (size_t l = i; l < j; ++l) out.lagT[L].push_back(lags[l]->T);
    out.lagCol[L].push_back(0);
    if (lr) {
      int c = 0;
      double mw = 0.0, mu = 0.0;
      for (size_t l = i; l < j; ++l) {
        c += lags[l]->rank;
        out.lagCol[L].push_back(c);
        for (double v : lags[l]->W) mw = std::max(mw, std::fabs(v));
        for (double v : lags[l]->U) mu = std::max(mu, std::fabs(v));
      }
      const double sw = f32 ? 1.0 : pow2_at_least(mw), su = f32 ? 1.0 : pow2_at_least(mu);
      it.scale = (float)(sw * su);
      const int ncol8 = round8(ncol);
      for (size_t l = i; l < j; ++l)  // W [ncol][q8]
        for (int r = 0; r < lags[l]->rank; ++r)
          for (int jj = 0; jj < q8; ++jj) put(jj < q ? lags[l]->W[(size_t)r * q + jj] / sw : 0.0);
      for (int ii = 0; ii < p; ++ii) {  // U [p][ncol8]
        for (size_t l = i; l < j; ++l)
          for (int r = 0; r < lags[l]->rank; ++r) put(lags[l]->U[(size_t)r * p + ii] / su);
        for (int cc = ncol; cc < ncol8; ++cc) put(0.0);
      }
    } else {
      for (int l = 0; l < it.nlag; ++l) out.lagCol[L].push_back(0);
      double md = 0.0;
      for (size_t l = i; l < j; ++l)
        for (double v : lags[l]->D) md = std::max(md, std::fabs(v));
      const double sd = f32 ? 1.0 : pow2_at_least(md);
      it.scale = (float)sd;
      for (int ii = 0; ii < p; ++ii)  // [p][nlag * q8]
        for (size_t l = i; l < j; ++l)
          for (int jj = 0; jj < q8; ++jj) put(jj < q ? lags[l]->D[(size_t)ii * q + jj] / sd : 0.0);
    }
    out.stored += elems;
    out.items[L].push_back(it);
    for (size_t l = i; l < j; ++l) {
      std::vector<double>().swap(lags[l]->U);
      std::vector<double>().swap(lags[l]->W);
      std::vector<double>().swap(lags[l]->D);
    }
    i = j;
  }
}

// Evaluate, compress and pack the columns [s0, s1) of block bd over the pair's
// window (every lag from max(1, T_init) to T_end; lag 0 is applied through the
// CSR of the lag-0 coupling) and its static tail.
static void build_subblock(const HostOp& op, const BlockDesc& bd, const PairWin& pw, int s0, int s1,
                           BlockOut& out) {
  const Fault& A = op.faults[bd.a];
  const Fault& B = pw.img ? op.images[bd.b] : op.faults[bd.b];
  // an image element carries the opposite slip of its original relative to its own
  // normal (the mirrored normal, negated to keep the element order), so its kernel
  // enters with sign -1
  const double sgn = pw.img ? -1.0 : 1.0;
  const int p = bd.r1 - bd.r0, q = s1 - s0;
  const double cs = op.prm.cs, dt = op.dt;
  const int S = op.time_block;
  const bool lowrank_ok = op.prm.compress && bd.adm;
  // ranks above kmax are stored dense: the factors would not be smaller, and one
  // lag's columns must fit the LDS column buffer of the kernel
  int kmax = std::min<int>({(int)(((int64_t)p * q) / (p + q)), kColMax, kZMax / S});
  if (op.seg) kmax = std::min(kmax, ((seg_z_limit(op.ncols, op.seg_eb, op.n_variants) / op.ncols) & ~7) - 8);
  // ensembles: lags that go to the FP32 list (list 3) meet its projection buffer
  const int kmax32 =
      op.ens32 ? std::min(kmax, ((seg_z_limit(op.ncols, 4, op.n_variants) / op.ncols) & ~7) - 8) : kmax;
  auto in_list3 = [&](int T) { return op.ens32 && !(bd.adm && T >= kEnsSplit); };
  const PairFrame fr = frame(A, B);
  // The corners r1' +- ds/2 of source element j are the offsets of its two edges,
  // and adjacent elements share an edge: the primitive is evaluated once per edge
  // (q + 1 per receiver and time level instead of 2 q). Edge e of the slice lies at
  // s_e = -L/2 + (s0 + e) dx along the source fault; r1' of receiver i from it is
  // its tangential offset from the source centroid minus s_e, and r2' (its normal
  // offset) is the same for every source element of a straight fault.
  const int qe = q + 1;
  std::vector<double> re((size_t)p * qe), r2i(p), C(qe);
  for (int i = 0; i < p; ++i) {
    const double ex = A.midx(bd.r0 + i) - B.cx, ey = A.midy(bd.r0 + i) - B.cy;
    const double along = ex * B.tx + ey * B.ty;
    r2i[i] = ex * B.nx + ey * B.ny;
    for (int e = 0; e < qe; ++e) re[(size_t)i * qe + e] = along - (-0.5 * B.L + (s0 + e) * B.dx);
  }
  auto level = [&](int T, std::vector<double>& G) {  // spatial difference at t = T dt
    const double ct = cs * (T * dt);
    for (int i = 0; i < p; ++i) {
      const double* r1e = &re[(size_t)i * qe];
      for (int e = 0; e < qe; ++e) C[e] = corner(r1e[e], r2i[i], ct, fr.n1, fr.n2);
      double* g = &G[(size_t)i * q];
      for (int j = 0; j < q; ++j) g[j] = sgn * (C[j] - C[j + 1]);
    }
  };
  std::vector<double> G0((size_t)p * q), G1((size_t)p * q), K((size_t)p * q), U, W, R;
  std::vector<LagFactor> lags;
  const int T_lo = std::max(1, pw.T_init), T_hi = bd.T_end;
  out.dense += (int64_t)p * q * (pw.T_end - pw.T_init + 1);
  auto compress = [&](int T) {
    LagFactor lf;
    lf.T = T;
    lf.rank = 0;
    if (lowrank_ok) {
      const int k = aca_full(K.data(), p, q, op.prm.aca_tol, in_list3(T) ? kmax32 : kmax, U, W, R);
      if (k > 0) {
        lf.rank = k;  // U: k columns of length p, W: k columns of length q
        lf.U = U;
        lf.W = W;
      }
    }
    if (lf.rank == 0) lf.D = K;
    lags.push_back(std::move(lf));
  };
  // aca_partial: from the first lag at which cs T dt exceeds every corner distance,
  // each entry of the block takes the primitive's branch behind both fronts at both
  // time levels (a smooth function of the offsets), and those lags are compressed
  // from rows and columns evaluated on demand
  int T_part = INT_MAX;
  if (lowrank_ok && op.prm.aca_partial) {
    double rmax = 0.0;
    for (int i = 0; i < p; ++i)
      for (int e = 0; e < qe; ++e) rmax = std::max(rmax, std::hypot(re[(size_t)i * qe + e], r2i[i]));
    T_part = std::max(T_lo, (int)(rmax / (cs * dt)));
    while (!(cs * (T_part * dt) > rmax)) ++T_part;
  }
  const int T_whole = std::min(T_hi, T_part - 1);
  if (T_whole >= T_lo) level(T_lo, G0);
  for (int T = T_lo; T <= T_whole; ++T) {
    level(T + 1, G1);
    bool any = false;
    for (size_t e = 0; e < K.size(); ++e) {
      K[e] = G1[e] - G0[e];
      any |= K[e] != 0.0;
    }
    std::swap(G0, G1);
    if (any) compress(T);
  }
  // one row or column of lag T, with the arithmetic of level() at T and T + 1
  std::vector<double> C1(qe);
  auto lag_row = [&](int T, int i, double* out) {
    const double c0 = cs * (T * dt), c1 = cs * ((T + 1) * dt);
    const double* r1e = &re[(size_t)i * qe];
    for (int e = 0; e < qe; ++e) {
      C[e] = corner(r1e[e], r2i[i], c0, fr.n1, fr.n2);
      C1[e] = corner(r1e[e], r2i[i], c1, fr.n1, fr.n2);
    }
    for (int j = 0; j < q; ++j) out[j] = sgn * (C1[j] - C1[j + 1]) - sgn * (C[j] - C[j + 1]);
  };
  auto lag_col = [&](int T, int j, double* out) {
    const double c0 = cs * (T * dt), c1 = cs * ((T + 1) * dt);
    for (int i = 0; i < p; ++i) {
      const double* r1e = &re[(size_t)i * qe + j];
      const double g1 = sgn * (corner(r1e[0], r2i[i], c1, fr.n1, fr.n2) - corner(r1e[1], r2i[i], c1, fr.n1, fr.n2));
      const double g0 = sgn * (corner(r1e[0], r2i[i], c0, fr.n1, fr.n2) - corner(r1e[1], r2i[i], c0, fr.n1, fr.n2));
      out[i] = g1 - g0;
    }
  };
  for (int T = std::max(T_lo, T_part); T <= T_hi; ++T) {
    // crosses to a quarter of the tolerance, then the SVD of their sum truncated
    // to the rest: the two errors together stay within aca_tol
    const int km = in_list3(T) ? kmax32 : kmax;
    int k = aca_partial(
        p, q, 0.25 * op.prm.aca_tol, 2 * km, [&](int i, double* o) { lag_row(T, i, o); },
        [&](int j, double* o) { lag_col(T, j, o); }, U, W);
    if (k == 0) continue;  // the whole block-lag is zero
    if (k > 0) k = svd_truncate(U, W, p, q, k, 0.75 * op.prm.aca_tol);
    if (k > 0 && k < km) {
      LagFactor lf;
      lf.T = T;
      lf.rank = k;
      lf.U = U;
      lf.W = W;
      lags.push_back(std::move(lf));
      continue;
    }
    for (int i = 0; i < p; ++i) lag_row(T, i, &K[(size_t)i * q]);  // rank cap: whole block, as above
    compress(T);
  }
  int toff = 0;
  if (op.prm.int_tail) {
    // static tail: stress per unit expired slip, scaled by -1/eta so that the
    // common -eta factor of the evaluation restores it
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < q; ++j)
        K[(size_t)i * q + j] = -sgn * static_stress(A, bd.r0 + i, B, s0 + j, op.prm.mu) / op.eta;
    compress(-1);
    toff = bd.tail_base - bd.s0;  // accumulator of source column s0 + j is toff + s0 + j
  }
  std::vector<LagFactor*> far, near;
  for (auto& lf : lags) {
    if (S == 1 || (lf.T >= S)) far.push_back(&lf);
    else near.push_back(&lf);
  }
  if (op.ens32) {
    // ensembles: the same split as one variant's time-blocked form, admissible
    // blocks' lags >= kEnsSplit in 16 bits, the rest (near-field blocks, the early
    // lags, the static tail) in FP32 on list 3
    std::vector<LagFactor*> l16, l32;
    for (LagFactor* lf : far) (in_list3(lf->T) ? l32 : l16).push_back(lf);
    pack_seg(bd.r0, bd.r1, s0, s1, A, B, l16, op.prm.factor_dtype, toff, S, op.n_variants, out, 0);
    pack_seg(bd.r0, bd.r1, s0, s1, A, B, l32, SEAS_F32, toff, S, op.n_variants, out, 3);
    pack_list(bd.r0, bd.r1, s0, s1, A, B, near, true, toff, 1, 1, out);
    return;
  }
  if (op.seg) {
    // 16-bit near-field blocks (one variant): far lags in FP32. Their entries span
    // the near-singular range of receivers close to a source (fault crossings), and
    // their sums cancel strongly; 16-bit storage of them would set the error.
    if (op.x16 && op.n_variants == 1 && !bd.adm)
      pack_list(bd.r0, bd.r1, s0, s1, A, B, far, true, toff, S, 2, out);
    else
      pack_seg(bd.r0, bd.r1, s0, s1, A, B, far, op.prm.factor_dtype, toff, S, op.n_variants, out);
    pack_list(bd.r0, bd.r1, s0, s1, A, B, near, true, toff, 1, 1, out);
    return;
  }
  const bool f32 = op.prm.factor_dtype == SEAS_F32;
  pack_list(bd.r0, bd.r1, s0, s1, A, B, far, f32, toff, S, 0, out);
  pack_list(bd.r0, bd.r1, s0, s1, A, B, near, f32, toff, 1, 1, out);
}

static void build_block(const HostOp& op, const BlockDesc& bd, const PairWin& pw, BlockOut& out) {
  // a source cluster wider than the kernel's history buffer holds for S rows is
  // packed as column slices, each compressed on its own; for ensembles, receiver
  // clusters taller than a segment's register-held rows are packed as row
  // slices, so that every item can share a segment (one partial set per
  // segment instead of one per item)
  int qmax = kHistMax / op.time_block;
  // (slices as narrow as one default panel: wider slices need ranks above the cap)
  // (FP32 segment builds keep the FP32 slices, which fit their staging buffer)
  if (op.seg) qmax = std::min(op.x16 ? kHistMax : qmax, ((kHist16 * 2 / op.seg_eb / op.ncols) & ~7) - 8);
  if (op.ens32) qmax = std::min(qmax, ((seg_hist_limit(op.ncols, 4, op.n_variants) / op.n_variants) & ~7) - 8);
  const int pmax = (op.seg && op.n_variants > 1) ? seg_rows_max(op.ncols) : bd.r1 - bd.r0;
  const int nrs = (bd.r1 - bd.r0 + pmax - 1) / pmax;
  for (int k = 0; k < nrs; ++k) {
    BlockDesc rs = bd;  // equal row slices
    rs.r0 = bd.r0 + (int)((int64_t)(bd.r1 - bd.r0) * k / nrs);
    rs.r1 = bd.r0 + (int)((int64_t)(bd.r1 - bd.r0) * (k + 1) / nrs);
    for (int s0 = bd.s0; s0 < bd.s1; s0 += qmax) build_subblock(op, rs, pw, s0, std::min(bd.s1, s0 + qmax), out);
  }
}

// ============================================================== driver
static void check_geometry(const std::vector<Fault>& F) {
  for (size_t a = 0; a < F.size(); ++a)
    for (size_t b = 0; b < F.size(); ++b) {
      if (a == b) continue;
      const Fault &A = F[a], &B = F[b];
      for (int i = 0; i < A.Np; ++i)
        for (int e = 0; e <= B.Np; ++e) {
          const double s = -0.5 * B.L + e * B.dx;
          const double d = std::hypot(A.midx(i) - (B.cx + s * B.tx), A.midy(i) - (B.cy + s * B.ty));
          if (d < 1e-6 * B.dx)
            throw Error(SEAS_ERR_INVALID_ARG, "a collocation point lies on another fault's element edge");
        }
    }
}

void build_host(const seas_fault_t* fin, int nf, const seas_params_t& prm, HostOp& op, HostFactors& hf) {
  const auto t_start = std::chrono::steady_clock::now();
  op.prm = prm;
  if (nf < 1) throw Error(SEAS_ERR_INVALID_ARG, "n_faults must be >= 1");
  if (!(prm.mu > 0) || !(prm.cs > 0) || !(prm.beta > 0) || prm.beta > 0.5 + 1e-12)
    throw Error(SEAS_ERR_INVALID_ARG, "mu, cs must be > 0 and 0 < beta <= 1/2");
  if (prm.leaf < 1 || !(prm.eta_H > 0) || !(prm.aca_tol > 0) || !(prm.eta_w > 0))
    throw Error(SEAS_ERR_INVALID_ARG, "leaf >= 1, eta_H > 0, aca_tol > 0, eta_w > 0 required");
  if (prm.factor_dtype < SEAS_F64 || prm.factor_dtype > SEAS_F16)
    throw Error(SEAS_ERR_INVALID_ARG, "factor_dtype must be SEAS_F64, SEAS_F32, SEAS_BF16 or SEAS_F16");
  if (prm.cluster_windows != 0 && prm.cluster_windows != 1)
    throw Error(SEAS_ERR_INVALID_ARG, "cluster_windows must be 0 or 1");
  if (prm.state_update != 0 && prm.state_update != 1)
    throw Error(SEAS_ERR_INVALID_ARG, "state_update must be 0 (explicit) or 1 (closed form at constant rate)");
  if (prm.adaptive_dt != 0 && prm.adaptive_dt != 1) throw Error(SEAS_ERR_INVALID_ARG, "adaptive_dt must be 0 or 1");
  if (prm.adaptive_dt && prm.time_block > 1)
    throw Error(SEAS_ERR_INVALID_ARG, "adaptive_dt needs time_block 0 or 1 (steps of varying length)");
  if (prm.gamma_max < 0 || !(prm.adapt_xi >= 0.0) || !std::isfinite(prm.adapt_xi))
    throw Error(SEAS_ERR_INVALID_ARG, "gamma_max must be >= 0 and adapt_xi finite and >= 0");
  if (prm.time_block < 0 || prm.time_block > kMaxTimeBlock ||
      (prm.time_block & (prm.time_block - 1)) != 0)
    throw Error(SEAS_ERR_INVALID_ARG, "time_block must be 0, 1, 2, 4, 8, 16 or 32");
  op.time_block = prm.time_block > 0 ? prm.time_block : 1;
  op.n_variants = prm.n_variants > 0 ? prm.n_variants : 1;
  op.x16 = prm.factor_dtype == SEAS_BF16 || prm.factor_dtype == SEAS_F16;
  if (op.n_variants > 1) {
    if (!op.x16) throw Error(SEAS_ERR_INVALID_ARG, "ensembles (n_variants > 1) need BF16 or F16 factors");
    if (op.n_variants != 16 && op.n_variants != 32 && op.n_variants != 64)
      throw Error(SEAS_ERR_INVALID_ARG, "n_variants must be 1, 16, 32 or 64");
    if (op.time_block != 1) throw Error(SEAS_ERR_INVALID_ARG, "ensembles use time_block 1");
  } else if (op.x16 && op.time_block != 16) {
    throw Error(SEAS_ERR_INVALID_ARG, "BF16 / F16 factors with one variant need time_block 16");
  }
  op.ncols = op.time_block * op.n_variants;
  op.use_mfma = std::getenv("SEAS_NO_MFMA") == nullptr;
  op.seg = op.x16 || (prm.factor_dtype == SEAS_F32 && (op.time_block == 16 || op.time_block == 32) &&
                      op.use_mfma && std::getenv("SEAS_NO_SEG") == nullptr);
  // 32 windows: the 32-column FP32 instance of the segment kernel
  if (op.time_block == 32 && !(prm.factor_dtype == SEAS_F32 && op.seg))
    throw Error(SEAS_ERR_INVALID_ARG, "time_block 32 needs FP32 factors (the matrix-core segment kernel)");
  op.seg_eb = op.x16 ? 2 : 4;
  op.ens32 = op.x16 && op.n_variants > 1;
  if (prm.n_threads > 0) omp_set_num_threads(prm.n_threads);
  // ---- geometry
  op.faults.clear();
  int off = 0;
  double dxmin = 1e300;
  for (int k = 0; k < nf; ++k) {
    const seas_fault_t& s = fin[k];
    const double nn = std::hypot(s.nx, s.ny);
    if (!(s.length > 0) || s.n_elem < 2 || !(nn > 0) || !std::isfinite(s.cx) || !std::isfinite(s.cy))
      throw Error(SEAS_ERR_INVALID_ARG, "fault " + std::to_string(k) + ": bad length, n_elem, normal or centre");
    Fault f;
    f.cx = s.cx;
    f.cy = s.cy;
    f.nx = s.nx / nn;
    f.ny = s.ny / nn;
    f.tx = -f.ny;
    f.ty = f.nx;
    f.L = s.length;
    f.Np = s.n_elem;
    f.dx = f.L / f.Np;
    f.off = off;
    off += f.Np;
    dxmin = std::min(dxmin, f.dx);
    op.faults.push_back(f);
  }
  op.N = off;
  op.dt = prm.beta * dxmin / prm.cs;
  op.eta = prm.mu / (2.0 * prm.cs);
  check_geometry(op.faults);
  op.images.clear();
  if (prm.free_surface != 0 && prm.free_surface != 1)
    throw Error(SEAS_ERR_INVALID_ARG, "free_surface must be 0 or 1");
  if (prm.self_tail != 0 && prm.self_tail != 1) throw Error(SEAS_ERR_INVALID_ARG, "self_tail must be 0 or 1");
  if (prm.aca_partial != 0 && prm.aca_partial != 1) throw Error(SEAS_ERR_INVALID_ARG, "aca_partial must be 0 or 1");
  if (prm.free_surface) {
    if (!std::isfinite(prm.surface_y)) throw Error(SEAS_ERR_INVALID_ARG, "surface_y must be finite");
    const double y0 = prm.surface_y;
    for (const Fault& f : op.faults) {
      const double tol = 1e-9 * f.L;
      for (int e = 0; e < 2; ++e)
        if (f.cy + (e == 0 ? -0.5 : 0.5) * f.L * f.ty > y0 + tol)
          throw Error(SEAS_ERR_INVALID_ARG, "a fault reaches above the free surface");
      for (int i = 0; i < f.Np; ++i)
        if (!(f.midy(i) < y0 - tol)) throw Error(SEAS_ERR_INVALID_ARG, "a collocation point lies on the free surface");
      // mirror across y = y0; the normal (nx, -ny) negated keeps the tangent the mirror
      // of the original's, so element j of the image is the mirror of element j
      Fault g = f;
      g.cy = 2.0 * y0 - f.cy;
      g.nx = -f.nx;
      g.ny = f.ny;
      g.tx = -g.ny;
      g.ty = g.nx;
      op.images.push_back(g);
    }
  }
  const double cs = prm.cs, dt = op.dt;
  // ---- causality windows (Section 2.3.2, "Truncation of elastodynamic time-window")
  op.pairs.clear();
  op.max_lag = 0;
  // real pairs (a != b) first, then (free surface) every receiver with every image
  for (int img = 0; img < (prm.free_surface ? 2 : 1); ++img)
  for (int a = 0; a < nf; ++a)
    for (int b = 0; b < nf; ++b) {
      if (a == b && !img) continue;
      const Fault &A = op.faults[a], &B = img ? op.images[b] : op.faults[b];
      double earl = 1e300, dmax = 0.0;
      for (int i = 0; i < A.Np; ++i)
        for (int j = 0; j < B.Np; ++j) {
          double r1, r2;
          offsets(A, i, B, j, r1, r2);
          const double r = std::hypot(r1, r2);
          const double ta = (r1 > 0.0 ? std::min(r, std::fabs(r2)) : r) / cs;
          earl = std::min(earl, ta);
        }
      for (int j = 0; j < B.Np; ++j)
        for (int e = 0; e < 2; ++e) {
          const double s = (e == 0 ? -0.5 : 0.5) * A.L;
          dmax = std::max(dmax, std::hypot(B.midx(j) - (A.cx + s * A.tx), B.midy(j) - (A.cy + s * A.ty)));
        }
      PairWin w;
      w.a = a;
      w.b = b;
      w.T_init = (int)std::floor((1.0 - prm.eta_tmin) * earl / dt);
      w.T_end = (int)std::ceil((1.0 + prm.eta_tmax) * dmax / cs / dt);
      w.img = img;
      op.pairs.push_back(w);
      op.max_lag = std::max(op.max_lag, w.T_end);
    }
  op.ring_len = op.max_lag + 3;
  // ---- partition
  std::vector<std::vector<Node>> trees(nf), itrees(op.images.size());
  for (int k = 0; k < nf; ++k) build_tree(op.faults[k], prm.leaf, trees[k]);
  for (size_t k = 0; k < op.images.size(); ++k) build_tree(op.images[k], prm.leaf, itrees[k]);
  op.blocks.assign(op.pairs.size(), {});
  std::vector<BlockDesc> all;
  // tail accumulators: one per (pair, source element), or per (block, source
  // element) with cluster-level windows
  op.tail_off.assign(op.pairs.size(), 0);
  op.tail_len = 0;
  for (size_t pi = 0; pi < op.pairs.size(); ++pi) {
    const PairWin& w = op.pairs[pi];
    traverse(trees[w.a], w.img ? itrees[w.b] : trees[w.b], prm.eta_H, (int)pi, w.a, w.b, op.blocks[pi]);
    op.tail_off[pi] = (int32_t)op.tail_len;
    if (!prm.cluster_windows) op.tail_len += op.faults[w.b].Np;
    const Fault &A = op.faults[w.a], &B = w.img ? op.images[w.b] : op.faults[w.b];
    for (BlockDesc& bd : op.blocks[pi]) {
      bd.T_end = w.T_end;
      bd.tail_base = op.tail_off[pi] + bd.s0;
      if (prm.cluster_windows) {
        // the pair rule on the block: source midpoints to the receiver cluster's end points
        double dmax = 0.0;
        for (int e = 0; e < 2; ++e) {
          const double sa = -0.5 * A.L + (e == 0 ? bd.r0 : bd.r1) * A.dx;
          const double ex = A.cx + sa * A.tx, ey = A.cy + sa * A.ty;
          for (int j = bd.s0; j < bd.s1; ++j) dmax = std::max(dmax, std::hypot(B.midx(j) - ex, B.midy(j) - ey));
        }
        bd.T_end = std::min(w.T_end, (int)std::ceil((1.0 + prm.eta_tmax) * dmax / cs / dt));
        bd.tail_base = (int32_t)op.tail_len;
        op.tail_len += bd.s1 - bd.s0;
      }
    }
    all.insert(all.end(), op.blocks[pi].begin(), op.blocks[pi].end());
  }
  // expired-slip updates per source element: (accumulator, upper lag) entries
  {
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per(op.N);
    for (size_t pi = 0; pi < op.pairs.size(); ++pi) {
      const Fault& B = op.faults[op.pairs[pi].b];
      if (!prm.cluster_windows) {
        for (int j = 0; j < B.Np; ++j) per[B.off + j].push_back({op.tail_off[pi] + j, op.pairs[pi].T_end});
      } else {
        for (const BlockDesc& bd : op.blocks[pi])
          for (int j = bd.s0; j < bd.s1; ++j) per[B.off + j].push_back({bd.tail_base + (j - bd.s0), bd.T_end});
      }
    }
    op.tail_src_ptr.assign(op.N + 1, 0);
    op.tail_src.clear();
    for (int r = 0; r < op.N; ++r) {
      for (auto& e : per[r]) {
        op.tail_src.push_back(e.first);
        op.tail_src.push_back(e.second);
      }
      op.tail_src_ptr[r + 1] = (int32_t)(op.tail_src.size() / 2);
    }
  }
  // ---- lag-0 CSR (pairs whose window starts at lag 0)
  {
    std::vector<std::vector<std::pair<int, double>>> rows(op.N);
    for (const PairWin& w : op.pairs) {
      if (w.T_init != 0) continue;
      const Fault &A = op.faults[w.a], &B = w.img ? op.images[w.b] : op.faults[w.b];
      const double sgn = w.img ? -1.0 : 1.0;
      for (int i = 0; i < A.Np; ++i)
        for (int j = 0; j < B.Np; ++j) {
          const double k0 = sgn * kernel_entry(A, i, B, j, 0, dt, cs);
          if (k0 != 0.0) rows[A.off + i].push_back({B.off + j, k0});
        }
    }
    op.l0_ptr.assign(op.N + 1, 0);
    op.l0_col.clear();
    op.l0_val.clear();
    for (int r = 0; r < op.N; ++r) {
      for (auto& e : rows[r]) {
        op.l0_col.push_back(e.first);
        op.l0_val.push_back(e.second);
      }
      op.l0_ptr[r + 1] = (int32_t)op.l0_col.size();
    }
  }
  // ---- blocks: evaluate, compress, pack (parallel over blocks, largest first)
  std::vector<size_t> order(all.size());
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](const BlockDesc& b) {
    const PairWin& w = op.pairs[b.pair];
    return (double)(b.r1 - b.r0) * (b.s1 - b.s0) * (b.T_end - w.T_init + 1);
  };
  std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost(all[x]) > cost(all[y]); });
  std::vector<BlockOut> outs(all.size());
  std::string err;
  const bool verbose = std::getenv("SEAS_VERBOSE") != nullptr;
  double total_cost = 0.0, done_cost = 0.0;
  for (const auto& b : all) total_cost += cost(b);
  int next_report = 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const size_t bi = order[oi];
    try {
      build_block(op, all[bi], op.pairs[all[bi].pair], outs[bi]);
    } catch (const std::exception& e) {
#pragma omp critical
      err = e.what();
    }
    if (verbose) {
#pragma omp critical
      {
        done_cost += cost(all[bi]);
        if (done_cost >= 0.1 * next_report * total_cost) {
          std::fprintf(stderr, "[seas build] %d%% of block work done (%.0f s)\n", 10 * next_report,
                       std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
          std::fflush(stderr);
          while (done_cost >= 0.1 * next_report * total_cost) ++next_report;
        }
      }
    }
  }
  if (!err.empty()) throw Error(SEAS_ERR_INTERNAL, "block build failed: " + err);
  // ---- global item lists, arena offsets, partial layouts
  for (int L = 0; L < 4; ++L) {
    op.items[L].clear();
    op.lagColOff[L].clear();
  }
  op.seg_ptr3.clear();
  op.arena32s_elems = 0;
  op.n_partials[0] = op.n_partials[1] = 0;
  op.lagT.clear();
  op.lagCol.clear();
  op.seg_ptr.clear();
  op.arena_elems = 0;
  op.arena_near_elems = 0;
  op.stored_entries = 0;
  op.dense_entries = 0;
  const bool f32 = prm.factor_dtype == SEAS_F32;
  const int S = op.time_block;
  hf.f64.assign(all.size(), {});
  hf.f32.assign(all.size(), {});
  hf.f16.assign(all.size(), {});
  hf.f32s.assign(all.size(), {});
  hf.off.assign(all.size(), 0);
  hf.off32.assign(all.size(), 0);
  hf.off3.assign(all.size(), 0);
  std::vector<int32_t> colOff[4];  // lagCol offset of each item, in build order
  for (size_t bi = 0; bi < all.size(); ++bi) {
    BlockOut& bo = outs[bi];
    hf.off[bi] = op.arena_elems;
    hf.off32[bi] = op.arena_near_elems;
    hf.off3[bi] = op.arena32s_elems;
    for (int L = 0; L < 4; ++L) {
      const int lag_base = (int)op.lagT.size();
      int col_cursor = (int)op.lagCol.size();
      // segment operators: the near list and list 2 live in the FP32 near arena,
      // list 3 in its own FP32 arena
      const int64_t base = L == 3 ? op.arena32s_elems
                                  : ((op.seg && L >= 1) ? op.arena_near_elems : op.arena_elems);
      for (Item it : bo.items[L]) {
        it.data += base;
        if (!op.seg || L == 1 || L == 2) it.scale = 1.0f;
        colOff[L].push_back(col_cursor);
        col_cursor += it.nlag + 1;
        it.lag_off += lag_base;
        op.items[L].push_back(it);
      }
      op.lagT.insert(op.lagT.end(), bo.lagT[L].begin(), bo.lagT[L].end());
      op.lagCol.insert(op.lagCol.end(), bo.lagCol[L].begin(), bo.lagCol[L].end());
    }
    if (op.seg) {
      op.arena_elems += op.x16 ? (int64_t)bo.d16.size() : (int64_t)bo.s32.size();
      if (op.ens32) op.arena32s_elems += (int64_t)bo.s32.size();
      op.arena_near_elems += (int64_t)bo.d32.size();
      hf.f16[bi].swap(bo.d16);
      hf.f32s[bi].swap(bo.s32);
      hf.f32[bi].swap(bo.d32);
    } else {
      op.arena_elems += f32 ? (int64_t)bo.d32.size() : (int64_t)bo.d64.size();
      if (f32) hf.f32[bi].swap(bo.d32);
      else hf.f64[bi].swap(bo.d64);
    }
    op.stored_entries += bo.stored;
    op.dense_entries += bo.dense;
  }
  // segment far list: items with the same receiver rows are ordered next to each
  // other and grouped into segments, one workgroup each, that keep the sums of
  // their rows in registers and write one partial set; rows beyond what the
  // registers hold make single-item segments. (FP16 ensembles: also list 3.)
  // block-start items: lags in [S, 2S) (time-blocked builds; never a tail item)
  auto first_item = [&](const Item& it) { return S > 1 && it.src == 0 && op.lagT[it.lag_off] < 2 * S; };
  auto make_segments = [&](std::vector<Item>& items, std::vector<int32_t>& colOffL, std::vector<int32_t>& seg_ptr,
                           int eb) -> int64_t {
    std::vector<size_t> ord(items.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
      const Item &a = items[x], &b = items[y];
      const bool fa = first_item(a), fb = first_item(b);
      if (fa != fb) return fb;
      return a.row0 != b.row0 ? a.row0 < b.row0 : a.p < b.p;
    });
    std::vector<Item> its;
    std::vector<int32_t> co;
    for (size_t x : ord) {
      its.push_back(items[x]);
      co.push_back(colOffL[x]);
    }
    items.swap(its);
    colOffL.swap(co);
    const int rmax = seg_rows_max(op.ncols);
    auto vals = [](const Item& it) {
      const int64_t q8 = round8(it.q);
      return it.kind == 0 ? (int64_t)it.ncol * q8 + (int64_t)it.p * round8(it.ncol) : (int64_t)it.nlag * it.p * q8;
    };
    seg_ptr.clear();
    size_t k = 0;
    while (k < items.size()) {
      const Item& f = items[k];
      size_t e = k + 1;
      int64_t v = vals(f);
      if (f.p <= rmax)
        while (e < items.size() && items[e].row0 == f.row0 && items[e].p == f.p &&
               first_item(items[e]) == first_item(f) && v + vals(items[e]) <= kSegElems * 2 / eb)
          v += vals(items[e++]);
      seg_ptr.push_back((int32_t)k);
      k = e;
    }
    seg_ptr.push_back((int32_t)items.size());
    // workgroups start in segment order: largest segments first, so that the
    // small ones fill in at the end of the pass (block-start segments after all others)
    const size_t ns = seg_ptr.size() - 1;
    std::vector<int64_t> sz(ns, 0);
    std::vector<char> fs(ns, 0);
    int64_t nfirst = 0;
    for (size_t g = 0; g < ns; ++g) {
      for (int32_t x = seg_ptr[g]; x < seg_ptr[g + 1]; ++x) sz[g] += vals(items[x]);
      fs[g] = first_item(items[seg_ptr[g]]);
      nfirst += fs[g];
    }
    std::vector<size_t> so(ns);
    std::iota(so.begin(), so.end(), 0);
    std::stable_sort(so.begin(), so.end(), [&](size_t x, size_t y) {
      return fs[x] != fs[y] ? fs[y] != 0 : sz[x] > sz[y];
    });
    std::vector<Item> its2;
    std::vector<int32_t> co2, sp2;
    for (size_t g : so) {
      sp2.push_back((int32_t)its2.size());
      for (int32_t x = seg_ptr[g]; x < seg_ptr[g + 1]; ++x) {
        its2.push_back(items[x]);
        co2.push_back(colOffL[x]);
      }
    }
    sp2.push_back((int32_t)its2.size());
    items.swap(its2);
    colOffL.swap(co2);
    seg_ptr.swap(sp2);
    // invariants the segment kernel relies on (LDS panel sizes, 16-byte alignment,
    // one row range per segment, register-held rows of multi-item segments)
    for (size_t sg = 0; sg + 1 < seg_ptr.size(); ++sg) {
      const int32_t a = seg_ptr[sg], b = seg_ptr[sg + 1];
      if (b <= a) throw Error(SEAS_ERR_INTERNAL, "empty segment");
      const Item& f = items[a];
      if (b - a > 1 && f.p > rmax) throw Error(SEAS_ERR_INTERNAL, "tall block in a multi-item segment");
      for (int32_t x = a; x < b; ++x) {
        const Item& it = items[x];
        const int q8 = round8(it.q);
        const int span = it.src == 0 ? it.nlag + S - 1 : 1;
        if (it.row0 != f.row0 || it.p != f.p || it.p < 1 || it.q < 1 || it.nlag < 1 ||
            (int64_t)span * op.n_variants * seg_ld(q8, eb) > seg_hist_limit(op.ncols, eb, op.n_variants) ||
            (it.data & 7) != 0 ||
            (it.kind == 0 && (int64_t)seg_ld(round8(it.ncol), eb) * op.ncols > seg_z_limit(op.ncols, eb, op.n_variants)) ||
            (it.src == 1 && op.n_variants == 1) ||
            it.row0 + it.p > op.N || it.col0 + it.q > op.N)
          throw Error(SEAS_ERR_INTERNAL, "segment item violates the kernel's limits");
        if (first_item(it) != first_item(f)) throw Error(SEAS_ERR_INTERNAL, "block-start item in a mixed segment");
      }
    }
    return nfirst;
  };
  // item lists applied by one workgroup per item: block-start items last
  auto move_first_last = [&](int L) {
    std::vector<Item>& its = op.items[L];
    std::vector<size_t> ord(its.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_partition(ord.begin(), ord.end(), [&](size_t x) { return !first_item(its[x]); });
    std::vector<Item> i2;
    std::vector<int32_t> c2;
    for (size_t x : ord) {
      i2.push_back(its[x]);
      c2.push_back(colOff[L][x]);
    }
    its.swap(i2);
    colOff[L].swap(c2);
    op.first_items[L] = 0;
    for (const Item& it : its) op.first_items[L] += first_item(it);
  };
  for (int L = 0; L < 4; ++L) op.first_items[L] = 0;
  op.first_segs = 0;
  if (!op.seg) move_first_last(0);
  move_first_last(2);
  if (op.seg) {
    op.first_segs = make_segments(op.items[0], colOff[0], op.seg_ptr, op.seg_eb);
    for (const Item& it : op.items[0]) op.first_items[0] += first_item(it);
  }
  if (op.ens32) make_segments(op.items[3], colOff[3], op.seg_ptr3, 4);
  // partial offsets: per item, or per segment on the segment far list (far
  // partials are [p][S] or [p][ncols], row-major)
  for (int L = 0; L < 2; ++L) {
    const int SL = L == 0 ? op.ncols : 1;
    auto& its = op.items[L];
    if (op.seg && L == 0) {
      for (size_t sg = 0; sg + 1 < op.seg_ptr.size(); ++sg) {
        const int32_t part = (int32_t)op.n_partials[0];
        for (int32_t x = op.seg_ptr[sg]; x < op.seg_ptr[sg + 1]; ++x) its[x].part = part;
        op.n_partials[0] += (int64_t)its[op.seg_ptr[sg]].p * SL;
      }
    } else {
      for (Item& it : its) {
        it.part = (int32_t)op.n_partials[L];
        op.n_partials[L] += (int64_t)it.p * SL;
      }
    }
    op.lagColOff[L] = colOff[L];
  }
  for (Item& it : op.items[2]) {  // FP32 far items: partials [p][S] in list 0's buffer
    it.part = (int32_t)op.n_partials[0];
    op.n_partials[0] += (int64_t)it.p * op.ncols;
  }
  op.lagColOff[2] = colOff[2];
  for (size_t sg = 0; sg + 1 < op.seg_ptr3.size(); ++sg) {  // list 3: per segment, in list 0's buffer
    const int32_t part = (int32_t)op.n_partials[0];
    for (int32_t x = op.seg_ptr3[sg]; x < op.seg_ptr3[sg + 1]; ++x) op.items[3][x].part = part;
    op.n_partials[0] += (int64_t)op.items[3][op.seg_ptr3[sg]].p * op.ncols;
  }
  op.lagColOff[3] = colOff[3];
  if (op.n_partials[0] > INT32_MAX || op.n_partials[1] > INT32_MAX || (int64_t)op.lagT.size() > INT32_MAX)
    throw Error(SEAS_ERR_INTERNAL, "operator too large for 32-bit item offsets");
  // reduction lists per receiver, in item (segment) order: the base index of the
  // row's partials
  for (int L = 0; L < 2; ++L) {
    const int SL = L == 0 ? op.ncols : 1;
    auto& ptr = op.red_ptr[L];
    auto& idx = op.red_idx[L];
    std::vector<const Item*> heads;
    if (op.seg && L == 0) {
      for (size_t sg = 0; sg + 1 < op.seg_ptr.size(); ++sg) heads.push_back(&op.items[0][op.seg_ptr[sg]]);
      for (const Item& it : op.items[2]) heads.push_back(&it);
      for (size_t sg = 0; sg + 1 < op.seg_ptr3.size(); ++sg) heads.push_back(&op.items[3][op.seg_ptr3[sg]]);
    } else {
      for (const Item& it : op.items[L]) heads.push_back(&it);
    }
    ptr.assign(op.N + 1, 0);
    for (const Item* it : heads)
      for (int i = 0; i < it->p; ++i) ptr[it->row0 + i + 1]++;
    for (int r = 0; r < op.N; ++r) ptr[r + 1] += ptr[r];
    idx.assign(ptr[op.N], 0);
    std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
    for (const Item* it : heads)
      for (int i = 0; i < it->p; ++i) idx[cur[it->row0 + i]++] = it->part + i * SL;
  }
  (void)S;
  // ---- self term (Section 2.3.1): windows, tables shared by identical faults
  op.self.clear();
  op.self_tab.clear();
  op.self_ring_len = 0;
  op.n_modes = 0;
  op.max_self_W = 0;
  op.self_entries = 0;
  struct Key {
    int Np;
    double L;
  };
  std::vector<std::pair<Key, size_t>> seen;
  for (int k = 0; k < nf; ++k) {
    const Fault& f = op.faults[k];
    SelfFault sf;
    sf.Np = f.Np;
    sf.M = 2 * f.Np;
    sf.nm = prm.mode_cap > 0 ? std::min(prm.mode_cap, f.Np) : f.Np;
    sf.mode_off = op.n_modes;
    op.n_modes += sf.nm;
    sf.cfac = prm.mu * prm.cs * M_PI / (2.0 * f.L);
    const int qw = prm.q_w > 0 ? prm.q_w : (int)std::lround(f.Np / 5.0);
    sf.W.resize(sf.nm);
    sf.tail = prm.self_tail;
    for (int n = 1; n <= sf.nm; ++n) {
      double Ln = 1.0;
      if (f.Np / 2.0 - 1.0 > 0.0) Ln = 1.0 / n + (qw - 1.0) / (f.Np / 2.0 - 1.0) * (1.0 - 1.0 / n);
      sf.W[n - 1] = (int)std::floor(prm.eta_w * (f.L / prm.cs) * Ln / dt * (1.0 + 1e-12));
      // the tail is one more lag, W_n + 1, whose coefficient is R_n
      op.max_self_W = std::max(op.max_self_W, sf.W[n - 1] + sf.tail);
      op.self_entries += sf.W[n - 1] + 1 + sf.tail;
    }
    sf.ring_off.resize(sf.nm);
    for (int n = 0; n < sf.nm; ++n) {
      sf.ring_off[n] = op.self_ring_len;
      op.self_ring_len += sf.W[n] + sf.tail;
    }
    size_t reuse = SIZE_MAX;
    for (auto& s : seen)
      if (s.first.Np == f.Np && s.first.L == f.L) reuse = s.second;
    if (reuse != SIZE_MAX && op.self[reuse].W == sf.W) {
      sf.tab_off = op.self[reuse].tab_off;
    } else {
      sf.tab_off.resize(sf.nm);
      int64_t base = (int64_t)op.self_tab.size();
      for (int n = 0; n < sf.nm; ++n) {
        sf.tab_off[n] = base;
        base += sf.W[n] + 1 + sf.tail;
      }
      op.self_tab.resize(base);
#pragma omp parallel for schedule(dynamic, 1)
      for (int n = 1; n <= sf.nm; ++n) {
        double* o = &op.self_tab[sf.tab_off[n - 1]];
        const int W = sf.W[n - 1];
        self_cells(n, W, dt, f.L, prm.cs, o);
        if (sf.tail) o[W + 1] = self_tail_integral(n, (W + 0.5) * dt, f.L, prm.cs);
        const double kn = M_PI * n / f.L;
        for (int T = 0; T <= W + sf.tail; ++T) o[T] *= kn;
      }
      seen.push_back({{f.Np, f.L}, op.self.size()});
    }
    op.self.push_back(sf);
  }
  op.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
}

}  // namespace seas
