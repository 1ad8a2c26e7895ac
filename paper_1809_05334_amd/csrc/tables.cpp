// Host tables of libvie: quadrature rules, special functions and the per-fill
// Ewald lattice-sum tables (Sec. 2.2, Eqs. 3-4 and the Ewald split).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <thread>
#include <vector>

#include "host.h"

namespace vie {

static const double kPi = 3.14159265358979323846;
static const double kSqrtPi = 1.77245385090551602730;

// ---------------------------------------------------------------- Gauss-Legendre
// Nodes/weights on [0, 1] by Newton iteration on the Legendre three-term
// recurrence, in extended precision.
using ld = long double;
using zl = std::complex<long double>;

static void gauss_legendre01(int n, std::vector<ld> &x, std::vector<ld> &w) {
  x.resize(n);
  w.resize(n);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    ld dp = 1;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = 0;
      for (int k = 1; k <= n; ++k) {
        ld p2 = p1;
        p1 = p0;
        p0 = ((2 * k - 1) * z * p1 - (k - 1) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1);
      ld dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    ld p0 = 1, p1 = 0;
    for (int k = 1; k <= n; ++k) {
      ld p2 = p1;
      p1 = p0;
      p0 = ((2 * k - 1) * z * p1 - (k - 1) * p2) / k;
    }
    dp = n * (z * p0 - p1) / (z * z - 1);
    x[i] = 0.5L * (1 - z);
    w[i] = 1.0L / ((1 - z * z) * dp * dp);  // (2 / ((1-z^2) P'^2)) / 2
  }
}

struct GL {
  std::vector<ld> x32, w32, x24, w24;
  GL() {
    gauss_legendre01(32, x32, w32);
    gauss_legendre01(24, x24, w24);
  }
};
static const GL &gl() {
  static GL g;
  return g;
}

// ---------------------------------------------------------------- special functions
// erfcx(z) = (2/sqrt(pi)) int_0^inf exp(-s^2 - 2 z s) ds, used for Re z >= 0 (the
// integrand is bounded by 1 there).  Composite Gauss-Legendre up to where the
// integrand falls below 1e-20, accumulated in extended precision.
static const ld kSqrtPiL = 1.772453850905516027298167483341145183L;

static zl erfcx_integral(zl z) {
  const GL &g = gl();
  ld x = z.real();
  ld S = -x + std::sqrt(x * x + 46.0L);
  const int panels = 12;
  zl acc = 0;
  for (int p = 0; p < panels; ++p) {
    ld lo = S * p / panels, h = S / panels;
    for (size_t i = 0; i < g.x24.size(); ++i) {
      ld s = lo + h * g.x24[i];
      acc += h * g.w24[i] * std::exp(-s * s - 2.0L * z * s);
    }
  }
  return acc * (2.0L / kSqrtPiL);
}

// erf(z) = (2 z / sqrt(pi)) int_0^1 exp(-z^2 t^2) dt  (moderate |z|)
static zl erf_integral(zl z) {
  const GL &g = gl();
  zl acc = 0;
  for (size_t i = 0; i < g.x32.size(); ++i) {
    ld t = g.x32[i];
    acc += g.w32[i] * std::exp(-z * z * (t * t));
  }
  return acc * z * (2.0L / kSqrtPiL);
}

static zl erfcx_l(zl z) {
  if (z.real() >= 0) return erfcx_integral(z);
  return 2.0L * std::exp(z * z) - erfcx_integral(-z);
}

static zl erfc_l(zl z) {
  if (z.real() >= 0.5L) return std::exp(-z * z) * erfcx_integral(z);
  if (z.real() <= -0.5L) return 2.0L - std::exp(-z * z) * erfcx_integral(-z);
  return 1.0L - erf_integral(z);
}

zd erfcx_c(zd z) {
  zl r = erfcx_l(zl(z.real(), z.imag()));
  return zd((double)r.real(), (double)r.imag());
}

zd erfc_c(zd z) {
  zl r = erfc_l(zl(z.real(), z.imag()));
  return zd((double)r.real(), (double)r.imag());
}

static ld erfi_l(ld y) {
  const GL &g = gl();
  ld acc = 0;
  for (size_t i = 0; i < g.x32.size(); ++i) {
    ld t = g.x32[i];
    acc += g.w32[i] * std::exp(y * y * t * t);
  }
  return acc * y * (2.0L / kSqrtPiL);
}

double erfi_r(double y) { return (double)erfi_l(y); }

// ---------------------------------------------------------------- quadrature
static double tet14_residual(const double p[6], double r[6]) {
  // exactness on one homogeneous degree-5 barycentric monomial per partition
  static const int parts[6][4] = {{5, 0, 0, 0}, {4, 1, 0, 0}, {3, 2, 0, 0},
                                  {3, 1, 1, 0}, {2, 2, 1, 0}, {2, 1, 1, 1}};
  auto fact = [](int n) {
    double f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  double pts[14][4], w[14];
  int c = 0;
  for (int o = 0; o < 2; ++o) {
    double a = p[2 * o], wa = p[2 * o + 1];
    for (int k = 0; k < 4; ++k, ++c) {
      for (int j = 0; j < 4; ++j) pts[c][j] = j == k ? 1 - 3 * a : a;
      w[c] = wa;
    }
  }
  static const int pr[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int k = 0; k < 6; ++k, ++c) {
    for (int j = 0; j < 4; ++j) pts[c][j] = (j == pr[k][0] || j == pr[k][1]) ? p[4] : 0.5 - p[4];
    w[c] = p[5];
  }
  double nrm = 0;
  for (int e = 0; e < 6; ++e) {
    double exact = 6.0 * fact(parts[e][0]) * fact(parts[e][1]) * fact(parts[e][2]) * fact(parts[e][3]) / fact(8);
    double s = 0;
    for (int i = 0; i < 14; ++i) {
      double m = w[i];
      for (int j = 0; j < 4; ++j) m *= std::pow(pts[i][j], parts[e][j]);
      s += m;
    }
    r[e] = s - exact;
    nrm = std::max(nrm, std::fabs(r[e]));
  }
  return nrm;
}

// Solve the 6x6 moment system of the symmetric 14-point degree-5 rule
// (two (a,a,a,1-3a) orbits and one (b,b,1/2-b,1/2-b) orbit) by Newton's method.
static void solve_tet14(double p[6]) {
  double start[6] = {0.0927, 0.0735, 0.3109, 0.1127, 0.0455, 0.0425};
  std::memcpy(p, start, sizeof(start));
  for (int it = 0; it < 60; ++it) {
    double r[6], J[6][6];
    if (tet14_residual(p, r) < 1e-17) break;
    for (int k = 0; k < 6; ++k) {
      double pp[6], pm[6], rp[6], rm[6];
      std::memcpy(pp, p, sizeof(pp));
      std::memcpy(pm, p, sizeof(pm));
      double h = 1e-7 * std::max(1.0, std::fabs(p[k]));
      pp[k] += h;
      pm[k] -= h;
      tet14_residual(pp, rp);
      tet14_residual(pm, rm);
      for (int e = 0; e < 6; ++e) J[e][k] = (rp[e] - rm[e]) / (2 * h);
    }
    // Gaussian elimination with partial pivoting on J dp = -r
    double A[6][7];
    for (int e = 0; e < 6; ++e) {
      for (int k = 0; k < 6; ++k) A[e][k] = J[e][k];
      A[e][6] = -r[e];
    }
    for (int c = 0; c < 6; ++c) {
      int piv = c;
      for (int e = c + 1; e < 6; ++e)
        if (std::fabs(A[e][c]) > std::fabs(A[piv][c])) piv = e;
      for (int k = 0; k < 7; ++k) std::swap(A[c][k], A[piv][k]);
      for (int e = c + 1; e < 6; ++e) {
        double f = A[e][c] / A[c][c];
        for (int k = c; k < 7; ++k) A[e][k] -= f * A[c][k];
      }
    }
    double dp[6];
    for (int c = 5; c >= 0; --c) {
      double s = A[c][6];
      for (int k = c + 1; k < 6; ++k) s -= A[c][k] * dp[k];
      dp[c] = s / A[c][c];
    }
    for (int k = 0; k < 6; ++k) p[k] += dp[k];
  }
}

void build_quadrature(QuadRules &q) {
  const double al = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0, be = (5.0 - std::sqrt(5.0)) / 20.0;
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) q.tet4[i][j] = i == j ? al : be;
    q.w4[i] = 0.25;
  }
  double p[6];
  solve_tet14(p);
  int c = 0;
  for (int o = 0; o < 2; ++o)
    for (int k = 0; k < 4; ++k, ++c) {
      for (int j = 0; j < 4; ++j) q.tet14[c][j] = j == k ? 1 - 3 * p[2 * o] : p[2 * o];
      q.w14[c] = p[2 * o + 1];
    }
  static const int pr[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int k = 0; k < 6; ++k, ++c) {
    for (int j = 0; j < 4; ++j) q.tet14[c][j] = (j == pr[k][0] || j == pr[k][1]) ? p[4] : 0.5 - p[4];
    q.w14[c] = p[5];
  }
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) q.tri3[i][j] = i == j ? 2.0 / 3.0 : 1.0 / 6.0;
    q.w3[i] = 1.0 / 3.0;
  }
  const double s15 = std::sqrt(15.0);
  const double b1 = (6.0 - s15) / 21.0, b2 = (6.0 + s15) / 21.0;
  const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  q.tri7[0][0] = q.tri7[0][1] = q.tri7[0][2] = 1.0 / 3.0;
  q.w7[0] = 9.0 / 40.0;
  c = 1;
  for (int o = 0; o < 2; ++o) {
    double bb = o == 0 ? b1 : b2, ww = o == 0 ? w1 : w2;
    for (int k = 0; k < 3; ++k, ++c) {
      for (int j = 0; j < 3; ++j) q.tri7[c][j] = j == k ? 1 - 2 * bb : bb;
      q.w7[c] = ww;
    }
  }
}

// ---------------------------------------------------------------- Chebyshev fits
// Interpolate f on [lo, hi] at n first-kind Chebyshev nodes; coefficients with
// c[0] halved (so f(t) = sum_k c_k T_k(t)).  A coefficient counts when it
// exceeds thr = max(abs_tol, rel_tol * max|f|); the series has converged when
// the last eight coefficients sit at that noise level.  The kept degree is
// the last counting coefficient.  Returns the degree, or -1 if neither 48 nor
// 96 nodes converge within maxdeg.
template <class F>
static int cheb_fit(F f, double lo, double hi, double abs_tol, double rel_tol, double *out, int maxdeg) {
  for (int n : {48, 96}) {
    std::vector<ld> fx(n);
    std::vector<double> c(n);
    double fmax = 0;
    for (int j = 0; j < n; ++j) {
      double t = (double)std::cos(3.141592653589793238462643383279502884L * (j + 0.5L) / n);
      fx[j] = f(lo + 0.5 * (t + 1) * (hi - lo));
      fmax = std::max(fmax, (double)std::fabs(fx[j]));
    }
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < n; ++k) {
      ld s = 0;
      for (int j = 0; j < n; ++j) s += fx[j] * std::cos(pi * k * (j + 0.5L) / n);
      c[k] = (double)(2.0L * s / n);
    }
    c[0] *= 0.5;
    const double thr = std::max(abs_tol, rel_tol * fmax);
    double tailmax = 0;
    for (int k = n - 8; k < n; ++k) tailmax = std::max(tailmax, std::fabs(c[k]));
    int deg = 0;
    for (int k = n - 1; k >= 1; --k)
      if (std::fabs(c[k]) > thr) {
        deg = k;
        break;
      }
    if (tailmax <= 16 * thr && deg <= maxdeg) {
      for (int k = 0; k <= deg; ++k) out[k] = c[k];
      for (int k = deg + 1; k <= maxdeg; ++k) out[k] = 0;
      return deg;
    }
  }
  return -1;
}

// Run body(i) for i in [0, n) on up to 16 host threads.
template <class Fn>
static void parallel_for(int n, Fn body) {
  const int nth = std::max(1, std::min<int>({16, n, (int)std::thread::hardware_concurrency()}));
  std::atomic<int> next(0);
  auto work = [&]() {
    for (int i = next++; i < n; i = next++) body(i);
  };
  std::vector<std::thread> th;
  for (int k = 1; k < nth; ++k) th.emplace_back(work);
  work();
  for (auto &t : th) t.join();
}

// ---------------------------------------------------------------- Ewald tables
std::string build_pgf_table(PgfTable &tab, double a, double b, double zspan, double lambda, double theta,
                            double phi, double *wood_margin) {
  std::memset(&tab, 0, sizeof(tab));
  const double k0 = 2 * kPi / lambda;
  const double kx = k0 * std::sin(theta) * std::cos(phi), ky = k0 * std::sin(theta) * std::sin(phi);
  const double E = std::sqrt(kPi / (a * b));
  const double y = k0 / (2 * E);
  tab.a = a;
  tab.b = b;
  tab.inv_a = 1 / a;
  tab.inv_b = 1 / b;
  tab.E = E;
  tab.k0 = k0;
  tab.kx = kx;
  tab.ky = ky;
  tab.two_pi_a = 2 * kPi / a;
  tab.two_pi_b = 2 * kPi / b;
  for (int m0 = -1; m0 <= 1; ++m0)
    for (int n0 = -1; n0 <= 1; ++n0) {
      double ph = -(kx * m0 * a + ky * n0 * b);
      tab.ph0re[(m0 + 1) * 3 + (n0 + 1)] = std::cos(ph);
      tab.ph0im[(m0 + 1) * 3 + (n0 + 1)] = std::sin(ph);
    }

  // Wood-anomaly margin over the non-specular orders
  double margin = 1e300;
  for (int p = -kPgfM; p <= kPgfM; ++p)
    for (int q = -kPgfM; q <= kPgfM; ++q) {
      if (p == 0 && q == 0) continue;
      double tx = kx + 2 * kPi * p / a, ty = ky + 2 * kPi * q / b;
      margin = std::min(margin, std::sqrt(std::fabs(tx * tx + ty * ty - k0 * k0)) / k0);
    }
  margin = std::min(margin, std::cos(theta));
  *wood_margin = margin;
  if (margin < 0.02) return "";  // the caller reports the anomaly; no tables near gamma = 0

  // Accuracy of the tables: a term is dropped when it stays below 1e-16 of
  // g_p's size at the largest in-cell separation, and the fits resolve every
  // term to 1e-15 (absolute) / 1e-14 (relative).  The lattice sum then stays
  // within a few 1e-13 of its converged value (relative), three orders of
  // magnitude inside what the fill is held to (1e-10 of each Z entry).
  const double G = 1.0 / (4 * kPi * std::sqrt(a * a + b * b + zspan * zspan));
  const double sig = 1e-16 * G;
  const double fit_abs = 1e-15, fit_rel = 1e-14;

  const ld yl = y;
  const ld erfi_y = erfi_l(yl);
  auto Fx = [&](double x) -> ld {
    // exp(y^2 - x^2) Re erfcx(x - j y) = Re[e^{-2jxy} erfc(x - jy)]   (x >= 0.5)
    const ld xl = x;
    return std::exp(yl * yl - xl * xl) * erfcx_integral(zl(xl, -yl)).real();
  };
  auto Hx = [&](double x) -> ld {
    // (F(x) - 1)/x = [-2 sin^2(xy) + sin(2xy) erfi(y) - Re(e^{-2jxy} I(x))]/x,
    // I(x) = (2/sqrt(pi)) int_0^x exp(-(s - jy)^2) ds  (no cancellation near x = 0)
    const ld xl = x;
    if (x > 3.0) return (Fx(x) - 1.0L) / xl;
    if (x == 0.0) return 2 * yl * erfi_y - 2 * std::exp(yl * yl) / kSqrtPiL;
    const GL &g = gl();
    zl I = 0;
    for (size_t i = 0; i < g.x32.size(); ++i) {
      ld s = xl * g.x32[i];
      zl d(s, -yl);
      I += g.w32[i] * std::exp(-d * d);
    }
    I *= xl * 2.0L / kSqrtPiL;
    ld sxy = std::sin(xl * yl);
    ld val = -2 * sxy * sxy + std::sin(2 * xl * yl) * erfi_y - (std::exp(zl(0, -2 * xl * yl)) * I).real();
    return val / xl;
  };
  auto Ffull = [&](double x) -> ld { return x >= 0.5 ? Fx(x) : 1.0L + (ld)x * Hx(x); };

  // ---- spatial images: significance cut first, then the fits in parallel
  struct ImgJob {
    int m, n;
    double xlo, xhi;
    bool touching;
  };
  std::vector<ImgJob> jobs;
  for (int m = -kPgfM; m <= kPgfM; ++m)
    for (int n = -kPgfM; n <= kPgfM; ++n) {
      double dxlo = std::max(0.0, (std::abs(m) - 0.5) * a), dylo = std::max(0.0, (std::abs(n) - 0.5) * b);
      double dxhi = (std::abs(m) + 0.5) * a, dyhi = (std::abs(n) + 0.5) * b;
      double Rlo = std::sqrt(dxlo * dxlo + dylo * dylo) * (1 - 1e-9);
      double Rhi = std::sqrt(dxhi * dxhi + dyhi * dyhi + zspan * zspan) * (1 + 1e-9);
      double xlo = Rlo * E, xhi = Rhi * E;
      bool touching_class = std::abs(m) <= 1 && std::abs(n) <= 1;
      if (!touching_class && Rlo > 0 && std::exp(y * y - xlo * xlo) / (4 * kPi * Rlo) < sig) continue;
      jobs.push_back({m, n, xlo, xhi, touching_class});
    }
  tab.nimg = (int)jobs.size();
  std::atomic<int> bad(0);
  parallel_for((int)jobs.size(), [&](int i) {
    const ImgJob &jb = jobs[i];
    PgfImage &im = tab.img[i];
    im.m = jb.m;
    im.n = jb.n;
    im.xa = jb.xlo;
    im.xs = 2.0 / (jb.xhi - jb.xlo);
    double ph = kx * jb.m * a + ky * jb.n * b;
    im.cre = std::cos(ph) / (4 * kPi);
    im.cim = std::sin(ph) / (4 * kPi);
    im.deg = cheb_fit(Ffull, jb.xlo, jb.xhi, fit_abs, fit_rel, im.f, kPgfMaxDeg - 1);
    im.hdeg = -1;
    if (jb.touching) im.hdeg = cheb_fit(Hx, jb.xlo, jb.xhi, 0.0, fit_rel, im.h, kPgfMaxDeg - 1);
    if (im.deg < 0 || (jb.touching && im.hdeg < 0)) bad = 1;
  });
  if (bad) return "lattice-sum table: spatial fit did not converge";

  // ---- spectral modes, K_pq as a function of w = (z E)^2 on [0, (zspan E)^2]
  const double wmax = std::max(1e-30, zspan * E * zspan * E) * (1 + 1e-9);
  tab.ws = 2.0 / wmax;
  parallel_for(kPgfTerms, [&](int idx) {
      const int p = idx / kPgfSide - kPgfM, q = idx % kPgfSide - kPgfM;
      double tx = kx + 2 * kPi * p / a, ty = ky + 2 * kPi * q / b;
      double kt2 = tx * tx + ty * ty;
      PgfMode &md = tab.mode[(p + kPgfM) * kPgfSide + (q + kPgfM)];
      md.deg = -1;
      md.p = p;
      md.q = q;
      if (kt2 > k0 * k0) {
        double gam = std::sqrt(kt2 - k0 * k0);
        double u = gam / (2 * E);
        double pref = 1.0 / (4 * a * b * gam);
        auto K = [&](double w) -> ld {
          const ld v = std::sqrt(std::max(0.0L, (ld)w)), ul = u;
          const ld t1 = std::exp(-ul * ul - v * v) * erfcx_l(zl(ul + v, 0)).real();
          const ld t2 = std::exp(-ul * ul - v * v) * erfcx_l(zl(ul - v, 0)).real();
          return (ld)pref * (t1 + t2);
        };
        double kmax = 0;
        for (int j = 0; j <= 16; ++j) kmax = std::max(kmax, (double)std::fabs(K(wmax * j / 16.0)));
        if (kmax < sig) return;  // deg stays -1
        md.cplx = 0;
        md.deg = cheb_fit(K, 0.0, wmax, sig, fit_rel, md.kre, kPgfMaxDeg - 1);
        if (md.deg < 0) bad = 1;
      } else {
        // propagating order: gamma = +j beta
        double beta = std::sqrt(k0 * k0 - kt2);
        double bb = beta / (2 * E);
        const zl pref = 1.0L / (4.0L * a * b * zl(0, beta));
        auto Kc = [&](double w) -> zl {
          const ld v = std::sqrt(std::max(0.0L, (ld)w)), bl = bb;
          const zl e1 = std::exp(zl(0, 2 * bl * v)), e2 = std::exp(zl(0, -2 * bl * v));
          return pref * (e1 * erfc_l(zl(v, bl)) + e2 * erfc_l(zl(-v, bl)));
        };
        md.cplx = 1;
        int d1 = cheb_fit([&](double w) { return Kc(w).real(); }, 0.0, wmax, sig, fit_rel, md.kre, kPgfMaxDeg - 1);
        int d2 = cheb_fit([&](double w) { return Kc(w).imag(); }, 0.0, wmax, sig, fit_rel, md.kim, kPgfMaxDeg - 1);
        if (d1 < 0 || d2 < 0) bad = 1;
        md.deg = std::max(d1, d2);
      }
    });
  if (bad) return "lattice-sum table: spectral fit did not converge";
  return "";
}

// ---------------------------------------------------------------- packing
// An integer field of the packed table: its value in the low 32 bits of the
// double slot (the device reads the register half, no conversion).
static double ibits(int v, int hi = 0) {
  const uint64_t u = (uint64_t)(uint32_t)hi << 32 | (uint32_t)v;
  double d;
  std::memcpy(&d, &u, sizeof d);
  return d;
}

void pack_pgf_table(const PgfTable &tab, std::vector<double> &out) {
  auto pad4 = [](int n) { return (n + 3) & ~3; };
  out.assign(kPackImages, 0.0);
  const double hdr[10] = {tab.E, tab.a, tab.b, tab.inv_a, tab.inv_b, tab.kx, tab.ky, tab.two_pi_a, tab.two_pi_b, tab.ws};
  for (int i = 0; i < 10; ++i) out[i] = hdr[i];
  for (int i = 0; i < 9; ++i) {
    out[10 + i] = tab.ph0re[i];
    out[19 + i] = tab.ph0im[i];
  }
  out[28] = ibits(tab.nimg);
  for (int i = 0; i < tab.nimg; ++i) {
    const PgfImage &im = tab.img[i];
    const int K = pad4(im.deg), HK = im.hdeg >= 0 ? pad4(im.hdeg) : -1;
    const size_t start = out.size();
    // the fit's argument t = (x - xa) xs - 1 with x = E R, stored as t = R (E xs) - (xa xs + 1)
    out.insert(out.end(), {tab.E * im.xs, -(im.xa * im.xs + 1.0), im.cre, im.cim, ibits(im.m), ibits(im.n), ibits(K), 0.0});
    for (int k = 0; k < pad4(K + 1); ++k) out.push_back(k <= im.deg ? im.f[k] : 0.0);
    if (HK >= 0) {
      out.insert(out.end(), {ibits(HK), 0.0, 0.0, 0.0});
      for (int k = 0; k < pad4(HK + 1); ++k) out.push_back(k <= im.hdeg ? im.h[k] : 0.0);
    }
    out[start + 7] = ibits((int)(out.size() - start));
  }
  for (int idx = 0; idx < kPgfTerms; ++idx) {
    const PgfMode &md = tab.mode[idx];
    if (md.deg < 0) continue;
    const int K = pad4(md.deg);
    out[32 + idx] = ibits((int)out.size(), K | (md.cplx ? 1 << 16 : 0));
    out.insert(out.end(), {ibits(K), ibits(md.cplx), 0.0, 0.0});
    for (int k = 0; k < pad4(K + 1); ++k) out.push_back(k <= md.deg ? md.kre[k] : 0.0);
    if (md.cplx)
      for (int k = 0; k < pad4(K + 1); ++k) out.push_back(k <= md.deg ? md.kim[k] : 0.0);
  }
  // each row's range of q with a mode, so that a pass over the grid skips the rest
  for (int p = 0; p < kPgfSide; ++p) {
    int lo = kPgfSide, hi = -1;
    for (int q = 0; q < kPgfSide; ++q)
      if (tab.mode[p * kPgfSide + q].deg >= 0) {
        lo = std::min(lo, q);
        hi = std::max(hi, q);
      }
    out[kPackRows + p] = ibits(hi < 0 ? 0 : lo | (hi + 1) << 8);
  }
}

}  // namespace vie
