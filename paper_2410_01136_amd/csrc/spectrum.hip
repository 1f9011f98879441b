// Host-side builder of the broken power-law table (see spectrum.h).
//
// The lower shares S(a, xb) are integrated upward in t = log2 x from their
// leading small-x power law: dS/dt = ln 2 x^(mu + 1) F(x) / M(mu) with M the
// complete moment (the closed form behind Eq. ji; for G, Eq. jp), six-point
// Gauss-Legendre per table interval.  Their derivatives in the index a
// (mu = (a - 3) / 2) are integrated alongside: d/da of the integrand is the
// integrand times (t ln 2 / 2 - d ln M / da).  The totals at the top of the
// table must come out at 1 and their index derivatives at 0: a check of F, G,
// the quadrature and the closed forms at once.
#include <cmath>
#include <mutex>
#include <vector>

#include "spectrum.h"

namespace sm {
namespace {

constexpr double kLn2 = 0.6931471805599453;

// F(x) = x int_x^inf K_5/3 and G(x) = x K_2/3(x), x > 0, from K_nu(x) =
// int_0^inf e^{-x cosh s} cosh(nu s) ds (exchanging the order of integration,
// int_x^inf K_5/3 = int_0^inf e^{-x cosh s} cosh(5s/3) / cosh s ds).  The
// integrands are even and analytic in a strip about the real axis, so the
// trapezoidal rule on the half line with half weight at s = 0 converges
// geometrically; its step resolves the width ~ x^-1/2 of the peak at s = 0 for
// large x, and terms below e^-64 of the first are dropped.
void synch_fg(double x, double* F, double* G) {
  const double hs = std::fmin(0.1, 0.4 / std::sqrt(x));
  double sf = 0.0, sg = 0.0;
  for (int k = 0;; ++k) {
    const double s = k * hs, c = std::cosh(s);
    if (x * (c - 1.0) > 64.0) break;
    const double e = (k == 0 ? 0.5 : 1.0) * std::exp(-x * c);
    sf += e * std::cosh(5.0 * s / 3.0) / c;
    sg += e * std::cosh(2.0 * s / 3.0);
  }
  *F = x * hs * sf;
  *G = x * hs * sg;
}

// Complete moments int_0^inf x^mu F dx and int_0^inf x^mu G dx.
double moment_f(double mu) {
  return std::pow(2.0, mu + 1.0) / (mu + 2.0) * std::tgamma(0.5 * mu + 7.0 / 3.0) *
         std::tgamma(0.5 * mu + 2.0 / 3.0);
}
double moment_g(double mu) {
  return std::pow(2.0, mu) * std::tgamma(0.5 * mu + 4.0 / 3.0) * std::tgamma(0.5 * mu + 2.0 / 3.0);
}

// Digamma: upward recurrence to x >= 10, then the asymptotic series
// ln x - 1/(2x) - sum B_2k / (2k x^2k) to the x^-10 term.
double digamma(double x) {
  double acc = 0.0;
  for (; x < 10.0; x += 1.0) acc -= 1.0 / x;
  const double r = 1.0 / (x * x);
  return acc + std::log(x) - 0.5 / x -
         r * (1.0 / 12.0 - r * (1.0 / 120.0 - r * (1.0 / 252.0 - r * (1.0 / 240.0 - r / 132.0))));
}

// d ln M / d mu of the two complete moments
double dlnmoment_f(double mu) {
  return std::log(2.0) - 1.0 / (mu + 2.0) + 0.5 * digamma(0.5 * mu + 7.0 / 3.0) +
         0.5 * digamma(0.5 * mu + 2.0 / 3.0);
}
double dlnmoment_g(double mu) {
  return std::log(2.0) + 0.5 * digamma(0.5 * mu + 4.0 / 3.0) + 0.5 * digamma(0.5 * mu + 2.0 / 3.0);
}

// Gauss-Legendre abscissae and weights on [0, 1]: roots of P_n by Newton's
// method from the usual cosine guesses.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1, then up to P_n by the three-term recurrence
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // (2 / ((1 - z^2) P_n'^2)) / 2 on [0, 1]
  }
}

constexpr int kGl = 6;
constexpr int kBelow = 16 * kBpPerOctave;  // intervals below node 0 (t from -56)

// F and G do not depend on the indices: their values at every point the
// builder visits (the start, the nodes and the Gauss-Legendre points of each
// interval) are computed once per process and shared by all tables.
struct FgTable {
  double gx[kGl], gw[kGl];
  double fs, gs;                 // at the start, t = -56
  std::vector<double> fn, gn;    // at the nodes
  std::vector<double> fq, gq;    // at the quadrature points, [interval][kGl]
};

const FgTable& fg_table() {
  static FgTable T;
  static std::once_flag once;
  std::call_once(once, [] {
    const double h = 1.0 / kBpPerOctave;
    gauss_legendre(kGl, T.gx, T.gw);
    synch_fg(std::exp2(kBpT0 - kBelow * h), &T.fs, &T.gs);
    const int nint = kBelow + kBpNodes - 1;
    T.fn.resize(kBpNodes);
    T.gn.resize(kBpNodes);
    T.fq.resize((size_t)nint * kGl);
    T.gq.resize((size_t)nint * kGl);
    for (int j = 0; j < kBpNodes; ++j) synch_fg(std::exp2(kBpT0 + j * h), &T.fn[j], &T.gn[j]);
    for (int i = 0; i < nint; ++i) {
      const double t = kBpT0 + (i - kBelow) * h;
      for (int k = 0; k < kGl; ++k)
        synch_fg(std::exp2(t + T.gx[k] * h), &T.fq[(size_t)i * kGl + k], &T.gq[(size_t)i * kGl + k]);
    }
  });
  return T;
}

}  // namespace

bool bp_build_table(double a1, double a2, float* nodes, std::string* err) {
  const FgTable& T = fg_table();
  const double h = 1.0 / kBpPerOctave;
  const double al[2] = {a1, a2};
  double mu[2], p[2], mF[2], mG[2], dF[2], dG[2];
  for (int i = 0; i < 2; ++i) {
    mu[i] = 0.5 * (al[i] - 3.0);
    p[i] = bp_power(al[i]);
    mF[i] = moment_f(mu[i]);
    mG[i] = moment_g(mu[i]);
    dF[i] = 0.5 * dlnmoment_f(mu[i]);  // d ln M / da
    dG[i] = 0.5 * dlnmoment_g(mu[i]);
  }
  // start: S(t_s) from the leading power law, int_0^xs x^mu A x^(1/3) dx =
  // xs^(mu + 1) F(xs) / p to relative O(xs^(2/3)); its index derivative from
  // the same form
  const double ts = kBpT0 - kBelow * h;
  const double xs = std::exp2(ts), Fs = T.fs, Gs = T.gs;
  double S[4], Sa[4];  // (F, a1), (G, a1), (F, a2), (G, a2) and d/da of each
  for (int i = 0; i < 2; ++i) {
    const double xm = std::pow(xs, mu[i] + 1.0);
    S[2 * i] = xm * Fs / (p[i] * mF[i]);
    S[2 * i + 1] = xm * Gs / (p[i] * mG[i]);
    const double common = 0.5 * ts * kLn2 - 0.5 / p[i];
    Sa[2 * i] = S[2 * i] * (common - dF[i]);
    Sa[2 * i + 1] = S[2 * i + 1] * (common - dG[i]);
  }
  // dS/dt and d2S/da dt of the four shares at t, where F(2^t) = F, G(2^t) = G
  auto rate = [&](double t, double F, double G, double* d, double* da) {
    const double x = std::exp2(t);
    for (int i = 0; i < 2; ++i) {
      const double xm = kLn2 * std::pow(x, mu[i] + 1.0);
      d[2 * i] = xm * F / mF[i];
      d[2 * i + 1] = xm * G / mG[i];
      da[2 * i] = d[2 * i] * (0.5 * t * kLn2 - dF[i]);
      da[2 * i + 1] = d[2 * i + 1] * (0.5 * t * kLn2 - dG[i]);
    }
  };
  float* part1 = nodes + kBpPartFloats;
  for (int j = -kBelow; j < kBpNodes; ++j) {
    const double t = kBpT0 + j * h;
    if (j >= 0) {
      double d[4], da[4];
      rate(t, T.fn[j], T.gn[j], d, da);
      float* o = nodes + (size_t)j * 8;
      float* oa = part1 + (size_t)j * 8;
      for (int c = 0; c < 4; ++c) {
        // g = S E, E = 2^(-p t), dE/da = -(t ln2 / 2) E
        const double pc = p[c / 2], E = std::exp2(-pc * t);
        const double gt = (d[c] - pc * kLn2 * S[c]) * E;
        o[c] = (float)(S[c] * E);
        o[4 + c] = (float)(h * gt);
        oa[c] = (float)((Sa[c] - 0.5 * t * kLn2 * S[c]) * E);
        oa[4 + c] = (float)(h * ((da[c] - 0.5 * kLn2 * S[c] - pc * kLn2 * Sa[c]) * E -
                                 0.5 * t * kLn2 * gt));
      }
    }
    if (j == kBpNodes - 1) break;
    const size_t iq = (size_t)(j + kBelow) * kGl;
    for (int k = 0; k < kGl; ++k) {
      double d[4], da[4];
      rate(t + T.gx[k] * h, T.fq[iq + k], T.gq[iq + k], d, da);
      for (int c = 0; c < 4; ++c) {
        S[c] += h * T.gw[k] * d[c];
        Sa[c] += h * T.gw[k] * da[c];
      }
    }
  }
  // above the table every share is 1 to ~e^-128 whatever the index: the running
  // totals must be 1 and their index derivatives 0
  for (int c = 0; c < 4; ++c) {
    if (!(std::fabs(S[c] - 1.0) < 1e-9) || !(std::fabs(Sa[c]) < 1e-8)) {
      if (err) *err = "broken power-law table: moment quadrature missed its closed form";
      return false;
    }
  }
  return true;
}

}  // namespace sm
