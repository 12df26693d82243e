// Uniform theory of diffraction for a wedge (Sec. II-E): the four
// cot * F terms of the Kouyoumjian-Pathak coefficient, evaluated in FP64 per
// diffracted path.
//
// Transition function F(x) = 2j sqrt(x) e^{jx} int_{sqrt(x)}^inf e^{-j t^2} dt:
//   x < 4:  int_0^a e^{-j t^2} dt as its power series sum (-j)^m a^{2m+1} /
//           (m! (2m+1)) (at most ~35 terms to reach FP64 rounding), subtracted
//           from the full integral sqrt(pi)/2 e^{-j pi/4};
//   x >= 4: with z = a e^{j pi/4} the tail is e^{-j pi/4} int_z^inf e^{-t^2} dt,
//           and Laplace's continued fraction for the complementary error
//           function, 2 e^{z^2} int_z^inf e^{-t^2} dt = 1/(z + (1/2)/(z + 1/(z +
//           (3/2)/(z + ...)))), gives F = e^{j pi/4} a / (z + (1/2)/(z + ...)),
//           evaluated bottom-up from a depth chosen by x (40 at x = 4 down to 5
//           at x >= 300, each below 1e-10 relative).
//
// Each term cot((pi +- b)/2n) F(k L a+-(b)) is written through the deviation
// eps = 2 n pi N - b -+ pi from its shadow or reflection boundary: a = 2
// sin^2(eps/2) and the cotangent is -+cot(eps/2n), so that both factors keep
// their relative accuracy as eps -> 0 (their product stays finite: the limit
// 2n sgn(eps) sqrt(pi k L / 2) e^{j pi/4}, used for |eps| < 1e-12).
#pragma once

#include "dev_common.h"

namespace rtc {

struct Cd {
  double x, y;
};
RTC_DEV Cd cd(double x, double y) { return Cd{x, y}; }
RTC_DEV Cd cd_add(Cd a, Cd b) { return Cd{a.x + b.x, a.y + b.y}; }
RTC_DEV Cd cd_mul(Cd a, Cd b) { return Cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
RTC_DEV Cd cd_scale(Cd a, double s) { return Cd{a.x * s, a.y * s}; }
RTC_DEV Cd cd_div(Cd a, Cd b) {
  const double d = b.x * b.x + b.y * b.y;
  return Cd{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
RTC_DEV Cd cd_expj(double t) {
  double s, c;
  sincos(t, &s, &c);
  return Cd{c, s};
}

constexpr double kUtdPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.7724538509055160273;
constexpr double kSqrtHalf = 0.70710678118654752440;

// Depth of the continued fraction for F(x) to 1e-10 relative (measured
// against the series and library Fresnel integrals), x >= 4.
RTC_DEV int cf_depth(double x) {
  return x < 6.0 ? 40 : x < 9.0 ? 28 : x < 14.0 ? 20 : x < 20.0 ? 15 : x < 30.0 ? 12
       : x < 60.0 ? 10 : x < 300.0 ? 7 : 5;
}

// F at four arguments together (the transition function by the methods
// above): the loops of the four evaluations are interleaved, independent
// dependency chains, instead of run one after the other.
RTC_DEV void utd_transition4(const double x[4], Cd F[4]) {
  Cd t[4], s[4];
  bool ser[4];
  int depth = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ser[i] = x[i] > 0.0 && x[i] < 4.0;
    t[i] = cd(sqrt(fmax(x[i], 0.0)), 0.0);
    s[i] = cd(0.0, 0.0);
    if (x[i] >= 4.0) depth = max(depth, cf_depth(x[i]));
  }
  // power series where x < 4 (all four advance until every one converged)
  for (int m = 0; m < 48; ++m) {
    bool more = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!ser[i]) continue;
      s[i] = cd_add(s[i], cd_scale(t[i], 1.0 / (2 * m + 1)));
      t[i] = cd_scale(cd(t[i].y, -t[i].x), x[i] / (m + 1));
      more |= fabs(t[i].x) + fabs(t[i].y) >= 1e-18 * (fabs(s[i].x) + fabs(s[i].y));
    }
    if (!more) break;
  }
  // continued fraction where x >= 4
  Cd z[4], c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double a = sqrt(fmax(x[i], 0.0));
    z[i] = cd(a * kSqrtHalf, a * kSqrtHalf);
    c[i] = x[i] >= 4.0 ? z[i] : cd(1.0, 0.0);
  }
  for (int m = depth; m >= 1; --m) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (x[i] >= 4.0) c[i] = cd_add(z[i], cd_div(cd(0.5 * m, 0.0), c[i]));
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double a = sqrt(fmax(x[i], 0.0));
    if (x[i] <= 0.0) {
      F[i] = cd(0.0, 0.0);
    } else if (ser[i]) {
      const Cd tail = cd(0.5 * kSqrtPi * kSqrtHalf - s[i].x, -0.5 * kSqrtPi * kSqrtHalf - s[i].y);
      F[i] = cd_mul(cd_mul(cd(0.0, 2.0 * a), cd_expj(x[i])), tail);
    } else {
      F[i] = cd_div(z[i], c[i]);
    }
  }
}

// The four terms of D for angles phi (diffraction) and phip (incidence),
// both measured from face 0: t[0], t[1] the incident-field terms (a+ and a-
// of phi - phip), t[2] the face-0 term (a- of phi + phip), t[3] the face-n
// term (a+ of phi + phip).  D = pre (t0 + t1 + R0 t2 + Rn t3).  Each term is
// s_cot * cot(eps / 2n) * F(k L 2 sin^2(eps/2)) with eps the deviation of its
// b from the term's boundary (sign = +1 for a+, -1 for a-).
RTC_DEV void utd_terms(double phi, double phip, double n, double kL, Cd t[4]) {
  const double b[4] = {phi - phip, phi - phip, phi + phip, phi + phip};
  const double sgn[4] = {1.0, -1.0, -1.0, 1.0};
  const double two_n_pi = 2.0 * n * kUtdPi;
  double x[4], cotf[4], eps[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double N = rint((b[i] + sgn[i] * kUtdPi) / two_n_pi);
    eps[i] = two_n_pi * N - b[i] - sgn[i] * kUtdPi;
    double se, ce;
    sincos(eps[i] / (2.0 * n), &se, &ce);
    const double sh = sin(0.5 * eps[i]);
    // cot((pi + b)/2n) = -cot(eps/2n) for a+, cot((pi - b)/2n) = cot(eps/2n) for a-
    cotf[i] = -sgn[i] * ce / se;
    x[i] = kL * 2.0 * sh * sh;
  }
  Cd F[4];
  utd_transition4(x, F);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (fabs(eps[i]) < 1e-12) {
      // the finite limit 2n sgn(eps) sqrt(pi k L / 2) e^{j pi/4} (times -sgn)
      const double lim = (eps[i] > 0.0 ? 1.0 : (eps[i] < 0.0 ? -1.0 : 0.0)) * 2.0 * n *
                         sqrt(kUtdPi * kL * 0.5) * (-sgn[i]);
      t[i] = cd(lim * kSqrtHalf, lim * kSqrtHalf);
    } else {
      t[i] = cd_scale(F[i], cotf[i]);
    }
  }
}

}  // namespace rtc
