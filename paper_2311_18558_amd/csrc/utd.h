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
//           evaluated bottom-up from a fixed depth of 40 (below 1e-10 at x = 4).
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

RTC_DEV Cd utd_transition(double x) {
  if (x <= 0.0) return cd(0.0, 0.0);
  const double a = sqrt(x);
  if (x < 4.0) {
    // sum_m (-j)^m a^{2m+1} / (m! (2m+1))
    Cd t = cd(a, 0.0), s = cd(0.0, 0.0);
    for (int m = 0; m < 48; ++m) {
      s = cd_add(s, cd_scale(t, 1.0 / (2 * m + 1)));
      // t *= -j x / (m + 1)
      t = cd_scale(cd(t.y, -t.x), x / (m + 1));
      if (fabs(t.x) + fabs(t.y) < 1e-18 * (fabs(s.x) + fabs(s.y))) break;
    }
    // sqrt(pi)/2 e^{-j pi/4} - s, times 2j a e^{jx}
    const Cd tail = cd(0.5 * kSqrtPi * kSqrtHalf - s.x, -0.5 * kSqrtPi * kSqrtHalf - s.y);
    return cd_mul(cd_mul(cd(0.0, 2.0 * a), cd_expj(x)), tail);
  }
  const Cd z = cd(a * kSqrtHalf, a * kSqrtHalf);
  Cd t = z;
  for (int m = 40; m >= 1; --m) t = cd_add(z, cd_div(cd(0.5 * m, 0.0), t));
  return cd_div(cd(a * kSqrtHalf, a * kSqrtHalf), t);
}

// s_cot * cot(eps / 2n) * F(k L 2 sin^2(eps/2)) with eps the deviation of b
// from the boundary of the term; sign = +1 for a+, -1 for a-.
RTC_DEV Cd utd_term(double b, double n, double kL, double sign) {
  const double two_n_pi = 2.0 * n * kUtdPi;
  const double N = rint((b + sign * kUtdPi) / two_n_pi);
  const double eps = two_n_pi * N - b - sign * kUtdPi;
  // cot((pi + b)/2n) = -cot(eps/2n) for a+, cot((pi - b)/2n) = cot(eps/2n) for a-
  const double s_cot = -sign;
  if (fabs(eps) < 1e-12) {
    const double lim = (eps > 0.0 ? 1.0 : (eps < 0.0 ? -1.0 : 0.0)) * 2.0 * n *
                       sqrt(kUtdPi * kL * 0.5) * s_cot;
    return cd(lim * kSqrtHalf, lim * kSqrtHalf);  // times e^{j pi/4}
  }
  double se, ce;
  sincos(eps / (2.0 * n), &se, &ce);
  const double sh = sin(0.5 * eps);
  const Cd F = utd_transition(kL * 2.0 * sh * sh);
  return cd_scale(F, s_cot * ce / se);
}

// The four terms of D for angles phi (diffraction) and phip (incidence),
// both measured from face 0: t[0], t[1] the incident-field terms (a+ and a-
// of phi - phip), t[2] the face-0 term (a- of phi + phip), t[3] the face-n
// term (a+ of phi + phip).  D = pre (t0 + t1 + R0 t2 + Rn t3).
RTC_DEV void utd_terms(double phi, double phip, double n, double kL, Cd t[4]) {
  t[0] = utd_term(phi - phip, n, kL, 1.0);
  t[1] = utd_term(phi - phip, n, kL, -1.0);
  t[2] = utd_term(phi + phip, n, kL, -1.0);
  t[3] = utd_term(phi + phip, n, kL, 1.0);
}

}  // namespace rtc
