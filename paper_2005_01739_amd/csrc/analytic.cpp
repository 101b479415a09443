// Analytic random-catalogue terms, host double precision.
//
// W~^a(R0) = 4 pi int_0^R0 r^2 jbar^a_0(r) W(r/R0) dr   (Sec. 3, eq. wka-def)
// is the binned spherical transform of the window; it supplies the RR term of
// the power spectrum (Sec. 3) and the RRR and DDR^I terms of the bispectrum
// (Sec. 4).  The integrand is smooth on each piece of W, [0, R0/2],
// [R0/2, 3R0/4], [3R0/4, R0]; each piece is integrated by composite
// Clenshaw-Curtis rules in extended precision, doubling the panel count until
// two successive estimates agree to 1e-18 of the integrand's absolute mass.
#include <math.h>

#include <vector>

#include "common.h"

namespace hipster {

namespace {

// Host extended precision (x86 80-bit long double, 64-bit significand): W~ is
// a small difference of a large oscillating integrand, and double-precision
// rounding of sin u - u cos u at u ~ k R0 ~ 10^2 adds up coherently.
typedef long double xd;
constexpr xd kPiX = 3.14159265358979323846264338327950288L;
constexpr int kCC = 32;  // Clenshaw-Curtis points - 1 per panel

struct CCRule {
  xd x[kCC + 1], w[kCC + 1];
  CCRule() {
    const int n = kCC;
    for (int k = 0; k <= n; ++k) {
      x[k] = cosl(kPiX * k / n);
      xd s = 0.0L;
      for (int j = 1; j <= n / 2; ++j) {
        const xd b = (j == n / 2) ? 1.0L : 2.0L;
        s += b / (4.0L * j * j - 1.0L) * cosl(2.0L * j * k * kPiX / n);
      }
      const xd c = (k == 0 || k == n) ? 1.0L : 2.0L;
      w[k] = c / n * (1.0L - s);
    }
  }
};

const CCRule &rule() {
  static CCRule r;
  return r;
}

// G_0(u) = (sin u - u cos u) / u^3, with its Taylor series for small u:
// sum_s (-1)^s u^(2s) / ((2s+3) 2^s s! (2s+1)!!).
xd G0(xd u) {
  if (u < 0.5L) {
    const xd v = u * u;
    xd t = 1.0L, sum = 0.0L;  // t = (-v/2)^s / (s! (2s+1)!!)
    for (int s = 0; s < 24; ++s) {
      sum += t / (2.0L * s + 3.0L);
      t *= -v / (2.0L * (s + 1.0L) * (2.0L * s + 3.0L));
    }
    return sum;
  }
  return (sinl(u) - u * cosl(u)) / (u * u * u);
}

xd window_x(xd x) {
  if (x < 0.5L) return 1.0L;
  if (x < 0.75L) {
    const xd t = 2.0L * x - 1.0L;
    return 1.0L - 8.0L * t * t * t + 8.0L * t * t * t * t;
  }
  if (x < 1.0L) {
    const xd t = x - 1.0L;
    return -64.0L * t * t * t - 128.0L * t * t * t * t;
  }
  return 0.0L;
}

xd integrand(xd r, xd r0, xd k1, xd k2) {
  const xd a3 = k1 * k1 * k1, b3 = k2 * k2 * k2;
  const xd jb = 3.0L * (b3 * G0(k2 * r) - a3 * G0(k1 * r)) / (b3 - a3);
  return r * r * jb * window_x(r / r0);
}

void composite(xd a, xd b, int panels, xd r0, xd k1, xd k2, xd &val, xd &mass) {
  const CCRule &R = rule();
  const xd h = (b - a) / panels;
  val = 0.0L;
  mass = 0.0L;
  for (int p = 0; p < panels; ++p) {
    const xd lo = a + p * h, half = 0.5L * h, mid = lo + half;
    for (int k = 0; k <= kCC; ++k) {
      const xd f = integrand(mid + half * R.x[k], r0, k1, k2);
      val += half * R.w[k] * f;
      mass += half * R.w[k] * fabsl(f);
    }
  }
}

}  // namespace

double wtilde_bin(double r0_, double k1_, double k2_) {
  const xd r0 = r0_, k1 = k1_, k2 = k2_;
  const xd cuts[4] = {0.0L, 0.5L * r0, 0.75L * r0, r0};
  xd total = 0.0L;
  for (int piece = 0; piece < 3; ++piece) {
    const xd a = cuts[piece], b = cuts[piece + 1];
    // start near two panels per radian of the fastest oscillation
    int panels = int(ceill((b - a) * k2 / 2.0L)) + 1;
    xd prev, mass;
    composite(a, b, panels, r0, k1, k2, prev, mass);
    for (int it = 0; it < 8; ++it) {
      panels *= 2;
      xd cur, m2;
      composite(a, b, panels, r0, k1, k2, cur, m2);
      const bool done = fabsl(cur - prev) <= 1e-18L * m2;
      prev = cur;
      if (done) break;
    }
    total += prev;
  }
  return double(4.0L * kPiX * total);
}

}  // namespace hipster
