// host_math.hpp -- set-up arithmetic done once on the host: the exponential
// integral E_3 and the per-iteration diffusion coefficient of the flat-cell
// kernel used by the Newton operator.
#pragma once
#include <cmath>

namespace iugkp {

// E_n(x) for n >= 1, x >= 0 (x > 0 for n == 1).
//  x <= 1: E_1 from its power series -gamma - ln x - sum_{k>=1} (-x)^k / (k k!),
//          then the upward recurrence E_{m+1} = (e^-x - x E_m) / m.
//  x  > 1: Legendre's continued fraction
//          E_n(x) = e^-x / (x + n - 1 n / (x + n + 2 - 2 (n+1) / (x + n + 4 - ...)))
//          evaluated with the modified Lentz method.
inline double expint_n(int n, double x)
{
  const double kEuler = 0.57721566490153286061;
  if (x == 0.0) return (n > 1) ? 1.0 / (n - 1) : INFINITY;
  if (x > 1.0) {
    const double tiny = 1e-300;
    double b = x + n;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double h = d;
    for (int i = 1; i < 10000; ++i) {
      const double an = -static_cast<double>(i) * (n - 1 + i);
      b += 2.0;
      d = 1.0 / (an * d + b);
      c = b + an / c;
      const double del = c * d;
      h *= del;
      if (std::fabs(del - 1.0) < 1e-17) break;
    }
    return h * std::exp(-x);
  }
  double sum = 0.0, term = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= -x / k;                      // (-x)^k / k!
    const double add = term / k;
    sum += add;
    if (std::fabs(add) < 1e-18 * std::fabs(sum)) break;
  }
  double e = -kEuler - std::log(x) - sum;   // E_1
  const double ex = std::exp(-x);
  for (int m = 1; m < n; ++m) e = (ex - x * e) / m;
  return e;
}

// D_eff(lam, delta) = (lam delta / 2) (1/2 + 2 sum_{j>=1} E_3(j delta / lam)):
// half the second moment of the cell-to-cell displacement of one flight
// between flat cells of width delta (summation by parts of sum m^2 delta^2 P_m).
inline double d_eff(double lam, double delta)
{
  const double a = delta / lam;
  long jmax = static_cast<long>(std::ceil(50.0 / a)) + 2;
  double s = 0.0;
  for (long j = jmax; j >= 1; --j) s += expint_n(3, static_cast<double>(j) * a);
  return (lam * delta / 2.0) * (0.5 + 2.0 * s);
}

}  // namespace iugkp
