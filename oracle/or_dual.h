/*
 * Forward-mode dual number for the tangent build of the oracle (C++ only).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/.  A value x + e x' with
 * e^2 = 0: every operation applies the chain rule to the second part, so a
 * computation seeded with input tangents returns, beside each result, its
 * directional derivative (the Jacobian-vector product).  The first part of
 * every operation is the plain double operation, evaluated in the same order
 * as in the double build, so the values of both builds agree bit for bit.
 * Comparisons, branches and integer conversions look at the value only: the
 * derivative is that of the branch taken.
 */
#ifndef OR_DUAL_H
#define OR_DUAL_H
#ifndef __cplusplus
#error "or_dual.h is the C++ tangent build"
#endif
#include <cmath>

struct real {
  double v, d;
  real() = default;
  constexpr real(double x) : v(x), d(0.0) {}
  constexpr real(double x, double t) : v(x), d(t) {}
};

inline real operator+(real a, real b) { return real(a.v + b.v, a.d + b.d); }
inline real operator-(real a, real b) { return real(a.v - b.v, a.d - b.d); }
inline real operator-(real a) { return real(-a.v, -a.d); }
inline real operator+(real a) { return a; }
inline real operator*(real a, real b) { return real(a.v * b.v, a.d * b.v + a.v * b.d); }
inline real operator/(real a, real b) {
  double q = a.v / b.v;
  return real(q, (a.d - q * b.d) / b.v);
}
inline real& operator+=(real& a, real b) { a = a + b; return a; }
inline real& operator-=(real& a, real b) { a = a - b; return a; }
inline real& operator*=(real& a, real b) { a = a * b; return a; }
inline real& operator/=(real& a, real b) { a = a / b; return a; }

inline bool operator<(real a, real b) { return a.v < b.v; }
inline bool operator>(real a, real b) { return a.v > b.v; }
inline bool operator<=(real a, real b) { return a.v <= b.v; }
inline bool operator>=(real a, real b) { return a.v >= b.v; }
inline bool operator==(real a, real b) { return a.v == b.v; }
inline bool operator!=(real a, real b) { return a.v != b.v; }

inline real exp(real a) { double e = std::exp(a.v); return real(e, e * a.d); }
inline real sqrt(real a) { double s = std::sqrt(a.v); return real(s, a.d / (2.0 * s)); }
inline real fabs(real a) { return (a.v < 0.0) ? -a : a; }
inline real cos(real a) { return real(std::cos(a.v), -std::sin(a.v) * a.d); }
inline real sin(real a) { return real(std::sin(a.v), std::cos(a.v) * a.d); }
/* x^y: d = y x^(y-1) x' + x^y ln(x) y' (the second term only when y' != 0) */
inline real pow(real a, real b) {
  double p = std::pow(a.v, b.v);
  double t = b.v * std::pow(a.v, b.v - 1.0) * a.d;
  if (b.d != 0.0) t += p * std::log(a.v) * b.d;
  return real(p, t);
}
inline bool isinf(real a) { return std::isinf(a.v); }
inline bool isnan(real a) { return std::isnan(a.v); }

#endif
