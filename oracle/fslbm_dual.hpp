/*
 * fslbm_dual.hpp -- forward-mode dual number (value and one directional
 * derivative) for the tangent-linear build of the CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY (see fslbm_oracle_tl.cpp). Every operation
 * applies the chain rule to the derivative part; comparisons and integer
 * conversions use the value only, so a branch differentiates the piece of
 * the function it selects.
 */
#pragma once

#include <math.h>

struct Dual {
    double v, d;
    Dual() = default;
    Dual(double x) : v(x), d(0.0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
    explicit operator long() const { return (long)v; }
    Dual &operator+=(const Dual &b) { v += b.v; d += b.d; return *this; }
    Dual &operator-=(const Dual &b) { v -= b.v; d -= b.d; return *this; }
    Dual &operator*=(const Dual &b) { d = d * b.v + v * b.d; v *= b.v; return *this; }
    Dual &operator/=(const Dual &b) { d = (d * b.v - v * b.d) / (b.v * b.v); v /= b.v; return *this; }
};

inline Dual operator+(const Dual &a) { return a; }
inline Dual operator-(const Dual &a) { return Dual(-a.v, -a.d); }
inline Dual operator+(const Dual &a, const Dual &b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual &a, const Dual &b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(const Dual &a, const Dual &b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual &a, const Dual &b)
{
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline bool operator<(const Dual &a, const Dual &b) { return a.v < b.v; }
inline bool operator>(const Dual &a, const Dual &b) { return a.v > b.v; }
inline bool operator<=(const Dual &a, const Dual &b) { return a.v <= b.v; }
inline bool operator>=(const Dual &a, const Dual &b) { return a.v >= b.v; }
inline bool operator==(const Dual &a, const Dual &b) { return a.v == b.v; }
inline bool operator!=(const Dual &a, const Dual &b) { return a.v != b.v; }

inline Dual sqrt(const Dual &a)
{
    const double s = sqrt(a.v);
    return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
inline Dual fabs(const Dual &a) { return a.v < 0.0 ? -a : a; }
inline Dual sin(const Dual &a) { return Dual(sin(a.v), cos(a.v) * a.d); }
inline Dual cos(const Dual &a) { return Dual(cos(a.v), -sin(a.v) * a.d); }
inline Dual atan2(const Dual &y, const Dual &x)
{
    const double r2 = x.v * x.v + y.v * y.v;
    return Dual(atan2(y.v, x.v), r2 > 0.0 ? (x.v * y.d - y.v * x.d) / r2 : 0.0);
}
inline Dual fmin(const Dual &a, const Dual &b) { return b.v < a.v ? b : a; }
inline Dual fmax(const Dual &a, const Dual &b) { return b.v > a.v ? b : a; }
inline bool isfinite(const Dual &a) { return isfinite(a.v) && isfinite(a.d); }
