// Forward-mode dual numbers for the tangent kernels of the adjoint: a value
// and N directional derivatives, FP64.  Value parts follow exactly the same
// operations as plain double code.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace ppm {

// the dual overloads below must not hide the double versions
using ::sqrt; using ::sin; using ::cos; using ::exp; using ::log; using ::log10;
using ::acos; using ::asin; using ::atan; using ::asinh; using ::fabs; using ::fmax; using ::fmin;

template <int N>
struct Dual {
    double v;
    double d[N];
    __device__ Dual() : v(0.0)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __device__ Dual(double x) : v(x)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    // x with unit tangent along direction k
    __device__ static Dual seed(double x, int k, double dk = 1.0)
    {
        Dual r(x);
        r.d[k] = dk;
        return r;
    }
};

// chain rule helper: f(a) with f'(a) = g
template <int N>
__device__ inline Dual<N> chain(const Dual<N> &a, double fv, double g)
{
    Dual<N> r;
    r.v = fv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r;
}

template <int N>
__device__ inline Dual<N> operator+(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N> &a)
{
    Dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__device__ inline Dual<N> operator*(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
__device__ inline Dual<N> operator/(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
template <int N>
__device__ inline Dual<N> operator+(const Dual<N> &a, double b)
{
    Dual<N> r = a;
    r.v = a.v + b;
    return r;
}
template <int N>
__device__ inline Dual<N> operator+(double a, const Dual<N> &b) { return b + a; }
template <int N>
__device__ inline Dual<N> operator-(const Dual<N> &a, double b)
{
    Dual<N> r = a;
    r.v = a.v - b;
    return r;
}
template <int N>
__device__ inline Dual<N> operator-(double a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -b.d[i];
    return r;
}
template <int N>
__device__ inline Dual<N> operator*(const Dual<N> &a, double b)
{
    Dual<N> r;
    r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N>
__device__ inline Dual<N> operator*(double a, const Dual<N> &b) { return b * a; }
template <int N>
__device__ inline Dual<N> operator/(const Dual<N> &a, double b)
{
    Dual<N> r;
    r.v = a.v / b;
    const double ib = 1.0 / b;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * ib;
    return r;
}
template <int N>
__device__ inline Dual<N> operator/(double a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a / b.v;
    const double g = -r.v / b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = g * b.d[i];
    return r;
}

template <int N> __device__ inline Dual<N> sqrt(const Dual<N> &a)
{
    double s = ::sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
template <int N> __device__ inline Dual<N> sin(const Dual<N> &a) { return chain(a, ::sin(a.v), ::cos(a.v)); }
template <int N> __device__ inline Dual<N> cos(const Dual<N> &a) { return chain(a, ::cos(a.v), -::sin(a.v)); }
template <int N> __device__ inline Dual<N> exp(const Dual<N> &a)
{
    double e = ::exp(a.v);
    return chain(a, e, e);
}
template <int N> __device__ inline Dual<N> log(const Dual<N> &a) { return chain(a, ::log(a.v), 1.0 / a.v); }
template <int N> __device__ inline Dual<N> log10(const Dual<N> &a)
{
    return chain(a, ::log10(a.v), 1.0 / (a.v * 2.302585092994045684));
}
template <int N> __device__ inline Dual<N> acos(const Dual<N> &a)
{
    return chain(a, ::acos(a.v), -1.0 / ::sqrt(1.0 - a.v * a.v));
}
template <int N> __device__ inline Dual<N> asin(const Dual<N> &a)
{
    return chain(a, ::asin(a.v), 1.0 / ::sqrt(1.0 - a.v * a.v));
}
template <int N> __device__ inline Dual<N> atan(const Dual<N> &a)
{
    return chain(a, ::atan(a.v), 1.0 / (1.0 + a.v * a.v));
}
template <int N> __device__ inline Dual<N> asinh(const Dual<N> &a)
{
    return chain(a, ::asinh(a.v), 1.0 / ::sqrt(1.0 + a.v * a.v));
}
template <int N> __device__ inline Dual<N> fabs(const Dual<N> &a) { return a.v < 0.0 ? -a : a; }
template <int N> __device__ inline Dual<N> fmax(const Dual<N> &a, const Dual<N> &b) { return a.v >= b.v ? a : b; }
template <int N> __device__ inline Dual<N> fmin(const Dual<N> &a, const Dual<N> &b) { return a.v <= b.v ? a : b; }

template <int N> __device__ inline Dual<N> &operator+=(Dual<N> &a, const Dual<N> &b) { return a = a + b; }
template <int N> __device__ inline Dual<N> &operator-=(Dual<N> &a, const Dual<N> &b) { return a = a - b; }
template <int N> __device__ inline Dual<N> &operator*=(Dual<N> &a, const Dual<N> &b) { return a = a * b; }

// 1/x and 1/sqrt(x) for positive finite x: the hardware estimate refined by
// two Newton steps (within about an ulp of the correctly rounded result, at
// half the instructions of an IEEE division or square root)
__device__ inline double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ inline double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}
template <int N> __device__ inline Dual<N> rcp_nr(const Dual<N> &a)
{
    const double r = rcp_nr(a.v);
    return chain(a, r, -r * r);
}
template <int N> __device__ inline Dual<N> rsqrt_nr(const Dual<N> &a)
{
    const double y = rsqrt_nr(a.v);
    return chain(a, y, -0.5 * y * y * y);
}

__device__ inline double value(double x) { return x; }
template <int N> __device__ inline double value(const Dual<N> &x) { return x.v; }

}  // namespace ppm
