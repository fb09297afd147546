// Forward-mode dual numbers for device code, and scalar helpers that work on
// double, float and duals alike.  The adjoint kernels evaluate the local
// Jacobians of the forward maps (one cell's chemistry over a subcycle, one
// face's flux, one cell's limited gradient) by running the same device code
// on Dual<K> with K seeded input directions; every branch is decided on the
// value part, so the derivative is that of the branch path taken.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_math.hpp"

namespace rtk {

template <int K>
struct Dual;

// Whether a scalar type carries derivative parts.
template <typename R>
struct IsDualT {
    static constexpr bool value = false;
};
template <int K>
struct IsDualT<Dual<K>> {
    static constexpr bool value = true;
};

template <int K>
struct Dual {
    double v;
    double d[K];
    __device__ Dual() : v(0.0) {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
    __device__ Dual(double x) : v(x) {  // NOLINT: implicit on purpose
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
};

template <int K> __device__ inline Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <int K> __device__ inline Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <int K> __device__ inline Dual<K> operator-(const Dual<K>& a) {
    Dual<K> r; r.v = -a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
    return r;
}
template <int K> __device__ inline Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <int K> __device__ inline Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
template <int K> __device__ inline Dual<K> operator+(const Dual<K>& a, double b) { Dual<K> r = a; r.v += b; return r; }
template <int K> __device__ inline Dual<K> operator+(double a, const Dual<K>& b) { Dual<K> r = b; r.v += a; return r; }
template <int K> __device__ inline Dual<K> operator-(const Dual<K>& a, double b) { Dual<K> r = a; r.v -= b; return r; }
template <int K> __device__ inline Dual<K> operator-(double a, const Dual<K>& b) { Dual<K> r = -b; r.v += a; return r; }
template <int K> __device__ inline Dual<K> operator*(const Dual<K>& a, double b) {
    Dual<K> r; r.v = a.v * b;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b;
    return r;
}
template <int K> __device__ inline Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K> __device__ inline Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> __device__ inline Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> __device__ inline Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> __device__ inline Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }
template <int K> __device__ inline Dual<K>& operator*=(Dual<K>& a, const Dual<K>& b) { a = a * b; return a; }
template <int K> __device__ inline Dual<K>& operator*=(Dual<K>& a, double b) { a = a * b; return a; }

__device__ inline double val(double x) { return x; }
__device__ inline float val(float x) { return x; }
template <int K> __device__ inline double val(const Dual<K>& a) { return a.v; }

template <int K> __device__ inline Dual<K> chain(const Dual<K>& a, double f, double df) {
    Dual<K> r; r.v = f;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = df * a.d[k];
    return r;
}

__device__ inline double m_sqrt(double x) { return sqrt(x); }
__device__ inline float m_sqrt(float x) { return sqrtf(x); }
template <int K> __device__ inline Dual<K> m_sqrt(const Dual<K>& a) {
    const double s = sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
// exp, log and powers of positive bases through rt_exp / rt_log.
__device__ inline double m_exp(double x) { return rt_exp(x); }
template <int K> __device__ inline Dual<K> m_exp(const Dual<K>& a) {
    const double e = rt_exp(a.v);
    return chain(a, e, e);
}
__device__ inline double m_pow(double x, double p) { return rt_exp(p * rt_log(x)); }
template <int K> __device__ inline Dual<K> m_pow(const Dual<K>& a, double p) {
    const double r = rt_exp(p * rt_log(a.v));
    return chain(a, r, p * r / a.v);
}
__device__ inline double m_log(double x) { return rt_log(x); }
template <int K> __device__ inline Dual<K> m_log(const Dual<K>& a) { return chain(a, rt_log(a.v), 1.0 / a.v); }
__device__ inline double m_log10(double x) { return 0.43429448190325182765 * rt_log(x); }
template <int K> __device__ inline Dual<K> m_log10(const Dual<K>& a) {
    return chain(a, 0.43429448190325182765 * rt_log(a.v), 0.43429448190325182765 / a.v);
}
// c ? a : b, for duals part by part (a select of whole structures would put
// them in scratch memory).
template <typename R> __device__ inline R sel(bool c, const R& a, const R& b) { return c ? a : b; }
template <int K> __device__ inline Dual<K> sel(bool c, const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r;
    r.v = c ? a.v : b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = c ? a.d[k] : b.d[k];
    return r;
}
template <typename R> __device__ inline R m_abs(const R& a) { return sel(val(a) < 0, R(-a), a); }
template <typename R> __device__ inline R m_max(const R& a, const R& b) { return sel(val(a) >= val(b), a, b); }
template <typename R> __device__ inline R m_min(const R& a, const R& b) { return sel(val(a) <= val(b), a, b); }

}  // namespace rtk
