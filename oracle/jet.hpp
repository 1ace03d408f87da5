// Second-order forward-mode jets for the FP64 oracle (test infrastructure).
//
// A Jet<N> carries a value, its gradient and its Hessian with respect to N
// independent variables.  The arithmetic below is the product and chain rule
// written out; it lets the oracle take exact first and second derivatives of
// the rendered colour with respect to a kernel's attributes, which is what the
// local Newton system of the paper's Sec. 4.2 (eq. local_hessian_gradient)
// needs, without hand-deriving every intermediate derivative.
#pragma once
#include <cmath>

template <int N>
struct Jet {
    double v;
    double g[N];
    double h[N][N];
    Jet() : v(0.0) { clear(); }
    Jet(double c) : v(c) { clear(); }  // NOLINT: implicit constant
    void clear() {
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            for (int j = 0; j < N; ++j) h[i][j] = 0.0;
        }
    }
    static Jet var(double x, int i) {
        Jet r(x);
        r.g[i] = 1.0;
        return r;
    }
};

inline double val(double x) { return x; }
template <int N> inline double val(const Jet<N>& x) { return x.v; }

template <int N> Jet<N> operator+(const Jet<N>& a, const Jet<N>& b) {
    Jet<N> r;
    r.v = a.v + b.v;
    for (int i = 0; i < N; ++i) {
        r.g[i] = a.g[i] + b.g[i];
        for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
    }
    return r;
}
template <int N> Jet<N> operator-(const Jet<N>& a, const Jet<N>& b) {
    Jet<N> r;
    r.v = a.v - b.v;
    for (int i = 0; i < N; ++i) {
        r.g[i] = a.g[i] - b.g[i];
        for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] - b.h[i][j];
    }
    return r;
}
template <int N> Jet<N> operator-(const Jet<N>& a) {
    Jet<N> r;
    r.v = -a.v;
    for (int i = 0; i < N; ++i) {
        r.g[i] = -a.g[i];
        for (int j = 0; j < N; ++j) r.h[i][j] = -a.h[i][j];
    }
    return r;
}
template <int N> Jet<N> operator*(const Jet<N>& a, const Jet<N>& b) {
    // (ab)'' = a''b + a b'' + a' b'^T + b' a'^T
    Jet<N> r;
    r.v = a.v * b.v;
    for (int i = 0; i < N; ++i) {
        r.g[i] = a.g[i] * b.v + a.v * b.g[i];
        for (int j = 0; j < N; ++j)
            r.h[i][j] = a.h[i][j] * b.v + a.v * b.h[i][j] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
    }
    return r;
}
template <int N> Jet<N> operator*(double c, const Jet<N>& a) {
    Jet<N> r;
    r.v = c * a.v;
    for (int i = 0; i < N; ++i) {
        r.g[i] = c * a.g[i];
        for (int j = 0; j < N; ++j) r.h[i][j] = c * a.h[i][j];
    }
    return r;
}
template <int N> Jet<N> operator*(const Jet<N>& a, double c) { return c * a; }
template <int N> Jet<N> operator+(const Jet<N>& a, double c) { Jet<N> r = a; r.v += c; return r; }
template <int N> Jet<N> operator+(double c, const Jet<N>& a) { return a + c; }
template <int N> Jet<N> operator-(const Jet<N>& a, double c) { Jet<N> r = a; r.v -= c; return r; }
template <int N> Jet<N> operator-(double c, const Jet<N>& a) { return (-a) + c; }

// Composition with a scalar function f: value f, first derivative d1, second d2.
template <int N> Jet<N> compose(const Jet<N>& a, double f, double d1, double d2) {
    Jet<N> r;
    r.v = f;
    for (int i = 0; i < N; ++i) {
        r.g[i] = d1 * a.g[i];
        for (int j = 0; j < N; ++j) r.h[i][j] = d1 * a.h[i][j] + d2 * a.g[i] * a.g[j];
    }
    return r;
}
template <int N> Jet<N> recip(const Jet<N>& a) {
    const double x = a.v;
    return compose(a, 1.0 / x, -1.0 / (x * x), 2.0 / (x * x * x));
}
template <int N> Jet<N> operator/(const Jet<N>& a, const Jet<N>& b) { return a * recip(b); }
template <int N> Jet<N> operator/(const Jet<N>& a, double c) { return a * (1.0 / c); }
template <int N> Jet<N> operator/(double c, const Jet<N>& b) { return c * recip(b); }
template <int N> Jet<N> exp(const Jet<N>& a) {
    const double e = std::exp(a.v);
    return compose(a, e, e, e);
}
template <int N> Jet<N> sqrt(const Jet<N>& a) {
    const double s = std::sqrt(a.v);
    return compose(a, s, 0.5 / s, -0.25 / (s * a.v));
}

inline double recip(double x) { return 1.0 / x; }
