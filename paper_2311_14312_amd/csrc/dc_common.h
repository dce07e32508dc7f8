// Shared definitions of the HIP library: error plumbing, device helpers for
// complex arithmetic and the closed-form chord integrals.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dcfmm.h"

namespace dc {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DC_HIP(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess)                                               \
            throw ::dc::Error(e_ == hipErrorOutOfMemory ? DC_ERR_OOM        \
                                                        : DC_ERR_HIP,       \
                              std::string(#expr) + ": " +                   \
                                  hipGetErrorString(e_));                   \
    } while (0)

#define DC_REQUIRE(cond, msg)                                               \
    do {                                                                    \
        if (!(cond)) throw ::dc::Error(DC_ERR_INVALID, msg);                \
    } while (0)

// Thread-local message returned by dc_last_error().
void set_last_error(const std::string& msg);

// Run f and map exceptions to the ABI's error codes (no exception crosses
// the C ABI).
template <typename F>
int guarded(F&& f) {
    try {
        f();
        return DC_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return DC_ERR_OOM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return DC_ERR_INVALID;
    }
}

// Owning device buffer (hipMalloc / hipFree).
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        if (count == n && p) return;
        release();
        if (count == 0) return;
        DC_HIP(hipMalloc(&p, count * sizeof(T)));
        n = count;
    }
    void upload(const std::vector<T>& v) {
        alloc(v.size());
        if (!v.empty())
            DC_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
};

// Owning pinned host buffer (hipHostMalloc / hipHostFree): copies from the
// device into it need no staging through a bounce buffer.
template <typename T>
struct PinnedHost {
    T* p = nullptr;
    explicit PinnedHost(size_t count) {
        DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), count * sizeof(T),
                             hipHostMallocDefault));
    }
    PinnedHost(const PinnedHost&) = delete;
    PinnedHost& operator=(const PinnedHost&) = delete;
    ~PinnedHost() {
        if (p) (void)hipHostFree(p);
    }
};

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ---------------------------------------------------------------- complex
template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cpx<T> cadd(cpx<T> a, cpx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ inline cpx<T> csub(cpx<T> a, cpx<T> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ inline cpx<T> cscale(cpx<T> a, T s) {
    return {a.re * s, a.im * s};
}
template <typename T>
__device__ inline cpx<T> cdiv(cpx<T> a, cpx<T> b) {
    // Smith's algorithm keeps the quotient finite for large |b| components.
    if (fabs(b.re) >= fabs(b.im)) {
        T r = b.im / b.re, den = b.re + b.im * r;
        return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    } else {
        T r = b.re / b.im, den = b.re * r + b.im;
        return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
    }
}
// 1/b = conj(b)/|b|^2 with one real division (the operands here are box-
// relative coordinates of moderate magnitude, so no scaling is needed).
template <typename T>
__device__ inline cpx<T> cinv(cpx<T> b) {
    const T r = T(1) / (b.re * b.re + b.im * b.im);
    return {b.re * r, -b.im * r};
}
// Principal logarithm.
template <typename T>
__device__ inline cpx<T> clog(cpx<T> z) {
    return {T(0.5) * log(z.re * z.re + z.im * z.im), atan2(z.im, z.re)};
}
// z^k by repeated squaring (k >= 0).
template <typename T>
__device__ inline cpx<T> cpow(cpx<T> z, int k) {
    cpx<T> r = {T(1), T(0)};
    while (k) {
        if (k & 1) r = cmul(r, z);
        z = cmul(z, z);
        k >>= 1;
    }
    return r;
}

// ---------------------------------------------------------------- chords
// Integral over a straight chord of ln|p - x| dS and the signed angle theta
// the chord subtends at x.  Chord coordinates (App. D, re-derived):
//   d = p1 - x, t = unit tangent, n = left normal (-t.y, t.x),
//   xi1 = d.t, xi2 = xi1 + |a|, h = d.n, r_i^2 = xi_i^2 + h^2,
//   int ln|p-x| dS = xi2 ln r2 - xi1 ln r1 - |a| + h theta,
//   theta = atan2(h |a|, h^2 + xi1 xi2).
// The logarithmic difference is evaluated from the endpoint farther from x:
// xi2 ln r2 - xi1 ln r1 = |a| ln r1 + xi2 ln(r2/r1), with
// r2^2/r1^2 = 1 + |a|(xi1+xi2)/r1^2 (and the mirror form when r2 > r1), so
// the log1p argument stays in [-1, 0] and far chords lose no digits.
// theta_f is theta with the principal value 0 for a target exactly on the
// open chord (h == 0, xi1 < 0 < xi2).
template <typename T>
__device__ inline void chord_log_theta(T dx, T dy, T tx, T ty, T la,
                                       T& int_log, T& theta_f) {
    const T xi1 = dx * tx + dy * ty;
    const T h = dy * tx - dx * ty;
    const T xi2 = xi1 + la;
    const T r1sq = xi1 * xi1 + h * h;
    const T r2sq = xi2 * xi2 + h * h;
    const T theta = atan2(h * la, h * h + xi1 * xi2);
    const T s = la * (xi1 + xi2);  // r2^2 - r1^2
    T lg_big, x_other, arg;
    if (r1sq >= r2sq) {
        lg_big = T(0.5) * log(r1sq);
        x_other = xi2;
        arg = s / r1sq;
    } else {
        lg_big = T(0.5) * log(r2sq);
        x_other = -xi1;
        arg = -s / r2sq;
    }
    const T l1p = log1p(arg);
    const T tail = (x_other == T(0)) ? T(0) : x_other * T(0.5) * l1p;
    int_log = la * lg_big + tail - la + h * theta;
    theta_f = (h == T(0) && xi1 < T(0) && xi2 > T(0)) ? T(0) : theta;
}

// Singular single layer of a collocation node on its own segment
// (App. D.3 with arc lengths, App. A): 2 pi * Ghat = l - e1 ln e1 - e2 ln e2.
__host__ __device__ inline double self_segment_2pi_G(double ell, double tstar) {
    const double e1 = tstar * ell, e2 = (1.0 - tstar) * ell;
    const double l1 = e1 > 0 ? e1 * log(e1) : 0.0;
    const double l2 = e2 > 0 ? e2 * log(e2) : 0.0;
    return ell - l1 - l2;
}

// Pixel centre coordinates; contraction is disabled so that host and device
// compute bit-identical values (cell assignment of pixels depends on them).
__host__ __device__ inline double pixel_x(double cx, double w, int W, int k) {
#pragma clang fp contract(off)
    return (cx - 0.5 * w) + ((double)k + 0.5) * (w / (double)W);
}
__host__ __device__ inline double pixel_y(double cy, double h, int H, int r) {
#pragma clang fp contract(off)
    return (cy + 0.5 * h) - ((double)r + 0.5) * (h / (double)H);
}
__host__ __device__ inline long long cell_coord(double v, double origin, double side_l) {
#pragma clang fp contract(off)
    return (long long)floor((v - origin) / side_l);
}

}  // namespace dc
