// Device helpers shared by the forward and the adjoint kernels: star
// geometry, the deflection quadrature, Hermite bases, table brackets, cell
// azimuths and the observed-phase lookup.  Templated helpers take double or
// a dual number (forward-mode tangents).
// Section and equation numbers refer to arXiv:2510.07764.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "ppm_internal.h"
#include "ppm_dual.h"
#include "../../include/ppm.h"

namespace ppm {

// g(theta)/g0 of Eqs. (10), (11)
template <class T>
__device__ inline T gravity_ratio_t(int mode, const T &x, const T &Obar, const T &th)
{
    if (mode != PPM_MODE_OS) return T(1.0);
    T O2 = Obar * Obar, O4 = O2 * O2, O6 = O4 * O2;
    T sn = sin(th), c = cos(th);
    T s2 = sn * sn, c2 = c * c;
    T e4 = O4 * (13.47 * x - 27.13 * x * x);
    return 1.0 + s2 * (O2 * (-0.791 + 0.776 * x) + O4 * (-1.315 * x + 2.431 * x * x) + O6 * (-1.172 * x))
         + c2 * (O2 * (1.138 - 1.431 * x) + O4 * (0.653 * x - 2.864 * x * x) + O6 * (0.975 * x) - e4)
         + fabs(c) * e4;
}

__device__ inline double gravity_ratio(const StarRec &st, int mode, double th)
{
    return gravity_ratio_t<double>(mode, st.x, st.Obar, th);
}

// azimuthal half-width of a ring at colatitude th inside a cap (tc, z)
template <class T>
__device__ inline T arc_halfwidth(const T &th, const T &tc, const T &z)
{
    T den = sin(th) * sin(tc);
    T num = cos(z) - cos(th) * cos(tc);
    if (value(den) <= 0.0) return T(value(num) <= 0.0 ? kPi : 0.0);
    T a = num / den;
    if (value(a) <= -1.0) return T(kPi);
    if (value(a) >= 1.0) return T(0.0);
    return acos(a);
}

__device__ inline double cdt_oblate(double Re, double Rs, double R)
{
    return Re - R + Rs * log((Re - Rs) / (R - Rs));   // Eq. (16)
}


template <class X, class V>
__device__ inline auto q_s2(const X &x, const V &v) -> decltype(x * v)
{
    auto t = 1.0 - x * x;
    return 2.0 - x * x - v * t * t / (1.0 - v);
}

// Gauss-Legendre rules on [0, 1] held back to back: 20, 24, 32, 48 and 64
// nodes (kGLNodes in all), at bx / bw (the plan's copy, or an LDS copy).
constexpr int kGLNodes = 188;
__device__ inline void gl_rule(const double *bx, const double *bw, int n, const double *&x, const double *&w)
{
    int off = n == 20 ? 0 : (n == 24 ? 20 : (n == 32 ? 44 : (n == 48 ? 76 : 124)));
    x = bx + off;
    w = bw + off;
}

// psi, dpsi/dalpha and c dt_p/R for an outgoing ray, 0 <= alpha <= pi/2.
// The rule order follows cos(alpha): the sinh map leaves an integrand
// analytic in a strip whose width shrinks only logarithmically as
// cos(alpha) -> 0; 20/24/32/48/64 nodes for cos(alpha) >= 0.5/0.2/0.05/1e-3
// and below keep the relative error of all three integrals below 1e-12 for
// u in [0.15, 0.64] (against a 128-node rule).
// With q0, qs the quadrature runs over the nodes q0, q0 + qs, ... only and the
// terms that are not quadrature sums come from q0 = 0 only, so that summing
// the results of q0 = 0 .. qs-1 gives the full values (lanes of one ray).
template <class U>
__device__ void bend_out(const double *bx, const double *bw, const U &u, double alpha, U &psi, U &dpsi, U &tp,
                         int q0 = 0, int qs = 1)
{
    const U sq = sqrt(1.0 - u);
    if (alpha <= 0.0) { psi = U(0.0); dpsi = q0 == 0 ? 1.0 / sq : U(0.0); tp = U(0.0); return; }
    double c = cos(alpha), s = sin(alpha);
    const U qa = 2.0 - u / (1.0 - u);
    const double *gx, *gw;
    if (c < 1e-9) {
        // tangent ray: x/sqrt(x^2 s^2 q) = 1/(s sqrt q), regular on [0, 1]
        gl_rule(bx, bw, 32, gx, gw);
        U I1 = U(0.0), IT = U(0.0);
        for (int q = q0; q < 32; q += qs) {
            double x = gx[q], w = gw[q];
            U rq = sqrt(q_s2(x, u));
            I1 += w / rq;
            IT += w / (rq * (1.0 + x * s * rq));
        }
        psi = 2.0 / sq * I1;
        dpsi = q0 == 0 ? 2.0 / (sq * qa) : U(0.0);
        tp = 2.0 * s / (1.0 - u) * IT;
        return;
    }
    const int n = c >= 0.5 ? 20 : (c >= 0.2 ? 24 : (c >= 0.05 ? 32 : (c >= 1e-3 ? 48 : 64)));
    gl_rule(bx, bw, n, gx, gw);
    U A = c / (s * sqrt(qa));
    U L = asinh(1.0 / A);
    const U w = u / (1.0 - u);        // q(x) = 2 - x^2 - w (1 - x^2)^2
    const U hA = 0.5 * A, hAL = 0.5 * A * L;
    const double s2 = s * s, c2 = c * c;
    U I1 = U(0.0), I3 = U(0.0), IT = U(0.0);
    // the rule is symmetric about 1/2 (n even): node q and its mirror 1 - x_q
    // share one exponential, exp(L (1 - x_q)) = exp(L) / exp(L x_q)
    const U EL = exp(L), iEL = rcp_nr(EL);
    auto point = [&](const U &ex, const U &iex, double wq) {
        U x = hA * (ex - iex);
        U dx = hAL * (ex + iex) * wq;
        U x2 = x * x, t = 1.0 - x2;
        U D = c2 + x2 * s2 * (2.0 - x2 - w * t * t);
        U ir = rsqrt_nr(D);
        U r = D * ir;
        U xr = x * ir * dx;
        I1 += xr;
        I3 += xr * ir * ir;
        IT += xr * rcp_nr(1.0 + r);
    };
    for (int q = q0; q < n / 2; q += qs) {
        const U ex = exp(L * gx[q]);
        const U iex = rcp_nr(ex);
        point(ex, iex, gw[q]);
        point(EL * iex, ex * iEL, gw[n - 1 - q]);
    }
    psi = 2.0 * s / sq * I1;
    dpsi = 2.0 * c / sq * I3;
    tp = 2.0 * s * s / (1.0 - u) * IT;
}

// psi(v, pi/2), c dt_p/R (v, pi/2) and their v-derivatives (periastron leg)
template <class U>
__device__ void grazing(const double *bx, const double *bw, const U &v, U &ph, U &dph, U &th, U &dth, int q0 = 0,
                        int qs = 1)
{
    U J = U(0.0), J3 = U(0.0), K = U(0.0), K1 = U(0.0);
    const double *gx, *gw;
    // smooth integrands while q(0) = 2 - v/(1 - v) > 0 (below the photon
    // sphere, v < 2/3); 20/24/32/48 nodes for v <= 0.6/0.64/0.66 and above
    // keep the relative error below 1e-13 (against a 128-node rule)
    const double vv = value(v);
    const int n = vv <= 0.6 ? 20 : (vv <= 0.64 ? 24 : (vv <= 0.66 ? 32 : 48));
    gl_rule(bx, bw, n, gx, gw);
    const U vw = v / (1.0 - v);
    for (int q = q0; q < n; q += qs) {
        double x = gx[q], w = gw[q];
        double t = 1.0 - x * x, tt = t * t;
        U Q = 2.0 - x * x - vw * tt;
        U irq = rsqrt_nr(Q);
        U rq = Q * irq;
        J += w * irq;
        J3 += w * tt * (irq * irq * irq);
        U gq = rq + x * Q;
        U igq = rcp_nr(gq);
        K += w * igq;
        K1 += w * (0.5 * irq + x) * tt * (igq * igq);
    }
    U om = 1.0 - v;
    ph = 2.0 / sqrt(om) * J;
    dph = (J + J3 / om) / (om * sqrt(om));
    th = 2.0 / om * K;
    dth = 2.0 / (om * om) * K + 2.0 / om * K1 / (om * om);
}


template <class T>
__device__ inline void hermite(const T &t, T &h00, T &h10, T &h01, T &h11)
{
    T t2 = t * t, t3 = t2 * t;
    h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
    h10 = t3 - 2.0 * t2 + t;
    h01 = -2.0 * t3 + 3.0 * t2;
    h11 = t3 - t2;
}

template <class T>
__device__ inline void dhermite(const T &t, T &d00, T &d10, T &d01, T &d11)
{
    T t2 = t * t;
    d00 = 6.0 * t2 - 6.0 * t;
    d10 = 3.0 * t2 - 4.0 * t + 1.0;
    d01 = -6.0 * t2 + 6.0 * t;
    d11 = 3.0 * t2 - 2.0 * t;
}


// x shift log10(1 + t) / hx of an interpolated redshift z_A (1 + t), with
// ixl = 1 / (hx ln 10): FP64 halvings (1 + t = (1 + t')^2, t' = t / (1 +
// sqrt(1 + t))) down to |t| <= 1/16, then ln(1 + t) = 2 atanh(s), s = t / (2
// + t), from its series in FP32 (|s| <= 1/31: s (1 + s^2/3 + s^4/5) is within
// 2e-10 relative).  Its error stays below the FP32 rounding of the x
// fraction it feeds.
__device__ inline float x_shift(double t, float ixl)
{
    int k = 0;
    while (fabs(t) > 0.0625 && k < 64) {     // |t'| < |t| / 2 for t > 0; capped for t near -1
        const double u = 1.0 + t;
        t = t * rcp_nr(1.0 + u * rsqrt_nr(u));
        ++k;
    }
    const float tf = (float)t;
    const float s = tf * __builtin_amdgcn_rcpf(2.0f + tf), s2 = s * s;
    const float l = 2.0f * s * (1.0f + s2 * (1.0f / 3.0f + s2 * (1.0f / 5.0f)));
    return ldexpf(l, k) * ixl;
}

// Energies whose x position I0 + fr + tbe[e] lies outside the table's node
// range (interval index below 0 or above nx - 2): stage B gives them a zero
// quad (windowed kernels).  fr + tbe[e] is computed as stage B computes it (FP32), so the count
// is that of the evaluation; tbe increases from tbe[0] = 0.
__device__ inline int x_outside_count(int I0, float fr, const float *tbe, int E, int nx)
{
    int n = 0;
    if (I0 < 0) {                                   // interval index I0 + floor(fr + tbe) < 0
        const float lim = (float)(-I0);
        int lo = 0, hi = E;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (fr + tbe[mid] < lim) lo = mid + 1; else hi = mid;
        }
        n += lo;
    }
    const float lim = (float)(nx - 1 - I0);         // interval index above nx - 2
    if (fr + tbe[E - 1] >= lim) {
        int lo = 0, hi = E;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (fr + tbe[mid] < lim) lo = mid + 1; else hi = mid;
        }
        n += E - lo;
    }
    return n;
}

__device__ inline int lin_bracket(double v, double v0, double h, int n, double &w1)
{
    double t = (v - v0) / h;
    if (t <= 0.0) { w1 = 0.0; return 0; }
    if (t >= n - 1) { w1 = 1.0; return n - 2; }
    int i = (int)floor(t);
    if (i > n - 2) i = n - 2;
    w1 = t - i;
    return i;
}


// cell azimuth, crescent mask, observed-phase lookup (Eqs. 45-46) on the
// ring's fine-phase arrays
__device__ inline double cell_offset(const RingRec &g, int j)
{
    if (g.shape == PPM_SHAPE_ANNULUS) {
        int h = g.n_cells / 2;
        if (j < h) return -(g.dphi_in + (h - 1 - j + 0.5) * g.dphi_cell);
        return g.dphi_in + (j - h + 0.5) * g.dphi_cell;
    }
    return -g.dphi_out + (j + 0.5) * g.dphi_cell;
}

// HEALPix ring i = 1 .. 4 nside - 1 (Sect. 2.8.1): cos(colatitude), pixels on
// the ring and the azimuth of its first pixel (pixels 2 pi / n apart); rings
// south of the equator mirror their northern counterparts.
__host__ __device__ inline void healpix_ring(int nside, int i, double &z, int &n, double &first)
{
    const int m = i > 2 * nside ? 4 * nside - i : i;
    const double ns = nside;
    double zz;
    if (m < nside) {
        zz = 1.0 - (double)m * m / (3.0 * ns * ns);
        n = 4 * m;
        first = kPi / (4.0 * m);
    } else {
        zz = 4.0 / 3.0 - 2.0 * m / (3.0 * ns);
        n = 4 * nside;
        first = kPi / (2.0 * ns) * ((m - nside) % 2 == 0 ? 0.5 : 1.0);
    }
    z = i > 2 * nside ? -zz : zz;
}

// index of the first pixel of HEALPix ring i in ring order
__host__ __device__ inline long long healpix_first_pixel(int nside, int i)
{
    const long long N = nside;
    if (i < nside) return 2LL * i * (i - 1);
    if (i <= 3 * nside) return 2LL * N * (N - 1) + 4LL * N * (i - nside);
    const long long m = 4LL * N - i;
    return 12LL * N * N - 2LL * m * (m + 1);
}

__device__ inline bool cell_masked(const RingRec &g, double off)
{
    if (g.shape != PPM_SHAPE_CRESCENT) return false;
    double cd = cos(g.theta) * cos(g.tm) + sin(g.theta) * sin(g.tm) * cos(off);
    return cd > g.cos_zm;
}

struct PhaseSample { double F, z, mu; };

__device__ inline PhaseSample phase_lookup(const double4 *tr, int nfp, double php)
{
    int lo = 0, hi = nfp;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (tr[mid].z <= php) lo = mid; else hi = mid;
    }
    const double4 a = tr[lo], c = tr[lo + 1];
    double w = (php - a.z) / (c.z - a.z);
    w = fmin(1.0, fmax(0.0, w));
    PhaseSample s;
    s.F = a.x + w * (c.x - a.x);
    s.z = a.y + w * (c.y - a.y);
    s.mu = a.w + w * (c.w - a.w);
    return s;
}

// The accumulation kernels run on 1D grids: block L is dispatched to XCD
// L % kXcds (round-robin), so the n_tile phase tiles of one ring are given
// block numbers on the same XCD and share its L2 copy of the ring's
// sub-table and trace.  Blocks past the work list return at once.
constexpr int kXcds = 8;

__host__ __device__ inline int xcd_grid(int n_list, int n_tile)
{
    return kXcds * n_tile * ((n_list + kXcds - 1) / kXcds);
}

// work-list entries one accumulation launch may take: its grid of n_tile
// blocks per entry, `threads` each, stays below 2^32 threads (a launch
// limit); a multiple of the XCD count.  PPM_MAX_LAUNCH_THREADS lowers the
// limit (tests use it to split launches on small workloads).
inline int max_list_per_launch(int n_tile, int threads)
{
    long long lim = 4294967295LL;
    if (const char *env = std::getenv("PPM_MAX_LAUNCH_THREADS")) {
        const long long v = std::strtoll(env, nullptr, 10);
        if (v >= 1 && v < lim) lim = v;
    }
    const long long m = lim / ((long long)n_tile * threads);
    return m < kXcds ? kXcds : (int)((m / kXcds) * kXcds);
}

__device__ inline bool xcd_block(int n_list, int n_tile, int &li, int &tile)
{
    const int L = blockIdx.x, x = L % kXcds, j = L / kXcds;
    const int g = j / n_tile;
    tile = j - g * n_tile;
    li = g * kXcds + x;
    return li < n_list;
}

__device__ inline float readlane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// value of lane + 1 (0 in lane 63): DPP whole-wave shift; bound control
// writes 0 where the source lane is past the wave, so no zero operand is
// materialised
__device__ inline float wave_next_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xf, 0xf, true));
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


}  // namespace ppm
