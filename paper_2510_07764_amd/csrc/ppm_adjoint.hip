// gfx950 kernels of the gradient of the Poisson log-likelihood with respect
// to the twelve model parameters (M, R_e, i, Phi, N_H and per spot theta,
// zeta, logT, plus spot 2's longitude offset).
//
// The gradient is the exact derivative of the discrete model the forward
// kernels evaluate (almost everywhere: interpolation stencils, visibility
// ranges and clamps are held fixed; node positions of the per-ring
// deflection table are held fixed in alpha).  It is assembled in three
// modes:
//   reverse  likelihood, response fold and absorption (Eqs. 22, 55):
//            g_m = d/m - 1, G[k][e] = (T_exp/P) sum_c g_m[k][c] RSP[e][c],
//            the flux adjoint G exp(-N_H sigma_e), and the N_H derivative;
//   reverse  over energies inside the accumulation (Eq. 47): per (cell,
//            phase) pair the five sums over e of G/E times I, dI/dx, dI/dmu,
//            dI/dlogT, dI/dlog g of the mixed-order interpolant (Sect. 4);
//   forward  dual-number tangents of the ring geometry (Eqs. 2-11, 18),
//            the deflection table (d/du at fixed alpha of Eqs. 14, 16, 17,
//            32, 35) and the fine-phase trace (Eqs. 38-44) along the five
//            geometric directions of a ring, contracted with the per-pair
//            sums in FP64.
// Section and equation numbers refer to arXiv:2510.07764.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ppm_internal.h"
#include "ppm_device.h"
#include "ppm_launch.h"
#include "../../include/ppm.h"

namespace ppm {

using D1 = Dual<1>;
using D5 = Dual<5>;

constexpr double kLn10 = 2.302585092994045684;

// ---------------------------------------------------------------------------
// k_fold_bwd: reverse mode through the likelihood, fold and absorption, on
// the matrix cores in FP64: G[row][e] = (T_exp/P) sum_c g_m[row][c] RSP[e][c]
// for rows (instance b, phase k), with g_m = d/m - 1 (-1 where d = 0; m the
// model plus background counts) formed as the A operand is loaded.  Block =
// one 16 x 16 tile (16 rows, 16 energies), four waves splitting the channels
// into quarters; per wave K in steps of 4 (v_mfma_f64_16x16x4f64): lane l
// supplies A[l%16][c0 + l/16] and RSP^T[c0 + l/16][l%16], and the tile comes
// back as D[l/16 + 4 v][l%16] in accumulator v.  The four partial tiles
// are added in wave order.  Epilogue: the flux adjoint divided by E (FP32,
// for the accumulation kernel) and the N_H derivative summed over the
// tile's 16 energies per row in a fixed lane butterfly.
// ---------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_fold_bwd(DevSpec S, const StarRec *stars, const double *counts,
                                                  const int32_t *data, const double *flux, float *gtil,
                                                  double *nh_part, int M)
{
    __shared__ doublex4 part[4][64];
    const int P = S.P, C = S.C, E = S.E;
    const int n0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int kq = ((C + 15) / 16) * 4;
    const int kb = wave * kq, ke = min(C, kb + kq);
    const int arow = m0 + li, ecol = n0 + li;
    const bool mrow = arow < M, ncol = ecol < E;
    const int ak = mrow ? arow % P : 0;
    const double *mrow_p = counts + (size_t)(mrow ? arow : 0) * C;
    const int32_t *drow_p = data + (size_t)ak * C;
    const double *brow_p = S.bkg ? S.bkg + (size_t)ak * C : nullptr;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    // eight K steps at a time: their operands loaded and formed first, then
    // the MFMAs in K order
    constexpr int kSteps = 8;
    for (int cc = kb; cc < ke; cc += 4 * kSteps) {
        double av[kSteps], bv[kSteps];
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const int c = cc + 4 * s + lk;
            const bool oka = mrow && c < ke, okb = ncol && c < ke;
            const int dc = oka ? drow_p[c] : 0;
            double mc = oka ? mrow_p[c] : 1.0;
            if (brow_p && oka) mc += brow_p[c];                          // model plus background
            av[s] = oka ? (dc == 0 ? -1.0 : dc / mc - 1.0) : 0.0;        // d/dm of d ln m - m
            bv[s] = okb ? S.rspT64[(size_t)c * E + ecol] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < kSteps; ++s)
            if (cc + 4 * s < ke) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
    }
    part[wave][l] = acc;
    __syncthreads();
    // wave w: output rows l/16 + 4 w of the tile
    const double *p0 = (const double *)&part[0][l], *p1 = (const double *)&part[1][l],
                 *p2 = (const double *)&part[2][l], *p3 = (const double *)&part[3][l];
    double t = p0[wave];
    t += p1[wave];
    t += p2[wave];
    t += p3[wave];
    const int row = m0 + lk + 4 * wave, e = n0 + li;
    double nh = 0.0;
    if (row < M && e < E) {
        const int b = row / P;
        const double Gp = t * (S.t_exp / P);                   // adjoint of the absorbed flux
        const double att = S.sigma ? exp(-stars[b].NH * S.sigma[e]) : 1.0;
        const size_t o = (size_t)row * E + e;
        gtil[o] = (float)(Gp * att / S.energy[e]);
        if (S.sigma) nh = -Gp * flux[o] * att * S.sigma[e] * 1e20;   // N_H in units of 1e20 cm^-2
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) nh += __shfl_xor(nh, o, 64);
    if (li == 0 && row < M) nh_part[(size_t)row * gridDim.x + blockIdx.x] = nh;
}

// ---------------------------------------------------------------------------
// k_table_u: d/du at fixed alpha of the per-ring table entries (psi, psi',
// c dt/R, its alpha derivative), by a dual number in u carried through the
// same quadrature as the forward table.  The oblate radial delay terms are
// written with kappa = R_e/R(theta) held fixed: their kappa derivative,
// 1 + u/(kappa - u), is the same on both branches and independent of alpha.
// ---------------------------------------------------------------------------
__device__ inline D1 acos_capped(const D1 &a)
{
    return a.v >= 1.0 ? D1(0.0) : acos(a);
}

__global__ __launch_bounds__(64) void k_table_u(DevSpec S, const int32_t *list, const StarRec *stars, const RingRec *rings,
                          double4 *table_u)
{
    const int ent = list[blockIdx.x], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const RingRec g = rings[(size_t)b * S.R_tot + r];
    if (!g.active) return;
    const StarRec st = stars[b];
    const D1 u = D1::seed(g.u, 0);
    const double kap = st.Re / g.R;
    const D1 sq = sqrt(1.0 - u);
    const D1 cdt_obl = kap - 1.0 + u * log((kap - u) / (1.0 - u));   // Eq. (16) over R
    const double dal = g.alpha_max / (S.n_alpha - 1);
    double4 *tab = table_u + ((size_t)b * S.R_tot + r) * S.n_alpha;
    for (int j = blockIdx.y * blockDim.x + threadIdx.x; j < S.n_alpha; j += gridDim.y * blockDim.x) {
        double a = dal * j;
        if (j == S.n_alpha - 1) a = g.alpha_max;
        D1 psi, dpsi, T, dT;
        if (a <= kHalfPi) {
            D1 tp;
            bend_out(S.glx, S.glw, u, a, psi, dpsi, tp);
            T = tp + cdt_obl;
            dT = dpsi * sin(a) / sq;
        } else {
            const double be = kPi - a;
            D1 psb, dpsb, tpb;
            bend_out(S.glx, S.glw, u, be, psb, dpsb, tpb);
            const double sa = sin(a), ca = cos(a);
            D1 kk = sqrt(3.0 * (1.0 - u));
            D1 arg = 3.0 * u * kk / (2.0 * sa);
            if (arg.v > 1.0) arg = D1(1.0);
            D1 rho = -2.0 * sa / kk * cos((acos_capped(arg) + kTwoPi) / 3.0);   // Eq. (14)
            D1 k = sa * sa / (1.0 - u), kp = 2.0 * sa * ca / (1.0 - u);
            D1 rhop = kp * (rho - u) / (3.0 * rho * rho - k);
            D1 v = u / rho, vp = -u * rhop / (rho * rho);
            D1 ph, dph, th, dth;
            grazing(S.glx, S.glw, v, ph, dph, th, dth);
            psi = 2.0 * ph - psb;
            dpsi = 2.0 * dph * vp + dpsb;
            D1 cdtp = kap - rho + u * log((kap - u) / (rho - u));
            T = 2.0 * rho * th - tpb + 2.0 * cdtp - cdt_obl;             // Eq. (17)
            D1 dtpb = dpsb * sin(be) / sq;
            dT = 2.0 * rhop * th + 2.0 * rho * dth * vp + dtpb - 2.0 * rhop * rho / (rho - u);
        }
        tab[j] = make_double4(psi.d[0], dpsi.d[0], T.d[0], dT.d[0]);
    }
}

// ---------------------------------------------------------------------------
// k_trace_tan: tangents of the fine-phase trace (F, z, phi_o, mu) of one ring
// along its five geometric directions, and the ring-level tangents.  Thread
// 0 redoes the ring setup of Eqs. (2)-(11), (18) and the spot grid in dual
// numbers; every thread then redoes the visible samples of Eqs. (38)-(40)
// with the table lookup differentiated through its node values (psi_j,
// psi'_j, T_j, T'_j move with u and kappa).  Visibility and the invisible
// range come from the forward trace; the fill of Eqs. (41)-(44) is linear
// in its end samples and so are its tangents.
// ---------------------------------------------------------------------------
struct RingDualRaw {   // plain storage of dual numbers in shared memory
    double sth[6], cth[6], u[6], sq1u[6], kap[6], R[6], coseta[6], sineta[6], beta[6], gamma[6], si[6], ci[6];
};

__device__ inline void put(double *dst, const D5 &x)
{
    dst[0] = x.v;
#pragma unroll
    for (int i = 0; i < 5; ++i) dst[1 + i] = x.d[i];
}

__device__ inline D5 get(const double *src)
{
    D5 x(src[0]);
#pragma unroll
    for (int i = 0; i < 5; ++i) x.d[i] = src[1 + i];
    return x;
}

// node value with its tangent: v + du * u' + dk * kappa'
__device__ inline D5 node(double v, double du, const D5 &u, double dk, const D5 &kap)
{
    D5 x(v);
#pragma unroll
    for (int i = 0; i < 5; ++i) x.d[i] = du * u.d[i] + dk * kap.d[i];
    return x;
}

__global__ __launch_bounds__(256) void k_trace_tan(DevSpec S, const int32_t *list, const double *params, const int32_t *n_cells,
                            const StarRec *stars, const RingRec *rings, const double4 *table,
                            const double4 *table_u, const double4 *trace, double4 *tangent, RingTan *ringtan)
{
    extern __shared__ double4 lds4[];
    const int ent = list[blockIdx.x], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const size_t slot = (size_t)b * S.R_tot + r;
    const RingRec g = rings[slot];
    if (!g.active) return;
    const int na = S.n_alpha, nfp = S.n_fp;
    double4 *tab = lds4;               // na
    double4 *tabu = tab + na;          // na
    double4 *tg = tabu + na;           // (nfp + 1) * 5
    __shared__ RingDualRaw rd;
    for (int j = threadIdx.x; j < na; j += blockDim.x) {
        tab[j] = table[slot * na + j];
        tabu[j] = table_u[slot * na + j];
    }
    if (threadIdx.x == 0) {
        const double *p = params + (size_t)b * PPM_NPARAM;
        const int spot = g.spot;
        const int lr = spot == 0 ? r : r - S.rings_max[0];
        const int ov = n_cells ? n_cells[b] : 0;
        const int nr = ov > 0 ? ov : S.n_rings_spec[spot];
        const int np = ov > 0 ? ov : S.n_phi_spec[spot];
        const D5 M = D5::seed(p[0], 0), Re = D5::seed(p[1] * 1e5, 1, 1e5), inc = D5::seed(p[2], 2);
        const D5 tc = D5::seed(p[8 + 4 * spot], 3), z = D5::seed(p[9 + 4 * spot], 4);
        const double nu = p[5], Dd = p[6] * kPc;
        D5 GM = M * kGMsun;
        D5 Rs = 2.0 * GM / (kC * kC);
        D5 x = GM / (kC * kC * Re);
        D5 Obar = kTwoPi * nu * sqrt(Re * Re * Re / GM);
        D5 o2 = (S.mode == PPM_MODE_OS) ? Obar * Obar * (-0.788 + 1.030 * x) : D5(0.0);   // Eq. (7)
        D5 g0 = GM / (Re * Re) / sqrt(1.0 - Rs / Re);
        D5 lo = fmax(D5(0.0), tc - z), hi = fmin(D5(kPi), tc + z);
        D5 e0 = lo + (hi - lo) * (double)lr / (double)nr, e1 = lo + (hi - lo) * (double)(lr + 1) / (double)nr;
        D5 th = 0.5 * (e0 + e1);
        D5 dcos = cos(e0) - cos(e1);
        D5 ct = cos(th), sn = sin(th);
        D5 R = Re * (1.0 + o2 * ct * ct);
        D5 dR = -2.0 * Re * o2 * ct * sn;
        D5 u = Rs / R;
        D5 sq1u = sqrt(1.0 - u);
        D5 f = dR / (R * sq1u);                                       // Eq. (2)
        D5 coseta = 1.0 / sqrt(1.0 + f * f), sineta = f / sqrt(1.0 + f * f);
        D5 logg = log10(g0 * gravity_ratio_t(S.mode, x, Obar, th));   // Eqs. (10), (11)
        D5 beta = kTwoPi * nu * R * sn / (kC * sq1u);                  // Eq. (18)
        D5 gamma = 1.0 / sqrt(1.0 - beta * beta);
        D5 dout = arc_halfwidth(th, tc, z), din(0.0), dcell;
        if (g.shape == PPM_SHAPE_ANNULUS) {
            din = arc_halfwidth(th, tc, S.shape_a[spot] * z);
            dcell = (dout - din) / (0.5 * np);
        } else {
            dcell = 2.0 * dout / (double)np;
        }
        D5 w = R * R * sqrt(1.0 + f * f) * dcos * dcell / (Dd * Dd);  // Eq. (9)
        RingTan rt;
        for (int i = 0; i < 5; ++i) {
            rt.dlogg[i] = logg.d[i];
            rt.dw[i] = w.d[i];
            rt.ddout[i] = dout.d[i];
            rt.ddin[i] = din.d[i];
        }
        ringtan[slot] = rt;
        put(rd.sth, sn); put(rd.cth, ct); put(rd.u, u); put(rd.sq1u, sq1u); put(rd.kap, Re / R); put(rd.R, R);
        put(rd.coseta, coseta); put(rd.sineta, sineta); put(rd.beta, beta); put(rd.gamma, gamma);
        put(rd.si, sin(inc)); put(rd.ci, cos(inc));
    }
    __syncthreads();
    const D5 sth = get(rd.sth), cth = get(rd.cth), u = get(rd.u), sq1u = get(rd.sq1u), kap = get(rd.kap);
    const D5 Rr = get(rd.R), coseta = get(rd.coseta), sineta = get(rd.sineta), beta = get(rd.beta);
    const D5 gamma = get(rd.gamma), si = get(rd.si), ci = get(rd.ci);
    const double nu = params[(size_t)b * PPM_NPARAM + 5];
    const double Xk = 1.0 + g.u / (kap.v - g.u);     // d(c dt/R)/d kappa, both branches
    const double dal = g.alpha_max / (na - 1);
    const double psi_top = tab[na - 1].x;
    const int a0 = g.inv_min, a1 = g.inv_max;
    for (int i = threadIdx.x; i <= nfp; i += blockDim.x) {
        double4 out[5];
        for (int d = 0; d < 5; ++d) out[d] = make_double4(0.0, 0.0, 0.0, 0.0);
        const bool vis = i < a0 || i > a1;
        if (vis) {
            const double phi = kTwoPi * i / nfp;
            double sphi, cphi;
            sincos(phi, &sphi, &cphi);
            D5 cpsi = si * sth * cphi + ci * cth;                      // Table 2
            if (cpsi.v > 1.0) cpsi = D5(1.0);
            if (cpsi.v < -1.0) cpsi = D5(-1.0);
            const double spsi = ::sqrt(fmax(0.0, 1.0 - cpsi.v * cpsi.v));
            D5 psi = spsi > 1e-7 ? acos(cpsi) : D5(::acos(cpsi.v));
            D5 a, sr, lf;
            if (psi.v < 1e-7) {
                a = psi * sq1u;
                sr = sq1u;
                lf = 1.0 - u;
            } else {
                int lo = 0, hi = na - 1;
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (tab[mid].x <= psi.v) lo = mid; else hi = mid;
                }
                (void)psi_top;
                const D5 p0 = node(tab[lo].x, tabu[lo].x, u, 0.0, kap);
                const D5 p1 = node(tab[lo + 1].x, tabu[lo + 1].x, u, 0.0, kap);
                const D5 m0 = 1.0 / node(tab[lo].y, tabu[lo].y, u, 0.0, kap);
                const D5 m1 = 1.0 / node(tab[lo + 1].y, tabu[lo + 1].y, u, 0.0, kap);
                const D5 h = p1 - p0;
                const D5 t = (psi - p0) / h;
                const double al0 = dal * lo;
                const double al1 = (lo + 1 == na - 1) ? g.alpha_max : dal * (lo + 1);
                D5 h00, h10, h01, h11, d00, d10, d01, d11;
                hermite(t, h00, h10, h01, h11);
                dhermite(t, d00, d10, d01, d11);
                a = h00 * al0 + h10 * h * m0 + h01 * al1 + h11 * h * m1;
                D5 dadpsi = (d00 * al0 + d10 * h * m0 + d01 * al1 + d11 * h * m1) / h;
                sr = sin(a) / sin(psi);
                lf = sr * dadpsi;
            }
            D5 ca = cos(a);
            D5 cs = ca * coseta + sr * sineta * (ci * sth - si * cth * cphi);   // Eq. (4)
            D5 cxi = -sr * si * sphi;
            D5 delta = 1.0 / (gamma * (1.0 - beta * cxi));                     // Eq. (19)
            D5 mu = delta * cs;                                                // Eq. (20)
            D5 F = sq1u * delta * delta * delta * mu * lf * gamma;             // Eq. (40)
            D5 zz = 1.0 / (delta * sq1u);
            int jj = (int)floor(a.v / dal);
            jj = jj < 0 ? 0 : (jj > na - 2 ? na - 2 : jj);
            D5 ta = (a - dal * jj) / dal;
            D5 h00, h10, h01, h11;
            hermite(ta, h00, h10, h01, h11);
            const D5 T0 = node(tab[jj].z, tabu[jj].z, u, Xk, kap), T1 = node(tab[jj + 1].z, tabu[jj + 1].z, u, Xk, kap);
            const D5 dT0 = node(tab[jj].w, tabu[jj].w, u, 0.0, kap), dT1 = node(tab[jj + 1].w, tabu[jj + 1].w, u, 0.0, kap);
            D5 T = h00 * T0 + h10 * dal * dT0 + h01 * T1 + h11 * dal * dT1;
            D5 po = nu * Rr * T / kC;                                          // phi/2pi has no tangent
            for (int d = 0; d < 5; ++d) out[d] = make_double4(F.d[d], zz.d[d], po.d[d], mu.d[d]);
        }
        for (int d = 0; d < 5; ++d) tg[i * 5 + d] = out[d];
    }
    __syncthreads();
    if (a0 <= a1) {
        const int ia = a0 - 1, ib = a1 + 1 > nfp ? nfp : a1 + 1;
        for (int i = a0 + threadIdx.x; i <= a1; i += blockDim.x) {
            const double t = (double)(i - ia) / (double)(ib - ia);
            for (int d = 0; d < 5; ++d) {
                const double4 va = tg[ia * 5 + d], vb = tg[ib * 5 + d];
                tg[i * 5 + d] = make_double4(0.0, va.y + (vb.y - va.y) * t, va.z + (vb.z - va.z) * t, 0.0);
            }
        }
    }
    __syncthreads();
    double4 *dst = tangent + slot * (size_t)(nfp + 1) * 5;
    for (int i = threadIdx.x; i < (nfp + 1) * 5; i += blockDim.x) dst[i] = tg[i];
}

// ---------------------------------------------------------------------------
// k_subtable_tg: logT and log g derivatives of the per-ring (logT, log g)
// collapse (linear on both axes; zero where the ring is clamped to an edge),
// over the same x window as the forward sub-table.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_subtable_tg(DevSpec S, const int32_t *list, const RingRec *rings, float2 *subtg)
{
    const int ent = list[blockIdx.x], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const RingRec g = rings[(size_t)b * S.R_tot + r];
    if (!g.active) return;
    double wt1, wg1;
    const int it = lin_bracket(g.logT, S.T0, S.hT, S.nT, wt1);
    const int ig = lin_bracket(g.logg, S.g0, S.hg, S.ng, wg1);
    const double tT = (g.logT - S.T0) / S.hT, tG = (g.logg - S.g0) / S.hg;
    const float dT = (tT <= 0.0 || tT >= S.nT - 1) ? 0.0f : (float)(1.0 / S.hT);
    const float dG = (tG <= 0.0 || tG >= S.ng - 1) ? 0.0f : (float)(1.0 / S.hg);
    const float vt1 = (float)wt1, vg1 = (float)wg1;
    const size_t slab = (size_t)S.nmu * S.nx;
    const float *s00 = S.atm + ((size_t)it * S.ng + ig) * slab;
    const float *s01 = s00 + slab;
    const float *s10 = S.atm + ((size_t)(it + 1) * S.ng + ig) * slab;
    const float *s11 = s10 + slab;
    const int W = S.W_max, xw0 = g.xw0, xw = g.xw;
    float2 *out = subtg + ((size_t)b * S.R_tot + r) * (size_t)S.sub_stride;
    for (int i = threadIdx.x; i < S.nmu * W; i += blockDim.x) {
        int m = i / W, c = i - m * W;
        float2 v = make_float2(0.0f, 0.0f);
        if (c < xw) {
            size_t o = (size_t)m * S.nx + xw0 + c;
            const float a00 = s00[o], a01 = s01[o], a10 = s10[o], a11 = s11[o];
            v.x = ((1.0f - vg1) * (a10 - a00) + vg1 * (a11 - a01)) * dT;
            v.y = ((1.0f - vt1) * (a01 - a00) + vt1 * (a11 - a10)) * dG;
        }
        out[i] = v;
    }
}

// ---------------------------------------------------------------------------
// k_accum_adj: reverse mode of the windowed accumulation (Eq. 47) over
// energies, per (cell, phase) pair, contracted with the geometry tangents.
// Block = (ring, tile of S.pt_adj phases), kAdjWaves waves; a wave owns one
// phase at a time.
//  stage A  lane = cell: observed-phase lookup (Eqs. 45-46), mu weights and
//           their mu derivatives (cubic Lagrange; linear in the protected
//           zone and the last interval; zero derivative where mu is clamped),
//           x position of the first energy; wave ballot of visible pairs;
//  stage B  per visible pair: lane = x interval, the moments sum_e G~ f^k
//           (k = 0..3) of the energies in it from per-bucket prefix sums
//           (built once per phase), turned into weights of the interval's
//           interpolation nodes and gathered per node by DPP wave shifts;
//           lane = x node, mu contraction of the sub-table and of its
//           logT / log g derivatives, times the node weights: the sums
//           over e of G~ V, G~ dV/dt, G~ dV/dmu (wave totals kept by the
//           pair's lane) and F_p G~ dV/dlogT, F_p G~ dV/dlog g (lane-local
//           FP64 sums), with G~ = G[k][e]/E_e;
//  stage C  lane = pair, FP64: chain rule through the phase interpolation
//           into the five geometric directions and the phase direction,
//           plus the ring-level sums for the cell weight, log g and logT.
// The nine per-lane FP64 sums are reduced over the block in a fixed order.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// sum over the 64 lanes, in every lane: DPP butterflies within rows of 16
// lanes (quad swaps, half-row and row mirrors), then swaps of rows 0/1 and 2/3
// (swizzle, xor 16) and of the two halves (lane permute, xor 32).  Every lane
// adds the same operands, so all lanes hold the same bits: for lane 63 the
// order is (R3 + R2) + (R1 + R0) over the row sums R.
__device__ inline float wave_allsum(float v, int bp32)
{
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    v += __int_as_float(__builtin_amdgcn_ds_bpermute(bp32, __float_as_int(v)));
    return v;
}


__device__ inline double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// d(cell azimuth)/d(outer half-width) and d/d(inner half-width) of cell j
__device__ inline void offset_coeffs(const RingRec &g, int j, double &ca, double &cb)
{
    if (g.shape == PPM_SHAPE_ANNULUS) {
        const int h = g.n_cells / 2;
        if (j < h) {
            const double q = (h - 1 - j + 0.5) / h;
            ca = -q;
            cb = -1.0 + q;
        } else {
            const double q = (j - h + 0.5) / h;
            ca = q;
            cb = 1.0 - q;
        }
    } else {
        ca = -1.0 + (2.0 * j + 1.0) / g.n_cells;
        cb = 0.0;
    }
}

// binary-search steps within an energy bucket the kernel unrolls (the plan
// refuses energy grids whose buckets need more)
constexpr int kMaxBucketSteps = 4;

// value of lane - 1 (0 in lane 0): DPP whole-wave shift (bound control
// writes the 0)
__device__ inline float wave_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// Node weights of interval lane's cubic (or linear, or zero) interpolant for
// its energy moments M: sum_e G_e V(f_e) = sum_j beta_j S_{lane + j} over the
// interval's four nodes S (V = q.x + q.y f + q.z f^2 + q.w f^3 with q from
// cubic_quad), and the same for dV/df (moments (0, M0, 2 M1, 3 M2)); each
// node then gathers the weights of the four intervals that use it (lanes
// n, n - 1, n - 2, n - 3), so that the sums over e become one product per
// node lane.
__device__ inline void node_weights(int kind, float M0, float M1, float M2, float M3, float &B, float &Bx)
{
    float b0, b1, b2, b3, d0, d1, d2, d3;
    if (kind == 0) {                               // cubic on nodes -1, 0, 1, 2
        b0 = -M1 * (1.0f / 3.0f) + 0.5f * M2 - M3 * (1.0f / 6.0f);
        b1 = M0 - 0.5f * M1 - M2 + 0.5f * M3;
        b2 = M1 + 0.5f * M2 - 0.5f * M3;
        b3 = (M3 - M1) * (1.0f / 6.0f);
        d0 = -M0 * (1.0f / 3.0f) + M1 - 0.5f * M2;
        d1 = -0.5f * M0 - 2.0f * M1 + 1.5f * M2;
        d2 = M0 + M1 - 1.5f * M2;
        d3 = 0.5f * M2 - M0 * (1.0f / 6.0f);
    } else if (kind == 1) {                        // linear between nodes 0 and 1
        b0 = 0.0f; b1 = M0 - M1; b2 = M1; b3 = 0.0f;
        d0 = 0.0f; d1 = -M0; d2 = M0; d3 = 0.0f;
    } else {                                       // outside the table: no contribution
        b0 = b1 = b2 = b3 = d0 = d1 = d2 = d3 = 0.0f;
    }
    B = b0 + wave_prev(b1 + wave_prev(b2 + wave_prev(b3)));
    Bx = d0 + wave_prev(d1 + wave_prev(d2 + wave_prev(d3)));
}

// Stage B of k_accum_adj for the visible pairs (mask) of one 64-cell group;
// the pair's lane keeps its three energy sums in R0, R1, R2.
// Energy sums by moments: lane l stands for x interval I0 + l of the pair,
// which holds the energies with l <= fr + tbe < l + 1, i.e. the tail of
// bucket l - 1 (tau >= 1 - fr, f = fr - 1 + tau) and the head of bucket l
// (tau < 1 - fr, f = fr + tau).  From the per-bucket inclusive prefix sums
// Lw[e] of G (1, tau, tau^2, tau^3) (the wave's phase) the interval's
// moments sum_e G f^k, k = 0..3, follow by the binomial expansion in the
// shift fr or fr - 1; every sum over e of G V, G dV/df, G dV/dmu, G dV/dlogT
// and G dV/dlog g is then a product of the node values with the interval
// weights of node_weights, summed over the wave.  The wave totals of a pair
// are taken while the next pair's table rows load.  INTERIOR: the ring's x
// window stays one interval clear of the table's first and last intervals
// (every interval an energy can use is cubic and every stencil column lies
// in the window; columns past it hold zeros), so the bounds tests drop out.
template <bool INTERIOR>
__device__ __forceinline__ void adj_pairs(uint64_t mask, const float4 *Pp, const float (&vv)[4], float fr, float Fpf,
                                          int I0, int m0, int lane, int bp32, const float *tab, const float2 *tab2,
                                          int W, int xw0, int xw, int nx, const float4 *Lw, const float *etau,
                                          int est, int een, int e_it, float &R0, float &R1, float &R2, double &accT,
                                          double &accG)
{
    float ps0 = 0.f, psx = 0.f, psm = 0.f;   // lane sums of the previous pair
    int pp = -1;                            // its lane (none yet)
    while (mask) {
        const int p = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        // the pair's mu weights, broadcast from its lane's LDS record; their mu
        // derivatives by lane reads
        const float4 pw = Pp[p];
        const float pw0 = pw.x, pw1 = pw.y, pw2 = pw.z, pw3 = pw.w;
        const float pv0 = readlane_f(vv[0], p), pv1 = readlane_f(vv[1], p), pv2 = readlane_f(vv[2], p),
                    pv3 = readlane_f(vv[3], p);
        const float pfr = readlane_f(fr, p), pF = readlane_f(Fpf, p);
        const int pI0 = __builtin_amdgcn_readlane(I0, p), pm0 = __builtin_amdgcn_readlane(m0, p);
        // the pair's four mu rows of the table and of its logT / log g planes at
        // x node pI0 - 1 + lane (zero outside the window)
        int col = pI0 - 1 + lane - xw0;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        float2 b0 = make_float2(0.f, 0.f), b1 = b0, b2 = b0, b3 = b0;
        if (INTERIOR || (col >= 0 && col < xw)) {
            if (INTERIOR) col = col < W - 1 ? col : W - 1;
            const float *t0 = tab + pm0 * W + col;
            const float2 *u0 = tab2 + pm0 * W + col;
            a0 = t0[0]; a1 = t0[W]; a2 = t0[2 * W]; a3 = t0[3 * W];
            b0 = u0[0]; b1 = u0[W]; b2 = u0[2 * W]; b3 = u0[3 * W];
        }
        {
            const float t0 = wave_allsum(ps0, bp32), t1 = wave_allsum(psx, bp32), t2 = wave_allsum(psm, bp32);
            const bool mine = lane == pp;
            R0 = mine ? t0 : R0;
            R1 = mine ? t1 : R1;
            R2 = mine ? t2 : R2;
        }
        // split of bucket `lane`: its first energy with tau + fr >= 1
        // (branch-free lower bound; etau[E] closes the array)
        int sp = est, n = een - est;
#pragma unroll
        for (int it = 0; it < kMaxBucketSteps; ++it) {
            if (it < e_it) {
                const int half = n >> 1;
                const float tv = etau[sp + half];
                const bool right = (n > 0) & (tv + pfr < 1.0f);
                sp = right ? sp + half + 1 : sp;
                n = right ? n - half - 1 : half;
            }
        }
        const bool has_hd = sp > est, has_b = een > est;
        float4 hd = Lw[has_hd ? sp - 1 : 0];               // head of the bucket: this interval
        float4 tb = Lw[has_b ? een - 1 : 0];               // whole bucket
        if (!has_hd) hd = make_float4(0.f, 0.f, 0.f, 0.f);
        if (!has_b) tb = make_float4(0.f, 0.f, 0.f, 0.f);
        // tail of bucket lane - 1: this interval's first energies
        const float t0 = wave_prev(tb.x - hd.x), t1 = wave_prev(tb.y - hd.y), t2 = wave_prev(tb.z - hd.z),
                    t3 = wave_prev(tb.w - hd.w);
        const float c = pfr, d = pfr - 1.0f;
        const float M0 = hd.x + t0;
        const float M1 = (hd.y + c * hd.x) + (t1 + d * t0);
        const float M2 = (hd.z + c * (2.0f * hd.y + c * hd.x)) + (t2 + d * (2.0f * t1 + d * t0));
        const float M3 = (hd.w + c * (3.0f * hd.z + c * (3.0f * hd.y + c * hd.x)))
                       + (t3 + d * (3.0f * t2 + d * (3.0f * t1 + d * t0)));
        int kind = 0;
        if (!INTERIOR) {
            const int gi = pI0 + lane;
            kind = (gi >= 1 && gi <= nx - 3) ? 0 : ((gi == 0 || gi == nx - 2) ? 1 : 2);
        }
        float Bn, Bx;
        node_weights(kind, M0, M1, M2, M3, Bn, Bx);
        const float va = pw0 * a0 + pw1 * a1 + pw2 * a2 + pw3 * a3;
        const float vm = pv0 * a0 + pv1 * a1 + pv2 * a2 + pv3 * a3;
        const float vT = pw0 * b0.x + pw1 * b1.x + pw2 * b2.x + pw3 * b3.x;
        const float vg = pw0 * b0.y + pw1 * b1.y + pw2 * b2.y + pw3 * b3.y;
        accT += (double)(pF * (vT * Bn));
        accG += (double)(pF * (vg * Bn));
        ps0 = va * Bn;
        psx = va * Bx;
        psm = vm * Bn;
        pp = p;
    }
    if (pp >= 0) {
        const float t0 = wave_allsum(ps0, bp32), t1 = wave_allsum(psx, bp32), t2 = wave_allsum(psm, bp32);
        const bool mine = lane == pp;
        R0 = mine ? t0 : R0;
        R1 = mine ? t1 : R1;
        R2 = mine ? t2 : R2;
    }
}

constexpr int kAdjWaves = 8;   // waves per block of k_accum_adj

__global__ __launch_bounds__(64 * kAdjWaves, 4) void k_accum_adj(DevSpec S, const int32_t *list, const RingRec *rings,
                                                   const RingTan *ringtan, const double4 *trace,
                                                   const double4 *tangent, const float *sub, const float2 *subtg,
                                                   const float *gtil, double *gpart, int n_list)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int PT = S.pt_adj;
    const int n_tile = (S.P + PT - 1) / PT;
    int li, tile;
    if (!xcd_block(n_list, n_tile, li, tile)) return;
    const int ent = list[li], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const size_t slot = (size_t)b * S.R_tot + r;
    const RingRec g = rings[slot];
    if (!g.active) return;
    const int nfp = S.n_fp, nmu = S.nmu, nx = S.nx, E = S.E, P = S.P, W = S.W_max;
    double4 *tr = (double4 *)lds_raw;                          // nfp + 1
    double *axmu = (double *)(tr + nfp + 1);                   // nmu (padded to 16 bytes)
    float *tab = (float *)(axmu + ((nmu + 1) & ~1));           // sub_stride
    float4 *Lb = (float4 *)(tab + S.sub_stride);               // kAdjWaves * E bucket prefix sums
    float4 *Pb = Lb + kAdjWaves * S.E;                         // kAdjWaves * 64 pair mu weights
    double *po = (double *)(Pb + kAdjWaves * 64);              // nfp + 1 phi_o, compact for the search
    double *ipo = po + nfp + 1;                                // nfp: 1 / (phi_o[i+1] - phi_o[i])
    double *mcf = ipo + nfp + 1;                               // nmu * 4 mu-interval coefficients
    int16_t *pbk = (int16_t *)(mcf + 4 * nmu);                 // 2 nfp phase buckets
    int16_t *mbk = pbk + 2 * nfp;                              // mu_nb mu buckets
    float *etau = (float *)(mbk + ((S.mu_nb + 1) & ~1));       // E + 1 bucket offsets of the energies
    const int n_pb = 2 * nfp;
    const double4 *tg = tangent + slot * (size_t)(nfp + 1) * 5;   // read through the caches in stage C
    const float2 *tab2 = subtg + slot * (size_t)S.sub_stride;      // logT / log g planes, read through L2
    {
        const double4 *gtr = trace + slot * (nfp + 1);
        for (int i = threadIdx.x; i <= nfp; i += blockDim.x) {
            const double4 v = gtr[i];
            // (F, z, x position of E_0 at z, mu); phi_o in po
            tr[i] = make_double4(v.x, v.y, log10(v.y) * S.ihx + g.tbk, v.w);
            po[i] = v.z;
        }
        for (int i = threadIdx.x; i < nmu; i += blockDim.x) axmu[i] = S.ax_mu[i];
        for (int i = threadIdx.x; i < 4 * nmu; i += blockDim.x) mcf[i] = S.mu_coef[i];
        for (int i = threadIdx.x; i < S.mu_nb; i += blockDim.x) mbk[i] = S.mu_bucket[i];
        for (int i = threadIdx.x; i <= E; i += blockDim.x) etau[i] = S.etau[i];
        const float4 *gs = (const float4 *)(sub + slot * (size_t)S.sub_stride);
        float4 *ts = (float4 *)tab;
        for (int i = threadIdx.x; i < S.sub_stride / 4; i += blockDim.x) ts[i] = gs[i];
    }
    __syncthreads();
    // phase buckets and inverse spacings of phi_o, as in the forward kernel
    for (int q = threadIdx.x; q < n_pb; q += blockDim.x) {
        const double edge = po[0] + (double)q / n_pb;
        int l0 = 0, h0 = nfp;
        while (h0 - l0 > 1) {
            int mid = (l0 + h0) >> 1;
            if (po[mid] <= edge) l0 = mid; else h0 = mid;
        }
        pbk[q] = (int16_t)l0;
    }
    for (int i = threadIdx.x; i < nfp; i += blockDim.x) ipo[i] = 1.0 / (po[i + 1] - po[i]);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float4 *Lw = Lb + wave * E;
    float4 *Pw = Pb + wave * 64;
    const int bp32 = (lane ^ 32) << 2;                     // byte address of the xor-32 partner
    const RingTan rt = ringtan[slot];
    const double phio0 = trace[slot * (nfp + 1)].z;        // phi_o of sample 0
    const double inv2pi = 1.0 / kTwoPi;
    const double ihx = S.ihx;
    const int est = S.ebkt[lane], een = S.ebkt[lane + 1], e_it = S.e_it;   // lane's energy bucket
    const double mu_lo = S.mu_lo, mu_hi = S.mu_hi;
    const int xw0 = g.xw0, xw = g.xw;
    double U[kGradAcc];
#pragma unroll
    for (int q = 0; q < kGradAcc; ++q) U[q] = 0.0;
    double accT = 0.0, accG = 0.0;   // lane-local F_p-weighted logT / log g sums
    const int k_begin = tile * PT;
    for (int kk = wave; kk < PT; kk += kAdjWaves) {
        const int k = k_begin + kk;
        if (k >= P) break;
        // per-bucket inclusive prefix sums of G (1, tau, tau^2, tau^3) for this
        // phase: G staged by energy, then lane = bucket
        {
            const float *gk = gtil + ((size_t)b * P + k) * E;
            wave_sync();                                   // the previous phase's sums are no longer read
            for (int e = lane; e < E; e += 64) ((float *)(Lw + e))[0] = gk[e];
            wave_sync();
            float4 run = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int e = est; e < een; ++e) {
                const float G = ((const float *)(Lw + e))[0], t = etau[e];
                const float g1 = G * t, g2 = g1 * t;
                run.x += G;
                run.y += g1;
                run.z += g2;
                run.w += g2 * t;
                Lw[e] = run;
            }
            wave_sync();
        }
        const double Phik = (k + 0.5) / S.Pd;
        for (int c0 = 0; c0 < g.n_cells; c0 += 64) {
            // ---------------- stage A: one (cell, phase) pair per lane
            const int j = c0 + lane;
            bool vis = false, mu_clamped = false;
            float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, fr = 0.f;
            int I0 = 0, m0 = 0, lo = 0;
            double wph = 0.0;
            float Fpf = 0.f;
            if (j < g.n_cells) {
                const double off = cell_offset(g, j);
                if (!cell_masked(g, off)) {
                    double a = Phik + (g.phi_spot + off) * inv2pi + 1.0 - phio0;
                    double php = (a - floor(a)) + phio0;                    // Eq. (45)
                    int q = (int)((php - phio0) * S.fpb);                  // bucket, bounded scan
                    int l0 = pbk[q < n_pb - 1 ? q : n_pb - 1];
                    while (l0 > 0 && po[l0] > php) --l0;
                    while (l0 < nfp - 1 && po[l0 + 1] <= php) ++l0;
                    const double4 A = tr[l0], Cn = tr[l0 + 1];
                    double w = (php - po[l0]) * ipo[l0];
                    w = fmin(1.0, fmax(0.0, w));
                    const double Fp = A.x + w * (Cn.x - A.x);                // Eq. (46)
                    if (Fp != 0.0) {
                        vis = true;
                        lo = l0;
                        wph = w;
                        Fpf = (float)Fp;
                        const double zp = A.y + w * (Cn.y - A.y);
                        const double mup = A.w + w * (Cn.w - A.w);
                        mu_clamped = !(mup > mu_lo && mup < mu_hi);
                        const double mu = fmin(mu_hi, fmax(mu_lo, mup));
                        int qm = (int)((mu - mu_lo) * S.mu_ibw);               // bucket, bounded scan
                        int ml = mbk[qm < S.mu_nb - 1 ? qm : S.mu_nb - 1];
                        while (ml > 0 && axmu[ml] > mu) --ml;
                        while (ml < nmu - 2 && axmu[ml + 1] <= mu) ++ml;
                        const double *cf = mcf + 4 * ml;
                        double wa, wb, wc, wd, da, db, dc, dd;
                        if (ml < 3 || ml == nmu - 2) {
                            // linear on [a_ml, a_ml+1]; node ml at slot ml - m0 of 0..2
                            const double ih = cf[0];
                            const double t = (mu - axmu[ml]) * ih;
                            m0 = ml < nmu - 4 ? ml : nmu - 4;
                            const int sl = ml - m0;
                            wa = sl == 0 ? 1.0 - t : 0.0;
                            wb = sl == 0 ? t : (sl == 1 ? 1.0 - t : 0.0);
                            wc = sl == 1 ? t : (sl == 2 ? 1.0 - t : 0.0);
                            wd = sl == 2 ? t : 0.0;
                            da = sl == 0 ? -ih : 0.0;
                            db = sl == 0 ? ih : (sl == 1 ? -ih : 0.0);
                            dc = sl == 1 ? ih : (sl == 2 ? -ih : 0.0);
                            dd = sl == 2 ? ih : 0.0;
                        } else {
                            // cubic Lagrange on nodes ml-1 .. ml+2 and its mu derivative
                            m0 = ml - 1;
                            const double d0 = mu - axmu[m0], d1 = mu - axmu[m0 + 1], d2 = mu - axmu[m0 + 2],
                                         d3 = mu - axmu[m0 + 3];
                            const double p01 = d0 * d1, p23 = d2 * d3, s01 = d0 + d1, s23 = d2 + d3;
                            wa = d1 * p23 * cf[0];
                            wb = d0 * p23 * cf[1];
                            wc = p01 * d3 * cf[2];
                            wd = p01 * d2 * cf[3];
                            da = (p23 + d1 * s23) * cf[0];
                            db = (p23 + d0 * s23) * cf[1];
                            dc = (p01 + d3 * s01) * cf[2];
                            dd = (p01 + d2 * s01) * cf[3];
                        }
                        if (mu_clamped) da = db = dc = dd = 0.0;
                        w0 = (float)wa; w1 = (float)wb; w2 = (float)wc; w3 = (float)wd;
                        v0 = (float)da; v1 = (float)db; v2 = (float)dc; v3 = (float)dd;
                        // x position at zp = z_A (1 + t): sample position plus the shift
                        const double T0 = A.z + (double)x_shift(w * (Cn.y - A.y) * rcp_nr(A.y), S.ixl);
                        const double fl = floor(T0);
                        I0 = (int)fl;
                        fr = (float)(T0 - fl);
                    }
                }
            }
            const uint64_t vmask = __ballot(vis);
            // ---------------- stage B: the visible pairs one after another
            float R0 = 0.f, R1 = 0.f, R2 = 0.f;
            const float vv[4] = {v0, v1, v2, v3};
            Pw[lane] = make_float4(w0, w1, w2, w3);
            wave_sync();
            if (g.interior)
                adj_pairs<true>(vmask, Pw, vv, fr, Fpf, I0, m0, lane, bp32, tab, tab2, W, xw0, xw, nx, Lw, etau, est,
                                een, e_it, R0, R1, R2, accT, accG);
            else
                adj_pairs<false>(vmask, Pw, vv, fr, Fpf, I0, m0, lane, bp32, tab, tab2, W, xw0, xw, nx, Lw, etau, est,
                                 een, e_it, R0, R1, R2, accT, accG);
            // ---------------- stage C: chain rule per pair, FP64
            if (vis) {
                const double4 A = tr[lo], Cn = tr[lo + 1];
                const double dph = po[lo + 1] - po[lo];
                const double w = wph;
                const double Fp = A.x + w * (Cn.x - A.x), zp = A.y + w * (Cn.y - A.y);
                const double S0 = R0, Sx = (double)R1 * ihx, Sm = R2;
                const double cF = S0, cz = Fp * Sx / (zp * kLn10), cm = mu_clamped ? 0.0 : Fp * Sm;
                const double dFd = Cn.x - A.x, dzd = Cn.y - A.y, dmd = Cn.w - A.w;
                double ca, cb;
                offset_coeffs(g, j, ca, cb);
#pragma unroll
                for (int d = 0; d < 5; ++d) {
                    const double4 t0 = tg[lo * 5 + d], t1 = tg[(lo + 1) * 5 + d];
                    const double dphp = (ca * rt.ddout[d] + cb * rt.ddin[d]) * inv2pi;
                    const double ww = (dphp - t0.z - w * (t1.z - t0.z)) / dph;
                    const double dF = t0.x + w * (t1.x - t0.x) + dFd * ww;
                    const double dz = t0.y + w * (t1.y - t0.y) + dzd * ww;
                    const double dm = t0.w + w * (t1.w - t0.w) + dmd * ww;
                    U[d] += cF * dF + cz * dz + cm * dm;
                }
                U[5] -= (cF * dFd + cz * dzd + cm * dmd) / dph;     // d php / d Phi = -1
                U[6] += Fp * S0;
                U[8] += Fp * (3.0 * kLn10 * S0 - Sx);
            }
        }
    }
    U[7] += accG;
    U[8] += accT;
    // fixed-order block reduction of the nine sums
    __shared__ double red[kAdjWaves][kGradAcc];
#pragma unroll
    for (int q = 0; q < kGradAcc; ++q) {
        const double v = wave_sum_d(U[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kGradAcc) {
        const int q = threadIdx.x;
        double v = 0.0;
        for (int w8 = 0; w8 < kAdjWaves; ++w8) v += red[w8][q];
        gpart[(slot * n_tile + tile) * kGradAcc + q] = v;
    }
}

// ---------------------------------------------------------------------------
// k_grad_final: per instance, the ring sums times the ring constants and
// ring-level tangents, in a fixed ring order, plus the N_H term.
// Gradient order: M, R_e, i, Phi, N_H, theta_1, zeta_1, logT_1, theta_2,
// zeta_2, logT_2, dphi_2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_grad_final(DevSpec S, const StarRec *stars, const RingRec *rings,
                                                   const RingTan *ringtan, const double *gpart, int n_tile,
                                                   const double *nh_part, double *grad)
{
    const int b = blockIdx.x;
    __shared__ double red[64][PPM_NGRAD];
    double acc[PPM_NGRAD];
#pragma unroll
    for (int q = 0; q < PPM_NGRAD; ++q) acc[q] = 0.0;
    for (int r = threadIdx.x; r < S.R_tot; r += blockDim.x) {
        const size_t slot = (size_t)b * S.R_tot + r;
        const RingRec g = rings[slot];
        if (!g.active) continue;
        const RingTan rt = ringtan[slot];
        double U[kGradAcc];
        for (int q = 0; q < kGradAcc; ++q) U[q] = 0.0;
        for (int t = 0; t < n_tile; ++t)
            for (int q = 0; q < kGradAcc; ++q) U[q] += gpart[(slot * n_tile + t) * kGradAcc + q];
        const double T3 = g.T * g.T * g.T, c = g.w_cell * T3;
        const int s = g.spot;
        for (int d = 0; d < 5; ++d) {
            const double v = c * (U[d] + U[7] * rt.dlogg[d]) + T3 * U[6] * rt.dw[d];
            const int idx = d < 3 ? d : (d == 3 ? 5 + 3 * s : 6 + 3 * s);
            acc[idx] += v;
        }
        acc[3] += c * U[5];
        if (s == 1) acc[11] += c * U[5];
        acc[7 + 3 * s] += c * U[8];
    }
    for (int q = 0; q < PPM_NGRAD; ++q) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < PPM_NGRAD) {
        const int q = threadIdx.x;
        double v = 0.0;
        for (int t = 0; t < 64; ++t) v += red[t][q];
        if (q == 4) {
            const int n = S.P * ((S.E + 15) / 16);   // per (phase, energy tile), in order
            for (int i = 0; i < n; ++i) v += nh_part[(size_t)b * n + i];
        }
        if (stars[b].status != PPM_INST_OK) v = NAN;
        grad[(size_t)b * PPM_NGRAD + q] = v;
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (host)
// ---------------------------------------------------------------------------
size_t accum_adj_lds(const DevSpec &S)
{
    return sizeof(double4) * (S.n_fp + 1) + sizeof(double) * ((S.nmu + 1) & ~1)
         + sizeof(float) * S.sub_stride + sizeof(float4) * kAdjWaves * 64
         + sizeof(float4) * kAdjWaves * S.E + sizeof(double) * 2 * (S.n_fp + 1) + sizeof(double) * 4 * S.nmu
         + sizeof(int16_t) * (2 * S.n_fp + ((S.mu_nb + 1) & ~1)) + sizeof(float) * (S.E + 1);
}

hipError_t launch_grad(const DevSpec &S, const Workspace &W, const double *params, const int32_t *ncells_dev,
                       int B, const int32_t *list, int n_list, const double *counts, const int32_t *data,
                       double *grad, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold_bwd, dim3((S.E + 15) / 16, (B * S.P + 15) / 16), dim3(256), 0, st, S, W.stars, counts,
                       data, W.flux, W.gtil, W.nh_part, B * S.P);
    hipLaunchKernelGGL(k_table_u, dim3(n_list, (S.n_alpha + 63) / 64), dim3(64), 0, st, S, list, W.stars, W.rings,
                       W.table_u);
    size_t lds_tt = sizeof(double4) * (2 * S.n_alpha + (S.n_fp + 1) * 5);
    hipLaunchKernelGGL(k_trace_tan, dim3(n_list), dim3(256), lds_tt, st, S, list, params, ncells_dev, W.stars,
                       W.rings, W.table, W.table_u, W.trace, W.tangent, W.ringtan);
    hipLaunchKernelGGL(k_subtable_tg, dim3(n_list), dim3(256), 0, st, S, list, W.rings, W.subtg);
    const int n_tile = (S.P + S.pt_adj - 1) / S.pt_adj;
    size_t lds = accum_adj_lds(S);
    const int step = max_list_per_launch(n_tile, 64 * kAdjWaves);
    for (int off = 0; off < n_list; off += step) {
        const int32_t *sl = list + off;
        const int n = n_list - off < step ? n_list - off : step;
        hipLaunchKernelGGL(k_accum_adj, dim3(xcd_grid(n, n_tile)), dim3(64 * kAdjWaves), lds, st, S, sl, W.rings,
                           W.ringtan, W.trace, W.tangent, W.sub, W.subtg, W.gtil, W.gpart, n);
    }
    hipLaunchKernelGGL(k_grad_final, dim3(B), dim3(64), 0, st, S, W.stars, W.rings, W.ringtan, W.gpart, n_tile,
                       W.nh_part, grad);
    return hipGetLastError();
}

}  // namespace ppm
