// gfx950 kernels of the pulse-profile forward model and Poisson likelihood.
//
// Pipeline of one evaluation (all instances of a batch at once):
//   k_setup      FP64 star and ring records, parameter validation
//   k_table      FP64 per-ring deflection / delay table on alpha nodes
//   k_trace      FP64 pseudo-patch fine-phase trace with invisible fill, then
//                the per-ring (logT, log g) collapse of the atmosphere table
//   k_accum_*    shift-and-add intensity accumulation (the hot loop)
//   k_reduce     deterministic sum over rings, absorption
//   k_fold_*     response fold on the matrix cores (MFMA)
//   k_loglike    Poisson log-likelihood, FP64
// Section and equation numbers refer to arXiv:2510.07764.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ppm_internal.h"
#include "ppm_device.h"
#include "ppm_launch.h"
#include "../../include/ppm.h"

namespace ppm {

constexpr int kTableSplit = 2;     // lanes per deflection-table node in k_table
constexpr int kTraceThreads = 512; // threads per ring block of k_trace

// ---------------------------------------------------------------------------
// parameter validation (host and device share these rules)
// ---------------------------------------------------------------------------
__host__ __device__ int validate_params(const double *p, int n_spots)
{
    const int used[14] = {0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 13, 14, 15};
    int nused = n_spots > 1 ? 14 : 10;
    for (int i = 0; i < nused; ++i)
        if (!isfinite(p[used[i]])) return PPM_INST_NONFINITE;
    if (p[0] <= 0.0 || p[1] <= 0.0 || p[6] <= 0.0 || p[5] < 0.0 || p[4] < 0.0) return PPM_INST_BAD_STAR;
    double GM = p[0] * kGMsun, Re = p[1] * 1e5;
    double Rs = 2.0 * GM / (kC * kC);
    if (Re <= 1.5 * Rs) return PPM_INST_BAD_STAR;
    if (GM / (kC * kC * Re) > 0.28 * (1.0 + 1e-12)) return PPM_INST_COMPACT;   // inclusive limit
    for (int s = 0; s < n_spots; ++s) {
        double th = p[8 + 4 * s], z = p[9 + 4 * s];
        if (th < 0.0 || th > kPi || z <= 0.0 || z > kPi) return PPM_INST_BAD_SPOT;
    }
    double beta_eq = kTwoPi * p[5] * Re / (kC * sqrt(1.0 - Rs / Re));
    if (beta_eq >= 0.6) return PPM_INST_FAST_SPIN;
    return PPM_INST_OK;
}

// ---------------------------------------------------------------------------
// k_setup: star (Eqs. 7, 8, 11) and spot rings (Eqs. 2, 3, 9, 10, 18), or
// for a temperature-map plan the HEALPix rings of the whole surface
// (Sect. 2.8.1; patch solid angle pi / (3 n_side^2))
// ---------------------------------------------------------------------------
__device__ inline StarRec make_star(const DevSpec &S, const double *p)
{
    StarRec s;
    s.status = validate_params(p, S.n_side > 0 ? 0 : S.n_spots);
    s.GM = p[0] * kGMsun;
    s.Re = p[1] * 1e5;
    s.Rs = 2.0 * s.GM / (kC * kC);
    s.x = s.GM / (kC * kC * s.Re);
    s.Obar = kTwoPi * p[5] * sqrt(s.Re * s.Re * s.Re / s.GM);
    s.o2 = (S.mode == PPM_MODE_OS) ? s.Obar * s.Obar * (-0.788 + 1.030 * s.x) : 0.0;
    s.g0 = s.GM / (s.Re * s.Re) / sqrt(1.0 - s.Rs / s.Re);
    s.D = p[6] * kPc;
    s.nu = p[5];
    s.si = sin(p[2]);
    s.ci = cos(p[2]);
    s.NH = p[4] * 1e20;
    s.pad = 0;
    return s;
}

// Block = 64 rings, eight waves; lane = ring.  The waves share a ring's
// transcendental work, two on each SIMD, so that no chain of FP64
// transcendentals is longer than it must be: wave 0 the shape and velocity
// chain (Eqs. 2, 3, 7, 18), wave 1 the outer arc half-width, wave 2 the inner
// one and the cosine of the mask radius, wave 3 the colatitude band and the
// surface gravity (Eqs. 10, 11), wave 4 the ray limit alpha_max, wave 5 the
// radial delay of Eq. (16), wave 6 the crescent mask half-width, wave 7 the
// temperature; waves 4 and 5 redo the few steps of wave 0 they start from
// (the same operations, so the same values).  Wave 0 takes the others'
// results from LDS and writes the record.  Every thread evaluates the star
// record itself (identical values).
constexpr int kSetupWaves = 8;
__global__ __launch_bounds__(64 * kSetupWaves) void k_setup(DevSpec S, const double *params, const int32_t *n_cells, StarRec *stars,
                        RingRec *rings, int32_t *vis_pairs, int32_t *diag)
{
    const int b = blockIdx.y;
    // the whole parameter vector in registers first: validation and setup
    // then wait for one round of independent loads, not a chain of them
    double p[PPM_NPARAM];
#pragma unroll
    for (int i = 0; i < PPM_NPARAM; ++i) p[i] = params[(size_t)b * PPM_NPARAM + i];
    const StarRec st = make_star(S, p);
    if (blockIdx.x == 0 && threadIdx.x == 0) stars[b] = st;
    const int role = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 64 + lane;
    const int rr = r < S.R_tot ? r : S.R_tot - 1;      // threads past the end mirror the last ring
    const int ncell_override = n_cells ? n_cells[b] : 0;
    const int spot = (rr < S.rings_max[0]) ? 0 : 1;
    const int lr = spot == 0 ? rr : rr - S.rings_max[0];
    const int nr = ncell_override > 0 ? ncell_override : S.n_rings_spec[spot];
    const int np = ncell_override > 0 ? ncell_override : S.n_phi_spec[spot];
    const bool live = st.status == PPM_INST_OK && spot < S.n_spots && lr < nr;
    double tc = p[8 + 4 * spot], z = p[9 + 4 * spot];
    if (!live) { tc = 0.5; z = 0.1; }
    double th, hp_first = 0.0, e0 = 0.0, e1 = 0.0;
    int hp_n = 0;
    if (S.n_side > 0) {
        double zr;
        healpix_ring(S.n_side, rr + 1, zr, hp_n, hp_first);
        th = acos(zr);
    } else {
        double lo = fmax(0.0, tc - z), hi = fmin(kPi, tc + z);
        e0 = lo + (hi - lo) * lr / nr;
        e1 = lo + (hi - lo) * (lr + 1) / nr;
        th = 0.5 * (e0 + e1);
    }
    const int shape = S.shape[spot];
    // results of waves 1-7 per ring: outer, inner half-width, cos(mask radius),
    // cos band difference, log g, T, crescent mask half-width, alpha_max,
    // c dt(R)/R
    __shared__ double xo[9][64];
    RingRec g;
    if (role == 1) {
        xo[0][lane] = arc_halfwidth(th, tc, z);
    } else if (role == 2) {
        xo[1][lane] = (S.n_side == 0 && shape == PPM_SHAPE_ANNULUS) ? arc_halfwidth(th, tc, S.shape_a[spot] * z) : 0.0;
        xo[2][lane] = cos(S.shape_a[spot] * z);
    } else if (role == 3) {
        xo[3][lane] = S.n_side > 0 ? 0.0 : cos(e0) - cos(e1);
        xo[4][lane] = log10(st.g0 * gravity_ratio(st, S.mode, th));   // Eqs. (10), (11)
    } else if (role == 7) {
        xo[5][lane] = pow(10.0, S.n_side > 0 ? 6.0 : p[10 + 4 * spot]);
    } else if (role == 6) {
        xo[6][lane] = 0.0;
        if (S.n_side == 0 && shape == PPM_SHAPE_CRESCENT) {
            const double sgn = (tc >= kHalfPi) ? 1.0 : -1.0;
            xo[6][lane] = arc_halfwidth(th, tc - sgn * S.shape_b[spot] * z, S.shape_a[spot] * z);
        }
    } else if (role == 4) {
        // the largest emission angle: below the cap of rays that reach the
        // observer and at most pi/2 beyond the local vertical
        const double ct = cos(th), sn = sin(th);
        const double R = st.Re * (1.0 + st.o2 * ct * ct);          // Eq. (7)
        const double dR = -2.0 * st.Re * st.o2 * ct * sn;
        const double u = st.Rs / R, sq1u = sqrt(1.0 - u);
        const double f = dR / (R * sq1u);                           // Eq. (2)
        const double v = 1.5 * u * sqrt(3.0 * (1.0 - u));
        const double acap = v >= 1.0 ? kHalfPi : kPi - asin(v);
        double amax = kHalfPi + fabs(atan(f));
        if (amax > acap - 1e-6) amax = acap - 1e-6;
        xo[7][lane] = amax;
    } else if (role == 5) {
        const double ct = cos(th);
        const double R = st.Re * (1.0 + st.o2 * ct * ct);          // Eq. (7)
        xo[8][lane] = cdt_oblate(st.Re, st.Rs, R) / R;
    } else {
        g.spot = spot;
        g.shape = shape;
        g.active = 0;
        g.visible = 0;
        g.inv_min = 0;
        g.inv_max = -1;
        g.interior = 0;
        g.n_cells = 0;
        g.theta = th;
        double ct = cos(th), sn = sin(th);
        g.R = st.Re * (1.0 + st.o2 * ct * ct);                    // Eq. (7)
        double dR = -2.0 * st.Re * st.o2 * ct * sn;
        g.u = st.Rs / g.R;
        g.sq1u = sqrt(1.0 - g.u);
        g.f = dR / (g.R * g.sq1u);                                 // Eq. (2)
        g.coseta = 1.0 / sqrt(1.0 + g.f * g.f);                    // Eq. (3)
        g.sineta = g.f / sqrt(1.0 + g.f * g.f);
        g.beta = kTwoPi * st.nu * g.R * sn / (kC * g.sq1u);        // Eq. (18)
        g.gamma = 1.0 / sqrt(1.0 - g.beta * g.beta);
        g.phi_spot = -kTwoPi * (p[3] + (spot == 1 ? p[15] : 0.0));
        // map rings: per-patch temperatures, 10^6 K is the reference the
        // accumulation scales by
        g.logT = S.n_side > 0 ? 6.0 : p[10 + 4 * spot];
        double sgn = (tc >= kHalfPi) ? 1.0 : -1.0;
        g.tm = tc - sgn * S.shape_b[spot] * z;
    }
    __syncthreads();                                   // waves 1-7 have written their results
    if (role != 0 || r >= S.R_tot) return;
    g.alpha_max = xo[7][lane];
    g.cdt_obl = xo[8][lane];
    g.dcos = xo[3][lane];
    g.logg = xo[4][lane];
    g.dphi_out = xo[0][lane];
    if (S.n_side > 0) {
        // cell j at azimuth first + j * 2 pi / n (cell_offset of a cap ring)
        g.dphi_cell = kTwoPi / hp_n;
        g.dphi_out = 0.5 * g.dphi_cell - hp_first;
        g.dphi_in = 0.0;
    } else if (g.shape == PPM_SHAPE_ANNULUS) {
        g.dphi_in = xo[1][lane];
        g.dphi_cell = (g.dphi_out - g.dphi_in) / (0.5 * np);
    } else {
        g.dphi_in = 0.0;
        g.dphi_cell = 2.0 * g.dphi_out / np;
    }
    const double patch = S.n_side > 0 ? kPi / (3.0 * S.n_side * (double)S.n_side) : g.dcos * g.dphi_cell;
    g.w_cell = g.R * g.R * sqrt(1.0 + g.f * g.f) * patch / (st.D * st.D);  // Eq. (9)
    g.T = xo[5][lane];
    g.kT = kKB * g.T;
    g.cos_zm = xo[2][lane];
    if (live) g.n_cells = S.n_side > 0 ? hp_n : np;
    // a crescent ring whose every cell centre lies inside the mask emits
    // nothing: switched off like a ring outside the spot (with a margin, so
    // that a cell on the mask edge is left to the per-cell test)
    if (g.shape == PPM_SHAPE_CRESCENT && S.n_side == 0 && g.dphi_out - 0.5 * g.dphi_cell < xo[6][lane] - 1e-9)
        g.n_cells = 0;
    const size_t slot = (size_t)b * S.R_tot + r;
    rings[slot] = g;
    vis_pairs[slot] = 0;
    // diagnostics: table clamps of the ring's logT and log g (Sect. 4), the
    // counters of the later kernels start at zero
    int flags = 0;
    if (S.intensity == PPM_I_TABLE) {
        if (S.n_side == 0 && (g.logT < S.T_end[0] || g.logT > S.T_end[1])) flags |= 1;
        if (g.logg < S.g_end[0] || g.logg > S.g_end[1]) flags |= 2;
    }
    int32_t *dg = diag + slot * kDiagFields;
    dg[0] = flags;
#pragma unroll
    for (int i = 1; i < kDiagFields; ++i) dg[i] = 0;
}

// ---------------------------------------------------------------------------
// k_table: FP64 deflection and delay table per ring (Sect. 2.3, 2.8.2).
// Nodes are uniform in alpha on [0, alpha_max]; each stores psi (Eq. 32),
// dpsi/dalpha, the total delay c dt / R (Eqs. 35, 16, 17) and its alpha
// derivative, so that lookups can use C1 cubic Hermite interpolation.
// Quadrature: Gauss-Legendre after x = A sinh(tau), A = cos(a)/(sin(a)
// sqrt(q0)), which resolves the boundary layer of width ~cos(alpha) at
// x -> 0 for near-grazing rays.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 3) void k_table(DevSpec S, const int32_t *list, const StarRec *stars, const RingRec *rings, double4 *table)
{
    const int ent = list[blockIdx.x], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const RingRec g = rings[(size_t)b * S.R_tot + r];
    if (g.n_cells == 0) return;
    // the quadrature rules in LDS: the node loops read them at LDS latency
    __shared__ double sgx[kGLNodes], sgw[kGLNodes];
    for (int i = threadIdx.x; i < kGLNodes; i += blockDim.x) {
        sgx[i] = S.glx[i];
        sgw[i] = S.glw[i];
    }
    __syncthreads();
    const StarRec st = stars[b];
    const double u = g.u;
    const double dal = g.alpha_max / (S.n_alpha - 1);
    double4 *tab = table + ((size_t)b * S.R_tot + r) * S.n_alpha;
    // kTableSplit lanes per node, each summing every kTableSplit-th quadrature
    // node; the lanes' results add up to the node's values
    const int kq = threadIdx.x % kTableSplit;
    const int per_block = blockDim.x / kTableSplit;
    for (int j0 = blockIdx.y * per_block; j0 < S.n_alpha; j0 += gridDim.y * per_block) {
        const int j = j0 + (int)threadIdx.x / kTableSplit;
        double psi = 0.0, dpsi = 0.0, T = 0.0, dT = 0.0;
        if (j < S.n_alpha) {
            double a = dal * j;
            if (j == S.n_alpha - 1) a = g.alpha_max;
            const bool lead = kq == 0;
            // one outgoing-ray quadrature per node: at alpha, or for an inward
            // ray at pi - alpha (its outgoing leg from the periastron)
            const bool inward = a > kHalfPi;
            double psb, dpsb, tpb;
            bend_out(sgx, sgw, u, inward ? kPi - a : a, psb, dpsb, tpb, kq, kTableSplit);
            const double sa = sin(a);
            if (!inward) {
                psi = psb;
                dpsi = dpsb;
                T = tpb + (lead ? g.cdt_obl : 0.0);
                dT = dpsb * sa / g.sq1u;               // d(c dt)/d psi = b (impact parameter)
            } else {
                // inward ray through a periastron at rho R (Eqs. 13, 14, 17)
                double ca = cos(a);
                double kk = sqrt(3.0 * (1.0 - u));
                double arg = 3.0 * u * kk / (2.0 * sa);
                if (arg > 1.0) arg = 1.0;
                double rho = -2.0 * sa / kk * cos((acos(arg) + kTwoPi) / 3.0);
                double k = sa * sa / (1.0 - u), kp = 2.0 * sa * ca / (1.0 - u);
                double rhop = kp * (rho - u) / (3.0 * rho * rho - k);
                double v = u / rho, vp = -u * rhop / (rho * rho);
                double ph, dph, th, dth;
                grazing(sgx, sgw, v, ph, dph, th, dth, kq, kTableSplit);
                psi = 2.0 * ph - psb;
                dpsi = 2.0 * dph * vp + dpsb;
                double Rp = rho * g.R;
                double cdtp = cdt_oblate(st.Re, st.Rs, Rp) / g.R;
                T = 2.0 * rho * th - tpb + (lead ? 2.0 * cdtp - g.cdt_obl : 0.0);
                double dtpb = dpsb * sa / g.sq1u;
                dT = 2.0 * rhop * th + 2.0 * rho * dth * vp + dtpb - (lead ? 2.0 * rhop * rho / (rho - u) : 0.0);
            }
        }
#pragma unroll
        for (int o = 1; o < kTableSplit; o <<= 1) {
            psi += __shfl_xor(psi, o, 64);
            dpsi += __shfl_xor(dpsi, o, 64);
            T += __shfl_xor(T, o, 64);
            dT += __shfl_xor(dT, o, 64);
        }
        if (j < S.n_alpha && kq == 0) tab[j] = make_double4(psi, dpsi, T, dT);
    }
}

// ---------------------------------------------------------------------------
// subtable_ring: linear (logT, log g) collapse of the atmosphere table for one
// ring (run by k_trace once the ring's x window is known) (mixed-order scheme of Sect. 4: linear on these two axes, clamped at
// the edges), giving sub[mu][x] = I/T^3 at the ring's (logT, log g).
// ---------------------------------------------------------------------------
// Four-node Lagrange weights on a uniform axis of n >= 4 nodes at position
// t (node units, clamped to the axis): stencil around the bracketing
// interval, shifted inward at the axis ends.  Returns the first node.
__device__ static inline int cubic_uniform(double t, int n, double w[4])
{
    t = fmin((double)(n - 1), fmax(0.0, t));
    int i = (int)floor(t);
    if (i > n - 2) i = n - 2;
    int s0 = i - 1;
    s0 = s0 < 0 ? 0 : (s0 > n - 4 ? n - 4 : s0);
    const double u = t - s0;
    w[0] = -(u - 1.0) * (u - 2.0) * (u - 3.0) / 6.0;
    w[1] = u * (u - 2.0) * (u - 3.0) / 2.0;
    w[2] = -u * (u - 1.0) * (u - 3.0) / 2.0;
    w[3] = u * (u - 1.0) * (u - 2.0) / 6.0;
    return s0;
}

__device__ static void subtable_ring(const DevSpec &S, const RingRec &g, int xw0, int xw, size_t slot, float *sub)
{
    if (S.interp != PPM_INTERP_MIXED) {
        // strategies (a)-(c): cubic in logT and log g (full x range; generic kernel)
        double wt[4], wg[4];
        const int it = cubic_uniform((g.logT - S.T0) / S.hT, S.nT, wt);
        const int ig = cubic_uniform((g.logg - S.g0) / S.hg, S.ng, wg);
        const size_t slab = (size_t)S.nmu * S.nx;
        float w16[16];
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 4; ++c) w16[4 * a + c] = (float)(wt[a] * wg[c]);
        float *out = sub + slot * slab;
        for (size_t i = threadIdx.x; i < slab; i += blockDim.x) {
            float v = 0.0f;
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 4; ++c)
                    v += w16[4 * a + c] * S.atm[((size_t)(it + a) * S.ng + ig + c) * slab + i];
            out[i] = v;
        }
        return;
    }
    double wt1, wg1;
    int it = lin_bracket(g.logT, S.T0, S.hT, S.nT, wt1);
    int ig = lin_bracket(g.logg, S.g0, S.hg, S.ng, wg1);
    const float w00 = (float)((1.0 - wt1) * (1.0 - wg1)), w01 = (float)((1.0 - wt1) * wg1);
    const float w10 = (float)(wt1 * (1.0 - wg1)), w11 = (float)(wt1 * wg1);
    const size_t slab = (size_t)S.nmu * S.nx;
    const float *s00 = S.atm + ((size_t)it * S.ng + ig) * slab;
    const float *s01 = s00 + slab;
    const float *s10 = S.atm + ((size_t)(it + 1) * S.ng + ig) * slab;
    const float *s11 = s10 + slab;
    if (S.fast) {
        // window [xw0, xw0 + W_max) of every mu row, row stride W_max
        const int W = S.W_max;
        float *out = sub + slot * (size_t)S.sub_stride;
        // four elements per thread per round: sixteen loads in flight together.
        // The loads are unconditional (an element outside the window reads
        // element 0 of the slabs and is multiplied by 0: the table is finite),
        // so that none of them waits behind a branch.
        const int n = S.nmu * W, step = blockDim.x;
        for (int i0 = threadIdx.x; i0 < n; i0 += 4 * step) {
            float a[4][4], keep[4];
            int o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k * step;
                const int m = i / W, c = i - m * W;
                const bool ok = i < n && c < xw;
                o[k] = ok ? m * S.nx + xw0 + c : 0;
                keep[k] = ok ? 1.0f : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                a[k][0] = s00[o[k]];
                a[k][1] = s01[o[k]];
                a[k][2] = s10[o[k]];
                a[k][3] = s11[o[k]];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float v = (w00 * a[k][0] + w01 * a[k][1] + w10 * a[k][2] + w11 * a[k][3]) * keep[k];
                if (i0 + k * step < n) out[i0 + k * step] = v;
            }
        }
        return;
    }
    float *out = sub + slot * slab;
    for (size_t i = threadIdx.x; i < slab; i += blockDim.x)
        out[i] = w00 * s00[i] + w01 * s01[i] + w10 * s10[i] + w11 * s11[i];
}

// ---------------------------------------------------------------------------
// k_trace: pseudo-patch light curve of one ring (Sect. 2.8.3, Eqs. 38-44)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTraceThreads) void k_trace(DevSpec S, const int32_t *list, const StarRec *stars, RingRec *rings, const double4 *table,
                        double4 *trace, float *sub, int32_t *diag)
{
    extern __shared__ double4 lds_tab[];
    const int ent = list[blockIdx.x], b = ent / S.R_tot, r = ent - b * S.R_tot;
    RingRec *gp = rings + (size_t)b * S.R_tot + r;
    const RingRec g = *gp;
    if (g.n_cells == 0) return;
    const StarRec st = stars[b];
    const int na = S.n_alpha, nfp = S.n_fp;
    double4 *tr_lds = lds_tab + na;            // n_fp + 1 entries
    const double4 *tab = table + ((size_t)b * S.R_tot + r) * na;
    for (int j = threadIdx.x; j < na; j += blockDim.x) lds_tab[j] = tab[j];
    __shared__ int imin, imax, n_multi;
    if (threadIdx.x == 0) { imin = nfp; imax = 0; n_multi = 0; }   // invisible-range initialisation of Sect. 2.8.3
    __syncthreads();
    const double psi_top = lds_tab[na - 1].x;
    // Sect. 6: beyond GM/(R c^2) ~ 0.28 a point can be seen along a second
    // ray; a visible sample with psi > 2 pi - psi_top has one (counted; the
    // primary image is kept)
    const bool multi_possible = psi_top > kPi;
    const double dal = g.alpha_max / (na - 1);
    const double sth = sin(g.theta), cth = cos(g.theta);
    for (int i = threadIdx.x; i <= nfp; i += blockDim.x) {
        double phi = kTwoPi * i / nfp;
        double sphi, cphi;
        sincos(phi, &sphi, &cphi);
        double cpsi = st.si * sth * cphi + st.ci * cth;           // Table 2
        cpsi = fmin(1.0, fmax(-1.0, cpsi));
        double psi = acos(cpsi);
        bool vis = psi <= psi_top;
        double F = 0.0, z = 0.0, po = 0.0, mu = 0.0;
        if (vis) {
            double a, sr, lf;
            if (psi < 1e-7) {
                a = psi * g.sq1u;            // sub-observer limit, alpha = psi sqrt(1-u)
                sr = g.sq1u;
                lf = 1.0 - g.u;
            } else {
                int lo = 0, hi = na - 1;
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (lds_tab[mid].x <= psi) lo = mid; else hi = mid;
                }
                double p0 = lds_tab[lo].x, p1 = lds_tab[lo + 1].x;
                double h = p1 - p0;
                double t = (psi - p0) / h;
                double a0 = dal * lo, a1 = dal * (lo + 1);
                if (lo + 1 == na - 1) a1 = g.alpha_max;
                double m0 = 1.0 / lds_tab[lo].y, m1 = 1.0 / lds_tab[lo + 1].y;
                double h00, h10, h01, h11, d00, d10, d01, d11;
                hermite(t, h00, h10, h01, h11);
                dhermite(t, d00, d10, d01, d11);
                a = h00 * a0 + h10 * h * m0 + h01 * a1 + h11 * h * m1;
                double dadpsi = (d00 * a0 + d10 * h * m0 + d01 * a1 + d11 * h * m1) / h;
                sr = sin(a) / sin(psi);
                lf = sr * dadpsi;                  // d cos(alpha) / d cos(psi)
            }
            double ca = cos(a);
            // Eq. (4)
            double cs = ca * g.coseta + sr * g.sineta * (st.ci * sth - st.si * cth * cphi);
            if (cs > 0.0) {
                double cxi = -sr * st.si * sphi;                      // Table 2
                double delta = 1.0 / (g.gamma * (1.0 - g.beta * cxi));  // Eq. (19)
                mu = delta * cs;                                        // Eq. (20)
                F = g.sq1u * delta * delta * delta * mu * lf * g.gamma; // Eq. (40)
                z = 1.0 / (delta * g.sq1u);
                int jj = (int)floor(a / dal);
                jj = jj < 0 ? 0 : (jj > na - 2 ? na - 2 : jj);
                double ta = (a - dal * jj) / dal;
                double h00, h10, h01, h11;
                hermite(ta, h00, h10, h01, h11);
                double T = h00 * lds_tab[jj].z + h10 * dal * lds_tab[jj].w + h01 * lds_tab[jj + 1].z
                         + h11 * dal * lds_tab[jj + 1].w;
                po = phi / kTwoPi + st.nu * g.R * T / kC;
                if (multi_possible && psi > kTwoPi - psi_top) atomicAdd(&n_multi, 1);
            } else {
                vis = false;
            }
        }
        if (!vis) {
            atomicMin(&imin, i);
            atomicMax(&imax, i);
            F = 0.0; z = 0.0; po = 0.0; mu = 0.0;
        }
        tr_lds[i] = make_double4(F, z, po, mu);
    }
    __syncthreads();
    const int a0 = imin, a1 = imax;
    const bool ring_visible = a0 != 0;    // invisible at phi = 0: the ring is skipped
    if (ring_visible && a0 <= a1) {
        // Eqs. (41)-(44): zero flux and mu, linear fill of z and phi_o
        // sample n_fp repeats sample 0, so a visible ring has a1 < n_fp
        const int ia = a0 - 1, ib = a1 + 1 > nfp ? nfp : a1 + 1;
        const double4 va = tr_lds[ia], vb = tr_lds[ib];
        for (int i = a0 + threadIdx.x; i <= a1; i += blockDim.x) {
            double t = (double)(i - ia) / (double)(ib - ia);
            tr_lds[i] = make_double4(0.0, va.y + (vb.y - va.y) * t, va.z + (vb.z - va.z) * t, 0.0);
        }
    }
    __syncthreads();
    double4 *out = trace + ((size_t)b * S.R_tot + r) * (nfp + 1);
    double zlo = 1e300, zhi = 0.0;
    for (int i = threadIdx.x; i <= nfp; i += blockDim.x) {
        double4 v = tr_lds[i];
        out[i] = v;
        if (v.y > 0.0) { zlo = fmin(zlo, v.y); zhi = fmax(zhi, v.y); }
    }
    __shared__ double red_lo[kTraceThreads / 64], red_hi[kTraceThreads / 64];
    __shared__ int sh_active, sh_w0, sh_w;
    // range of z over the block: wave butterflies, then the four waves
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        zlo = fmin(zlo, __shfl_xor(zlo, o, 64));
        zhi = fmax(zhi, __shfl_xor(zhi, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red_lo[threadIdx.x >> 6] = zlo;
        red_hi[threadIdx.x >> 6] = zhi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < (int)(blockDim.x >> 6); ++t) { zlo = fmin(zlo, red_lo[t]); zhi = fmax(zhi, red_hi[t]); }
        diag[((size_t)b * S.R_tot + r) * kDiagFields + 1] = n_multi;
        gp->visible = ring_visible ? 1 : 0;
        gp->inv_min = a0;
        gp->inv_max = a1;
        int active = (ring_visible && g.w_cell > 0.0) ? 1 : 0;
        gp->zmin = zlo;
        gp->zmax = zhi;
        if (active && S.intensity == PPM_I_TABLE && S.n_side == 0) {
            // x nodes any (cell, phase, energy) of this ring can touch, plus the
            // cubic stencil: t = (log10(z E / kT) - x0) / hx
            double lkt = log10(g.kT) / S.hx;
            gp->tbk = S.tb0 - lkt;
            double tlo = log10(zlo) / S.hx + S.tb0 - lkt;
            double thi = log10(zhi) / S.hx + S.tb0 + S.r_span - lkt;
            int w0 = (int)floor(tlo) - 2, w1 = (int)floor(thi) + 3;
            w0 = w0 < 0 ? 0 : w0;
            w1 = w1 > S.nx - 1 ? S.nx - 1 : w1;
            int w = w1 - w0 + 1;
            if (w < 1) { w0 = 0; w = 1; }
            if (w > S.W_max) w = S.W_max;   // cannot happen for surface speeds below 0.6 c
            gp->xw0 = w0;
            gp->xw = w;
            // every interval used lies in [floor(tlo), floor(thi)], up to one interval
            // of slip from the rounding of a pair's x position: clear of the axis ends
            // with that margin, every interval is cubic and every column in the window
            gp->interior = (floor(tlo) >= 2.0 && floor(thi) <= S.nx - 4) ? 1 : 0;
        } else {
            gp->xw0 = 0;
            gp->xw = 0;
            gp->interior = 0;
        }
        gp->active = active;
        sh_active = active;
        sh_w0 = gp->xw0;
        sh_w = gp->xw;
    }
    __syncthreads();
    // the ring's (logT, log g) collapse of the atmosphere table
    if (sh_active && S.intensity == PPM_I_TABLE && S.n_side == 0)
        subtable_ring(S, g, sh_w0, sh_w, (size_t)b * S.R_tot + r, sub);
}


// ---------------------------------------------------------------------------
// k_accum_table: shift-and-add with the mixed-order atmosphere table
// (Eq. 47).  Block = (ring, tile of phases); wave = one phase at a time;
// lane = EPL consecutive energies (FP32 accumulators in registers).
// Per (cell, phase): FP64 phase lookup, mu weights (cubic Lagrange, linear
// in the protected small-mu zone and the last interval), contraction of the
// ring's sub-table over mu into S[x] in LDS; per energy: x = log10(z E / kT),
// cubic Lagrange in x (linear in the first and last interval, zero outside).
// ---------------------------------------------------------------------------
// The partial of work-list entry li goes to partial[li] (groups of one ring).
template <int EPL>
__global__ __launch_bounds__(256) void k_accum_table(DevSpec S, const int32_t *list, const RingRec *rings,
                                                     const double4 *trace, const float *sub,
                                                     float *partial, int32_t *vis_pairs, int32_t *diag, int PT,
                                                     int n_list)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int li, tile;
    if (!xcd_block(n_list, (S.P + PT - 1) / PT, li, tile)) return;
    const int ent = list[li], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const RingRec g = rings[(size_t)b * S.R_tot + r];
    if (!g.active) return;
    const int nfp = S.n_fp, nmu = S.nmu, nx = S.nx, E = S.E, P = S.P;
    double4 *tr = (double4 *)lds_raw;                          // nfp + 1
    double *axmu = (double *)(tr + nfp + 1);                   // nmu
    float *tab = (float *)(axmu + nmu);                        // nmu * nx
    float *Sb = tab + nmu * nx;                                // 4 waves * nx
    const double4 *gtr = trace + ((size_t)b * S.R_tot + r) * (nfp + 1);
    for (int i = threadIdx.x; i <= nfp; i += blockDim.x) tr[i] = gtr[i];
    for (int i = threadIdx.x; i < nmu; i += blockDim.x) axmu[i] = S.ax_mu[i];
    const float *gsub = sub + ((size_t)b * S.R_tot + r) * nmu * nx;
    for (int i = threadIdx.x; i < nmu * nx; i += blockDim.x) tab[i] = gsub[i];
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *Sw = Sb + wave * nx;
    const double phio0 = tr[0].z;
    const double inv2pi = 1.0 / kTwoPi;
    const double lkT = log10(g.kT);
    double tb[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
        int e = lane * EPL + m;
        tb[m] = e < E ? (log10(S.energy[e]) - lkT - S.x0) / S.hx : 0.0;
    }
    const double mu_lo = axmu[0], mu_hi = axmu[nmu - 1];
    int npairs = 0, nxout = 0, nneg = 0;
    const int k_begin = tile * PT;
    for (int kk = wave; kk < PT; kk += 4) {
        const int k = k_begin + kk;
        if (k >= P) break;
        float acc[EPL];
#pragma unroll
        for (int m = 0; m < EPL; ++m) acc[m] = 0.0f;
        const double Phik = (k + 0.5) / P;
        for (int j = 0; j < g.n_cells; ++j) {
            const double off = cell_offset(g, j);
            if (cell_masked(g, off)) continue;
            double a = Phik + (g.phi_spot + off) * inv2pi + 1.0 - phio0;
            double php = (a - floor(a)) + phio0;                       // Eq. (45)
            PhaseSample ps = phase_lookup(tr, nfp, php);               // Eq. (46)
            if (ps.F == 0.0) continue;
            ++npairs;
            // mu weights
            double mu = fmin(mu_hi, fmax(mu_lo, ps.mu));
            int lo = 0, hi = nmu - 1;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (axmu[mid] <= mu) lo = mid; else hi = mid;
            }
            float wm[4];
            int m0;
            const bool lin_mu = S.interp == PPM_INTERP_MIXED ? (lo < 3 || lo == nmu - 2)
                              : (S.interp == PPM_INTERP_CUBIC_LINMU && lo < 3);
            if (lin_mu) {
                double t = (mu - axmu[lo]) / (axmu[lo + 1] - axmu[lo]);
                m0 = lo;
                wm[0] = (float)(1.0 - t); wm[1] = (float)t; wm[2] = 0.0f; wm[3] = 0.0f;
            } else {
                m0 = lo - 1;
                m0 = m0 < 0 ? 0 : (m0 > nmu - 4 ? nmu - 4 : m0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double num = 1.0, den = 1.0;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        if (s == q) continue;
                        num *= mu - axmu[m0 + s];
                        den *= axmu[m0 + q] - axmu[m0 + s];
                    }
                    wm[q] = (float)(num / den);
                }
            }
            const int nrow = lin_mu ? 2 : 4;
            const float *t0 = tab + m0 * nx;
            for (int n = lane; n < nx; n += 64) {
                float s = wm[0] * t0[n] + wm[1] * t0[nx + n];
                if (nrow == 4) s += wm[2] * t0[2 * nx + n] + wm[3] * t0[3 * nx + n];
                Sw[n] = s;
            }
            wave_sync();
            const double tz = log10(ps.z) / S.hx;
            const float Fp = (float)ps.F;
#pragma unroll
            for (int m = 0; m < EPL; ++m) {
                double t = tz + tb[m];
                if (lane * EPL + m >= E) continue;
                if (t < 0.0 || t > nx - 1) {      // x outside the table: no contribution (counted)
                    ++nxout;
                    continue;
                }
                int i = (int)floor(t);
                if (i > nx - 2) i = nx - 2;
                float f = (float)(t - i);
                float I;
                if (S.interp != PPM_INTERP_MIXED && (i == 0 || i == nx - 2)) {
                    // cubic stencil shifted inward at the axis end
                    const int s0 = i == 0 ? 0 : nx - 4;
                    const float u = (float)(t - s0);
                    const float a0 = -(u - 1.0f) * (u - 2.0f) * (u - 3.0f) * (1.0f / 6.0f);
                    const float a1 = u * (u - 2.0f) * (u - 3.0f) * 0.5f;
                    const float a2 = -u * (u - 1.0f) * (u - 3.0f) * 0.5f;
                    const float a3 = u * (u - 1.0f) * (u - 2.0f) * (1.0f / 6.0f);
                    I = a0 * Sw[s0] + a1 * Sw[s0 + 1] + a2 * Sw[s0 + 2] + a3 * Sw[s0 + 3];
                } else if (i == 0 || i == nx - 2) {
                    I = Sw[i] + f * (Sw[i + 1] - Sw[i]);
                } else {
                    float fm1 = f - 1.0f, fm2 = f - 2.0f, fp1 = f + 1.0f;
                    float w0 = -f * fm1 * fm2 * (1.0f / 6.0f);
                    float w1 = fp1 * fm1 * fm2 * 0.5f;
                    float w2 = -fp1 * f * fm2 * 0.5f;
                    float w3 = fp1 * f * fm1 * (1.0f / 6.0f);
                    I = w0 * Sw[i - 1] + w1 * Sw[i] + w2 * Sw[i + 1] + w3 * Sw[i + 2];
                }
                nneg += I < 0.0f;
                if (S.interp == PPM_INTERP_CUBIC_CLIP) I = fmaxf(0.0f, I);
                acc[m] += Fp * I;
            }
            wave_sync();
        }
        const double scale = g.w_cell * g.T * g.T * g.T;
        float *out = partial + ((size_t)li * P + k) * E;
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            int e = lane * EPL + m;
            if (e < E) out[e] = (float)(acc[m] * (scale / S.energy[e]));
        }
    }
    const size_t slot = (size_t)b * S.R_tot + r;
    if (lane == 0 && npairs) atomicAdd(&vis_pairs[slot], npairs);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nxout += __shfl_xor(nxout, o, 64);
        nneg += __shfl_xor(nneg, o, 64);
    }
    if (lane == 0 && nxout) atomicAdd(&diag[slot * kDiagFields + 2], nxout);
    if (lane == 0 && nneg) atomicAdd(&diag[slot * kDiagFields + 3], nneg);
}


// ---------------------------------------------------------------------------
// k_accum_fast: shift-and-add with the mixed-order atmosphere table (Eq. 47),
// windowed formulation.  Block = (ring, tile of PT phases), NW waves; a wave
// owns one phase at a time and EPL energies per lane, 64 apart (FP32
// accumulators in registers, fixed summation order over cells; neighbouring
// lanes then read neighbouring or equal interval quads, which keeps the quad
// reads free of LDS bank conflicts).
//  stage A  lane = cell: FP64 observed-phase lookup (Eqs. 45-46), mu
//           weights (cubic Lagrange; linear in the protected small-mu zone
//           and the last interval) pre-scaled by F_p, and the x position
//           T0 = (log10(z_p E_0 / kT) - x0)/hx split into I0 = floor(T0) and
//           frac0; visible pairs are compacted with a wave ballot;
//  stage B  per visible pair: lane = x node I0 - 1 + lane, mu contraction of
//           the ring's LDS sub-table; lane = x interval I0 + lane (the next
//           three nodes' values by DPP whole-wave shifts), cubic
//           coefficients of the interpolant on that interval (linear in the
//           first and last interval of the table, zero outside) into an LDS
//           quad; per energy, t = frac0 + (tb_e - tb_0), one quad read and a
//           three-FMA Horner step.
// The polynomial form equals the cubic Lagrange interpolant of the oracle
// on each interval; the energy window of one pair spans at most 61
// intervals (checked at plan creation).
// ---------------------------------------------------------------------------

// Stage B of k_accum_fast for rings whose x window stays clear of the first
// and last table interval: every interval is cubic, no selects.
template <int EPL>
__device__ __forceinline__ void pairs_interior(uint64_t mask, const float4 *Pp, float fr, int pk, int lane, const float *tab,
                                               int W, int NMP, int xw0, float4 *Qw,
                                               const float (&tbr)[EPL], float (&acc)[EPL])
{
    while (mask) {
        const int p = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        // the pair's mu weights, broadcast from its lane's LDS record
        const float4 pw = Pp[p];
        const float pfr = readlane_f(fr, p);
        const float pw0 = pw.x, pw1 = pw.y, pw2 = pw.z, pw3 = pw.w;
        const int ppk = __builtin_amdgcn_readlane(pk, p);
        const int pI0 = ppk >> 8, pm0 = ppk & 255;
        // mu contraction at x node I0 - 1 + lane (columns past the window hold zeros)
        int col = pI0 - 1 + lane - xw0;
        col = col < W - 1 ? col : W - 1;
        // 24-bit multiply-add on byte offsets (full-rate, unlike a 32-bit multiply)
        const float *t0 = (const float *)((const char *)(tab + pm0) + __umul24((unsigned)col, 4u * NMP));
        const float Sv = pw0 * t0[0] + pw1 * t0[1] + pw2 * t0[2] + pw3 * t0[3];
        const float s1 = wave_next_f(Sv), s2 = wave_next_f(s1), s3 = wave_next_f(s2);
        const float c2 = 0.5f * (Sv + s2) - s1;
        const float c3 = (s3 - Sv) * (1.0f / 6.0f) + 0.5f * (s1 - s2);
        Qw[lane] = make_float4(s1, s2 - s1 - c2 - c3, c2, c3);
        wave_sync();
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            const float t = pfr + tbr[m];
            const float f = __builtin_amdgcn_fractf(t);
            const float4 q = Qw[(int)t];
            acc[m] += q.x + f * (q.y + f * (q.z + f * q.w));
        }
        wave_sync();
    }
}

// Stage B for rings that may reach the edge intervals (linear there) or
// leave the table (zero contribution).
template <int EPL>
__device__ __forceinline__ void pairs_general(uint64_t mask, const float4 *Pp, float fr,
                                              int I0, int m0, int lane, const float *tab, int NMP, int xw0, int xw,
                                              int nx, float4 *Qw, const float (&tbr)[EPL],
                                              float (&acc)[EPL])
{
    while (mask) {
        const int p = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const float4 pw = Pp[p];
        const float pfr = readlane_f(fr, p);
        const float pw0 = pw.x, pw1 = pw.y, pw2 = pw.z, pw3 = pw.w;
        const int pI0 = __builtin_amdgcn_readlane(I0, p), pm0 = __builtin_amdgcn_readlane(m0, p);
        const int col = pI0 - 1 + lane - xw0;
        float Sv = 0.0f;
        if (col >= 0 && col < xw) {
            const float *t0 = (const float *)((const char *)(tab + pm0) + __umul24((unsigned)col, 4u * NMP));
            Sv = pw0 * t0[0] + pw1 * t0[1] + pw2 * t0[2] + pw3 * t0[3];
        }
        const float s1 = wave_next_f(Sv), s2 = wave_next_f(s1), s3 = wave_next_f(s2);
        // interpolant on x interval gi = I0 + lane (nodes gi-1 .. gi+2)
        const int gi = pI0 + lane;
        float4 qd = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gi >= 0 && gi <= nx - 2) {
            if (gi == 0 || gi == nx - 2) {
                qd = make_float4(s1, s2 - s1, 0.f, 0.f);
            } else {
                float c2 = 0.5f * (Sv + s2) - s1;
                float c3 = (s3 - Sv) * (1.0f / 6.0f) + 0.5f * (s1 - s2);
                qd = make_float4(s1, s2 - s1 - c2 - c3, c2, c3);
            }
        }
        Qw[lane] = qd;
        wave_sync();
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            const float t = pfr + tbr[m];
            const float f = __builtin_amdgcn_fractf(t);
            const float4 q = Qw[(int)t];
            acc[m] += q.x + f * (q.y + f * (q.z + f * q.w));
        }
        wave_sync();
    }
}

// Block = (group of up to ring_group consecutive work-list rings of one
// instance, tile of PT phases), NW waves.  The rings are processed one after
// another: each is staged to LDS and its phases go to the waves as they
// finish (waves start on phases 0 .. NW-1; each phase is done by one wave in
// a fixed order over cells, so the sums do not depend on the assignment).
// The group's partial spectrum [P][E] is written by its first active ring
// and read, added to and rewritten by the next ones (the block barrier
// between rings orders them), so one FP32 partial per group and phase goes
// out instead of one per ring.
// GRP false: groups of one ring (the ring loop compiles away, and with it
// the registers the loop keeps live).
template <int EPL, int NW, bool GRP>
__global__ __launch_bounds__(64 * NW, NW >= 8 ? 6 : 4) void k_accum_fast(DevSpec S, const int32_t *list,
                                                    const int32_t *glist, const RingRec *rings,
                                                    const double4 *trace, const float *sub, float *partial,
                                                    int32_t *vis_pairs, int32_t *diag, int PT, int n_groups)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int gi, tile;
    if (!xcd_block(n_groups, (S.P + PT - 1) / PT, gi, tile)) return;
    const int g_first = glist[2 * gi], g_count = GRP ? glist[2 * gi + 1] : 1;
    const int nfp = S.n_fp, nmu = S.nmu, nx = S.nx, E = S.E, P = S.P, W = S.W_max;
    double4 *tr = (double4 *)lds_raw;                          // nfp + 1
    double *axmu = (double *)(tr + nfp + 1);                   // nmu (padded to 16 bytes)
    float *tab = (float *)(axmu + ((nmu + 1) & ~1));           // x-major sub-table, 16-byte aligned
    const int NMP = fast_tab_stride(nmu);
    float4 *Qb = (float4 *)(tab + fast_tab_floats(S));         // NW waves * 64 quads
    float4 *Pb = Qb + NW * 64;                                 // NW waves * 64 pair mu weights
    float *hs = (float *)(Pb + NW * 64);                       // NW waves * EPL * 64 first-half partials
    double *po = (double *)(hs + NW * EPL * 64);               // nfp + 1 phi_o, compact for the search
    double *ipo = po + nfp + 1;                                // nfp: 1 / (phi_o[i+1] - phi_o[i])
    double *mcf = ipo + nfp + 1;                               // nmu * 4 mu-interval coefficients
    int16_t *pbk = (int16_t *)(mcf + 4 * nmu);                 // 2 nfp phase buckets
    int16_t *mbk = pbk + 2 * nfp;                              // mu_nb mu buckets
    float *sce = (float *)(mbk + S.mu_nb);                     // E: output scale w_cell T^3 / E_e
    float *tbl = sce + E;                                      // E: the energies' x offsets
    const int n_pb = 2 * nfp;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ int k_next;
    __shared__ int half_done[NW];   // first halves of split phases stored (see the phase loop)
    // ring-independent tables, staged once per block.  Every load of a round
    // is issued (at a clamped, valid index) before the round's LDS writes, so
    // that the tables cost one memory latency, not one per table.
    {
        const int n_st = max(max(4 * nmu, S.mu_nb), E);
        for (int i = threadIdx.x; i < n_st; i += blockDim.x) {
            const double ax = S.ax_mu[i < nmu ? i : 0];
            const double cf = S.mu_coef[i < 4 * nmu ? i : 0];
            const int16_t bk = S.mu_bucket[i < S.mu_nb ? i : 0];
            const float tb = S.tbe[i < E ? i : 0];
            if (i < nmu) axmu[i] = ax;
            if (i < 4 * nmu) mcf[i] = cf;
            if (i < S.mu_nb) mbk[i] = bk;
            if (i < E) tbl[i] = tb;
        }
    }
    float4 *Qw = Qb + wave * 64;
    float4 *Pw = Pb + wave * 64;
    // x offsets of the lane's energies (past E: the last energy's, a valid
    // window position; those sums are never written)
    float tbr[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
        int e = lane + 64 * m;
        tbr[m] = S.tbe[e < E ? e : E - 1];
    }
    const double mu_lo = S.mu_lo, mu_hi = S.mu_hi;
    const double inv2pi = 1.0 / kTwoPi;
    // the tile's phases are interleaved over the ring's rotation (phase tile +
    // n_tile kk for kk < PT), so that every tile of a ring gets a similar mix
    // of phases where much or little of the ring is in view
    const int n_tile = (P + PT - 1) / PT;
    bool first = true;                              // no active ring of the group done yet
    for (int q = 0; q < g_count; ++q) {
        const int ent = list[g_first + q], b = ent / S.R_tot, r = ent - b * S.R_tot;
        const size_t slot = (size_t)b * S.R_tot + r;
        const RingRec g = rings[slot];
        if (!g.active) continue;
        if (!first) __syncthreads();                // the previous ring's LDS tables are no longer read
        const double4 *gtr = trace + slot * (nfp + 1);
        if (threadIdx.x == 0) k_next = NW;
        if (threadIdx.x < NW) half_done[threadIdx.x] = 0;
        // per round of blockDim threads: the output scales of E energies, the
        // LDS trace per fine-phase sample i (F, z_{i+1}/z_i - 1, x position of
        // E_0 at z_i, mu; phi_o in po) and four sub-table quads per thread (the
        // ring's sub-table is [nmu][W] in HBM, per-ring stride a multiple of 4
        // floats, transposed into the x-major LDS layout).  All of a round's
        // loads are issued at clamped, valid indices before its LDS writes.
        {
            const double scale = g.w_cell * g.T * g.T * g.T;
            const float4 *gsub = (const float4 *)(sub + slot * (size_t)S.sub_stride);
            const int nsub = S.sub_stride / 4;
            for (int r0 = 0; r0 < E || r0 <= nfp || 4 * r0 < nsub; r0 += blockDim.x) {
                const int i = r0 + threadIdx.x;
                const int it = i <= nfp ? i : 0;
                const double en = S.energy[i < E ? i : 0];
                const double4 v = gtr[it];
                const double zn = gtr[it < nfp ? it + 1 : it].y;
                float4 sq[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int si = 4 * r0 + threadIdx.x + k * blockDim.x;
                    sq[k] = gsub[si < nsub ? si : 0];
                }
                if (i < E) sce[i] = (float)(scale / en);
                if (i <= nfp) {
                    tr[i] = make_double4(v.x, zn / v.y - 1.0, log10(v.y) * S.ihx + g.tbk, v.w);
                    po[i] = v.z;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int si = 4 * r0 + threadIdx.x + k * blockDim.x;
                    if (si >= nsub) continue;
                    const float vk[4] = {sq[k].x, sq[k].y, sq[k].z, sq[k].w};
                    int m = (4 * si) / W, c = 4 * si - m * W;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (m < nmu) tab[c * NMP + m] = vk[q];
                        if (++c == W) {
                            c = 0;
                            ++m;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // phase buckets: bucket q covers phi_o[0] + [q, q + 1) / (2 nfp) and holds
        // the largest i < nfp with phi_o[i] at or below its lower edge
        for (int qb = threadIdx.x; qb < n_pb; qb += blockDim.x) {
            const double edge = po[0] + (double)qb / n_pb;
            int l0 = 0, h0 = nfp;
            while (h0 - l0 > 1) {
                int mid = (l0 + h0) >> 1;
                if (po[mid] <= edge) l0 = mid; else h0 = mid;
            }
            pbk[qb] = (int16_t)l0;
        }
        for (int i = threadIdx.x; i < nfp; i += blockDim.x) ipo[i] = 1.0 / (po[i + 1] - po[i]);
        __syncthreads();

        const double phio0 = gtr[0].z;                 // phi_o of sample 0 (tr holds x positions)
        const int xw0 = g.xw0, xw = g.xw;
        int npairs = 0, nxout = 0;
        // Work units.  With groups of one ring every phase is summed in two
        // halves, cells [0, H) and [H, n) with H = 64 ceil(n / 128): its
        // partial is S_A w + S_B w, the second half added to the stored first
        // (a ring of at most 64 cells has one part).  Whole phases go to the
        // waves as they finish; the last (phases of the tile mod NW) phases
        // are handed out as halves, the second half of one adding after the
        // first half's store, so that the block's last round is half as long.
        // The sums do not depend on which wave takes which unit.  Groups of
        // several rings (batches, where the tail is shared by more blocks)
        // sum a phase in one part.
        const int pte = min(PT, (P - tile + n_tile - 1) / n_tile);   // phases of this tile
        const int H = 64 * ((g.n_cells + 127) / 128);
        const bool two = !GRP && g.n_cells > H;
        const int n_split = two ? pte % NW : 0;
        const int n_whole = pte - n_split;
        const int n_units = n_whole + 2 * n_split;
        for (int uu = wave; uu < n_units;) {
            int kk = uu, part = 0;                     // part 0: whole phase, 1: first half, 2: second half
            if (uu >= n_whole) {
                kk = n_whole + ((uu - n_whole) >> 1);
                part = 1 + ((uu - n_whole) & 1);
            }
            const int k = tile + n_tile * kk;
            float *out = partial + ((size_t)gi * P + k) * E;
            float acc[EPL];
#pragma unroll
            for (int m = 0; m < EPL; ++m) acc[m] = 0.0f;
            const double Phik = (k + 0.5) / S.Pd;
            const int c_beg = part == 2 ? H : 0, c_end = part == 1 ? H : g.n_cells;
            for (int c0 = c_beg; c0 < c_end; c0 += 64) {
                if (c0 == H && part == 0) {
                    // whole phase: the first half's scaled partial waits in the
                    // wave's LDS slot while the second half is summed
#pragma unroll
                    for (int m = 0; m < EPL; ++m) {
                        int e = lane + 64 * m;
                        hs[(wave * EPL + m) * 64 + lane] = e < E ? acc[m] * sce[e] : 0.0f;
                        acc[m] = 0.0f;
                    }
                }
                // ---------------- stage A: one (cell, phase) pair per lane
                const int j = c0 + lane;
                bool vis = false;
                float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, fr = 0.f;
                int I0 = 0, m0 = 0;
                if (j < g.n_cells) {
                    const double off = cell_offset(g, j);
                    if (!cell_masked(g, off)) {
                        double a = Phik + (g.phi_spot + off) * inv2pi + 1.0 - phio0;
                        double php = (a - floor(a)) + phio0;                    // Eq. (45)
                        // Eq. (46): fine interval [phi_o[l0], phi_o[l0+1]) holding php, from
                        // its bucket and a bounded scan (phi_o increases)
                        int qb = (int)((php - phio0) * S.fpb);
                        int l0 = pbk[qb < n_pb - 1 ? qb : n_pb - 1];
                        while (l0 > 0 && po[l0] > php) --l0;
                        while (l0 < nfp - 1 && po[l0 + 1] <= php) ++l0;
                        const double4 A = tr[l0], Cn = tr[l0 + 1];
                        double wp = (php - po[l0]) * ipo[l0];
                        wp = fmin(1.0, fmax(0.0, wp));
                        PhaseSample ps;
                        ps.F = A.x + wp * (Cn.x - A.x);
                        ps.mu = A.w + wp * (Cn.w - A.w);
                        if (ps.F != 0.0) {
                            vis = true;
                            double mu = fmin(mu_hi, fmax(mu_lo, ps.mu));
                            // mu interval [a_lo, a_lo+1) from its bucket and a bounded scan
                            int qm = (int)((mu - mu_lo) * S.mu_ibw);
                            int lo = mbk[qm < S.mu_nb - 1 ? qm : S.mu_nb - 1];
                            while (lo > 0 && axmu[lo] > mu) --lo;
                            while (lo < nmu - 2 && axmu[lo + 1] <= mu) ++lo;
                            const double *cf = mcf + 4 * lo;
                            double v0, v1, v2, v3;
                            if (lo < 3 || lo == nmu - 2) {
                                // linear on [a_lo, a_lo+1]; node lo sits at slot lo - m0 of 0..2
                                const double t = (mu - axmu[lo]) * cf[0];
                                m0 = lo < nmu - 4 ? lo : nmu - 4;
                                const int sl = lo - m0;
                                v0 = sl == 0 ? 1.0 - t : 0.0;
                                v1 = sl == 0 ? t : (sl == 1 ? 1.0 - t : 0.0);
                                v2 = sl == 1 ? t : (sl == 2 ? 1.0 - t : 0.0);
                                v3 = sl == 2 ? t : 0.0;
                            } else {
                                // cubic Lagrange on nodes lo-1 .. lo+2, inverse denominators cf
                                m0 = lo - 1;
                                const double d0 = mu - axmu[m0], d1 = mu - axmu[m0 + 1], d2 = mu - axmu[m0 + 2],
                                             d3 = mu - axmu[m0 + 3];
                                const double p01 = d0 * d1, p23 = d2 * d3;
                                v0 = d1 * p23 * cf[0];
                                v1 = d0 * p23 * cf[1];
                                v2 = p01 * d3 * cf[2];
                                v3 = p01 * d2 * cf[3];
                            }
                            w0 = (float)(v0 * ps.F);
                            w1 = (float)(v1 * ps.F);
                            w2 = (float)(v2 * ps.F);
                            w3 = (float)(v3 * ps.F);
                            // x position at the interpolated z = z_A (1 + wp q_A)
                            const double T0 = A.z + (double)x_shift(wp * A.y, S.ixl);
                            double fl = floor(T0);
                            I0 = (int)fl;
                            fr = (float)(T0 - fl);
                            // energies beyond the table's x range contribute nothing
                            // (counted; none on a ring whose window is interior)
                            if (!g.interior && (I0 < 0 || (float)I0 + fr + tbl[E - 1] >= (float)(nx - 2)))
                                nxout += x_outside_count(I0, fr, tbl, E, nx);
                        }
                    }
                }
                uint64_t mask = __ballot(vis);
                npairs += __popcll(mask);
                Pw[lane] = make_float4(w0, w1, w2, w3);
                wave_sync();
                // ---------------- stage B: the visible pairs one after another
                if (g.interior)
                    pairs_interior<EPL>(mask, Pw, fr, (I0 << 8) | m0, lane, tab, W, NMP, xw0, Qw, tbr, acc);
                else
                    pairs_general<EPL>(mask, Pw, fr, I0, m0, lane, tab, NMP, xw0, xw, nx, Qw, tbr, acc);
            }
            if (part == 1) {
                // first half of a split phase (groups of one ring: a plain store)
#pragma unroll
                for (int m = 0; m < EPL; ++m) {
                    int e = lane + 64 * m;
                    if (e < E) out[e] = acc[m] * sce[e];
                }
                __builtin_amdgcn_s_waitcnt(0);         // the stores have completed
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane == 0) __hip_atomic_store(&half_done[kk - n_whole], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else if (part == 0 && two) {
                // whole phase in two halves: first half (LDS slot) + second half
#pragma unroll
                for (int m = 0; m < EPL; ++m) {
                    int e = lane + 64 * m;
                    if (e < E) out[e] = hs[(wave * EPL + m) * 64 + lane] + acc[m] * sce[e];
                }
            } else if (part == 2 || (GRP && !first)) {
                if (part == 2) {
                    // the first half was handed out earlier, so its wave is running: a
                    // bounded wait for its store
                    for (int it = 0; it < (1 << 22); ++it) {
                        if (__hip_atomic_load(&half_done[kk - n_whole], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                            break;
                        __builtin_amdgcn_s_sleep(2);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                }
#pragma unroll
                for (int m = 0; m < EPL; ++m) {
                    int e = lane + 64 * m;
                    if (e < E) out[e] += acc[m] * sce[e];
                }
            } else {
#pragma unroll
                for (int m = 0; m < EPL; ++m) {
                    int e = lane + 64 * m;
                    if (e < E) out[e] = acc[m] * sce[e];
                }
            }
            int nk = 0;
            if (lane == 0) nk = atomicAdd(&k_next, 1);
            uu = __builtin_amdgcn_readfirstlane(nk);
        }
        // wave totals of the ring's counters
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) nxout += __shfl_xor(nxout, o, 64);
        if (lane == 0 && npairs) atomicAdd(&vis_pairs[slot], npairs);
        if (lane == 0 && nxout) atomicAdd(&diag[slot * kDiagFields + 2], nxout);
        first = false;
    }
}

// ---------------------------------------------------------------------------
// k_accum_bb: FP64 shift-and-add with the isotropic blackbody of App. C
// ---------------------------------------------------------------------------
template <int EPL>
__global__ __launch_bounds__(256) void k_accum_bb(DevSpec S, const int32_t *list, const RingRec *rings, const double4 *trace,
                                                  double *partial, int32_t *vis_pairs, int PT, int n_list)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int li, tile;
    if (!xcd_block(n_list, (S.P + PT - 1) / PT, li, tile)) return;
    const int ent = list[li], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const RingRec g = rings[(size_t)b * S.R_tot + r];
    if (!g.active) return;
    const int nfp = S.n_fp, E = S.E, P = S.P;
    double4 *tr = (double4 *)lds_raw;
    const double4 *gtr = trace + ((size_t)b * S.R_tot + r) * (nfp + 1);
    for (int i = threadIdx.x; i <= nfp; i += blockDim.x) tr[i] = gtr[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double phio0 = tr[0].z;
    const double inv2pi = 1.0 / kTwoPi;
    const double ikT = 1.0 / g.kT;
    const double pref = 2.0 / (kH * kH * kH * kC * kC);
    double Ee[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
        int e = lane * EPL + m;
        Ee[m] = e < E ? S.energy[e] : 1.0;
    }
    int npairs = 0;
    const int k_begin = tile * PT;
    for (int kk = wave; kk < PT; kk += 4) {
        const int k = k_begin + kk;
        if (k >= P) break;
        double acc[EPL];
#pragma unroll
        for (int m = 0; m < EPL; ++m) acc[m] = 0.0;
        const double Phik = (k + 0.5) / P;
        for (int j = 0; j < g.n_cells; ++j) {
            const double off = cell_offset(g, j);
            if (cell_masked(g, off)) continue;
            double a = Phik + (g.phi_spot + off) * inv2pi + 1.0 - phio0;
            double php = (a - floor(a)) + phio0;
            PhaseSample ps = phase_lookup(tr, nfp, php);
            if (ps.F == 0.0) continue;
            ++npairs;
#pragma unroll
            for (int m = 0; m < EPL; ++m) {
                double Ep = ps.z * Ee[m];
                double I = pref * Ep * Ep * Ep / expm1(Ep * ikT);
                acc[m] += ps.F * I;
            }
        }
        double *out = partial + ((size_t)li * P + k) * E;
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            int e = lane * EPL + m;
            if (e < E) out[e] = acc[m] * g.w_cell / Ee[m];
        }
    }
    if (lane == 0 && npairs) atomicAdd(&vis_pairs[(size_t)b * S.R_tot + r], npairs);
}

// ---------------------------------------------------------------------------
// k_reduce: fixed-order FP64 sum of the ring-group partials of an instance
// (groups grange[b] .. in work-list order), then absorption (Eq. 22) and the
// exposure per phase bin, ready for the fold.  A group none of whose rings
// is active wrote no partial and is skipped.
// ---------------------------------------------------------------------------
__device__ inline void stage_group_flags(const int32_t *list, const int32_t *glist, const RingRec *rings, int g0,
                                         int ng, unsigned char *act)
{
    for (int i = threadIdx.x; i < ng; i += blockDim.x) {
        const int f = glist[2 * (g0 + i)], c = glist[2 * (g0 + i) + 1];
        int a = 0;
        for (int q = 0; q < c; ++q) a |= rings[list[f + q]].active;
        act[i] = (unsigned char)a;
    }
}

template <typename TP, typename TA>
__global__ __launch_bounds__(256) void k_reduce(DevSpec S, const StarRec *stars, const RingRec *rings,
                                                const int32_t *list, const int32_t *glist, const int32_t *grange,
                                                const TP *partial, double *flux, TA *fold_in)
{
    // block: phase k, energies [64 e0, 64 e0 + 64); thread (g, e): groups i = g mod 4
    extern __shared__ unsigned char act[];
    __shared__ double red[4][64];
    const int k = blockIdx.x, b = blockIdx.z;
    const int E = S.E, P = S.P;
    const int g0 = grange[2 * b], ng = grange[2 * b + 1] - g0;
    const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int e = blockIdx.y * 64 + el;
    stage_group_flags(list, glist, rings, g0, ng, act);
    __syncthreads();
    double s0 = 0.0, s1 = 0.0;
    if (e < E) {
        const TP *base = partial + ((size_t)g0 * P + k) * E + e;
        const size_t rs = (size_t)P * E;
        int i = grp;
        for (; i + 4 < ng; i += 8) {
            if (act[i]) s0 += (double)base[i * rs];
            if (act[i + 4]) s1 += (double)base[(i + 4) * rs];
        }
        for (; i < ng; i += 4)
            if (act[i]) s0 += (double)base[i * rs];
    }
    red[grp][el] = s0 + s1;
    __syncthreads();
    if (grp == 0 && e < E) {
        double s = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
        const StarRec st = stars[b];
        if (st.status != PPM_INST_OK) s = 0.0;
        if (flux) flux[((size_t)b * P + k) * E + e] = s;
        double att = S.sigma ? exp(-st.NH * S.sigma[e]) : 1.0;
        fold_in[((size_t)b * P + k) * E + e] = (TA)(s * att * (S.t_exp / P));
    }
}

// FP32 partials with E % 4 == 0: a thread owns four consecutive energies and
// reads them with 16-byte loads.
constexpr int kReduceGroups = 16;   // summing groups of k_reduce4, group q taking partials q, q + 16, ...
constexpr int kReduceBatch = 16;    // partial loads in flight per lane

// Block = (phase k, 128 energies, instance b), 8 waves: lane l of wave w
// holds energies 4 (l % 32) .. +3 of the block's 128 for summing group
// 2 w + l / 32.  Each summing group adds its ring-group partials in
// increasing order, then the 16 sums are added in group order (groups 0..3
// take one energy of the four each): a fixed order independent of the
// launch.  256 blocks per instance at 128 phases keep every CU busy.
__global__ __launch_bounds__(32 * kReduceGroups) void k_reduce4(DevSpec S, const StarRec *stars, const RingRec *rings,
                                                 const int32_t *list, const int32_t *glist,
                                                 const int32_t *grange, const float *partial, double *flux,
                                                 float *fold_in)
{
    extern __shared__ unsigned char act[];
    __shared__ double4 red[kReduceGroups][32];
    const int k = blockIdx.x, b = blockIdx.z;
    const int E = S.E, P = S.P;
    const int g0 = grange[2 * b], ng = grange[2 * b + 1] - g0;
    const int el = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int e = (blockIdx.y * 32 + el) * 4;
    const bool live = e < E;
    const float *base = partial + ((size_t)g0 * P + k) * E + (live ? e : 0);
    const size_t rs = (size_t)P * E;
    // the first batch of partials is in flight while the group flags are
    // staged (a partial of an inactive group is read but not added).  The
    // loads are unconditional, all of a batch in flight together: past the
    // instance's groups they re-read its first group, and the sums take
    // only groups below ng with their flag set.
    float4 v[kReduceBatch];
    if (ng > 0) {
#pragma unroll
        for (int j = 0; j < kReduceBatch; ++j) {
            const int i = grp + j * kReduceGroups;
            v[j] = *(const float4 *)(base + (i < ng ? i : 0) * rs);
        }
    }
    stage_group_flags(list, glist, rings, g0, ng, act);
    __syncthreads();
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int i0 = grp; i0 < ng; i0 += kReduceGroups * kReduceBatch) {
        if (i0 != grp) {
#pragma unroll
            for (int j = 0; j < kReduceBatch; ++j) {
                const int i = i0 + j * kReduceGroups;
                v[j] = *(const float4 *)(base + (i < ng ? i : 0) * rs);
            }
        }
#pragma unroll
        for (int j = 0; j < kReduceBatch; ++j) {
            const int i = i0 + j * kReduceGroups;
            const bool add = i < ng && act[i < ng ? i : 0];
            s0 += add ? (double)v[j].x : 0.0;
            s1 += add ? (double)v[j].y : 0.0;
            s2 += add ? (double)v[j].z : 0.0;
            s3 += add ? (double)v[j].w : 0.0;
        }
    }
    red[grp][el] = make_double4(s0, s1, s2, s3);
    __syncthreads();
    // group q < 4 adds the group sums of energy component q in group order
    if (grp < 4 && live) {
        const int q = grp;
        double t = 0.0;
        for (int g2 = 0; g2 < kReduceGroups; ++g2) {
            const double *vv = (const double *)&red[g2][el];
            t += vv[q];
        }
        const StarRec st = stars[b];
        const size_t o = ((size_t)b * P + k) * E + e + q;
        const double sv = st.status != PPM_INST_OK ? 0.0 : t;
        if (flux) flux[o] = sv;
        const double att = S.sigma ? exp(-st.NH * S.sigma[e + q]) : 1.0;
        fold_in[o] = (float)(sv * att * (S.t_exp / P));
    }
}

// ---------------------------------------------------------------------------
// k_fold: counts[M][C] = A[M][E] . RSP[E][C] on the matrix cores.  Block =
// one 16x16 output tile, four waves splitting K into quarters; per wave K in
// steps of 4 (v_mfma_f32_16x16x4f32): lane l supplies A[l%16][k0 + l/16] and
// RSP[k0 + l/16][l%16]; the tile comes back as D[4 (l/16) + v][l%16] in
// accumulator v.  The four partial tiles are summed in LDS in wave order.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_fold_f32(const float *A, const float *B, double *out, int M,
                                                  int N, int K)
{
    __shared__ floatx4 part[4][64];
    const int n0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int kq = ((K + 15) / 16) * 4;
    const int kb = wave * kq, ke = min(K, kb + kq);
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool mrow = (m0 + li) < M, ncol = (n0 + li) < N;
    // sixteen K steps at a time: all their operands loaded first (in-bounds
    // addresses, zero where outside), then the MFMAs in K order
    constexpr int kSteps = 16;
    for (int kc = kb; kc < ke; kc += 4 * kSteps) {
        float av[kSteps], bv[kSteps];
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const int k = kc + 4 * s + lk;
            const bool oka = mrow && k < ke, okb = ncol && k < ke;
            const float va = A[oka ? (size_t)(m0 + li) * K + k : 0];
            const float vb = B[okb ? (size_t)k * N + n0 + li : 0];
            av[s] = oka ? va : 0.0f;
            bv[s] = okb ? vb : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < kSteps; ++s)
            if (kc + 4 * s < ke) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
    }
    part[wave][l] = acc;
    __syncthreads();
    if (wave == 0) {
        floatx4 t = part[0][l];
        t += part[1][l];
        t += part[2][l];
        t += part[3][l];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int row = m0 + 4 * lk + v, col = n0 + li;
            if (row < M && col < N) out[(size_t)row * N + col] = (double)t[v];
        }
    }
}

// k_fold_ll: the fold of k_fold_f32 (same tiles, same K split, the same
// result bits) followed by the Poisson log-likelihood terms of the tile's
// bins (FP64; d = 0 contributes -m, m <= 0 with d > 0 is flagged): wave w
// takes the tile's rows 4 j + w, and per output row (instance b, phase k)
// the tile's 16 channels are summed in a fixed lane butterfly into
// part[row][column tile].  k_ll_sum then adds an instance's P x n_ct
// partials in a fixed order that depends only on P and C, so an instance
// gives the same logL alone and in a batch.  out (model counts) may be NULL.
__device__ inline double log_dfact(int d, const double *lfact)
{
    return (unsigned)d < (unsigned)kLogFact ? lfact[d] : lgamma(d + 1.0);   // log d!, tabulated below kLogFact
}

__global__ __launch_bounds__(256) void k_fold_ll(const float *A, const float *Bm, double *out, int M, int N, int K,
                                                 int P, const double *bkg, const int32_t *data,
                                                 const double *lfact, double *part, int32_t *bad)
{
    __shared__ floatx4 tile[4][64];
    const int n0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int kq = ((K + 15) / 16) * 4;
    const int kb = wave * kq, ke = min(K, kb + kq);
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool mrow = (m0 + li) < M, ncol = (n0 + li) < N;
    constexpr int kSteps = 16;
    for (int kc = kb; kc < ke; kc += 4 * kSteps) {
        float av[kSteps], bv[kSteps];
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const int k = kc + 4 * s + lk;
            const bool oka = mrow && k < ke, okb = ncol && k < ke;
            const float va = A[oka ? (size_t)(m0 + li) * K + k : 0];
            const float vb = Bm[okb ? (size_t)k * N + n0 + li : 0];
            av[s] = oka ? va : 0.0f;
            bv[s] = okb ? vb : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < kSteps; ++s)
            if (kc + 4 * s < ke) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
    }
    tile[wave][l] = acc;
    __syncthreads();
    // wave w: accumulator element w of the four partial tiles, summed in
    // wave order as in k_fold_f32
    const float *t0 = (const float *)&tile[0][l], *t1 = (const float *)&tile[1][l],
                *t2 = (const float *)&tile[2][l], *t3 = (const float *)&tile[3][l];
    float t = t0[wave];
    t += t1[wave];
    t += t2[wave];
    t += t3[wave];
    const int col = n0 + li, row = m0 + 4 * lk + wave, n_ct = gridDim.x;
    double term = 0.0;
    int nbad = 0;
    if (row < M && col < N) {
        const double mv = (double)t;
        if (out) out[(size_t)row * N + col] = mv;
        const int k = row % P;
        const int d = data[(size_t)k * N + col];
        const double mi = bkg ? mv + bkg[(size_t)k * N + col] : mv;   // model plus background counts
        if (d == 0) term = -mi;
        else if (!(mi > 0.0)) nbad = 1;
        else term = d * log(mi) - mi - log_dfact(d, lfact);
    }
    // the row's 16 channels: lanes 16 lk .. 16 lk + 15
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        term += __shfl_xor(term, o, 64);
        nbad += __shfl_xor(nbad, o, 64);
    }
    if (li == 0 && row < M) {
        part[(size_t)row * n_ct + blockIdx.x] = term;
        bad[(size_t)row * n_ct + blockIdx.x] = nbad;
    }
}

// k_ll_sum: block b adds instance b's n = P x n_ct likelihood partials:
// thread t the entries t, t + 256, ... in order, then the 256 sums in a
// fixed tree; -inf where a bin had m <= 0 with d > 0 or the instance is not
// evaluable.
__global__ __launch_bounds__(256) void k_ll_sum(int n, const StarRec *stars, const double *part,
                                                const int32_t *bad, double *logl)
{
    __shared__ double red[256];
    __shared__ int redb[256];
    const int b = blockIdx.x;
    const double *pp = part + (size_t)b * n;
    const int32_t *pb = bad + (size_t)b * n;
    double sv = 0.0;
    int sb = 0;
    constexpr int kU = 8;   // loads in flight per thread
    for (int i0 = threadIdx.x; i0 < n; i0 += 256 * kU) {
        double v[kU];
        int f[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = i0 + 256 * u;
            v[u] = i < n ? pp[i] : 0.0;
            f[u] = i < n ? pb[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            sv += v[u];
            sb += f[u];
        }
    }
    red[threadIdx.x] = sv;
    redb[threadIdx.x] = sb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            redb[threadIdx.x] += redb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double s = red[0];
        if (redb[0] || stars[b].status != PPM_INST_OK) s = -INFINITY;
        logl[b] = s;
    }
}

// FP64 path (small workloads): one thread per output element, plain FMA loop.
__global__ __launch_bounds__(256) void k_fold_f64(const double *A, const double *B, double *out, int M,
                                                  int N, int K)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x, row = blockIdx.y;
    if (col >= N || row >= M) return;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc = fma(A[(size_t)row * K + k], B[(size_t)k * N + col], acc);
    out[(size_t)row * N + col] = acc;
}

// ---------------------------------------------------------------------------
// k_loglike: Poisson log-likelihood per instance, FP64, fixed-order block
// reduction.  d = 0 contributes -m; m <= 0 with d > 0 gives -inf.
// ---------------------------------------------------------------------------
constexpr int kLLChunk = 512;    // bins per block of the first likelihood stage

// Block = kLLChunk bins of one instance: per-block sums, then the block that
// finishes last for the instance (a per-instance counter) adds the block sums
// in block order (wave 0: lane-strided sums, then a fixed butterfly) and
// resets the counter for the next call.
__global__ __launch_bounds__(256) void k_loglike(const StarRec *stars, const double *counts, const double *bkg,
                                                 const int32_t *data, const double *lfact, int PC, double *part,
                                                 int32_t *bad, unsigned *done, double *logl)
{
    const int b = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
    __shared__ double red[256];
    __shared__ int nb[256];
    __shared__ bool last;
    double s = 0.0;
    int nbad = 0;
    const double *m = counts + (size_t)b * PC;
    const int i0 = blk * kLLChunk, i1 = min(PC, i0 + kLLChunk);
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        int d = data[i];
        double mi = bkg ? m[i] + bkg[i] : m[i];   // model plus background counts
        if (d == 0) { s -= mi; continue; }
        if (!(mi > 0.0)) { ++nbad; continue; }
        s += d * log(mi) - mi - ((unsigned)d < (unsigned)kLogFact ? lfact[d] : lgamma(d + 1.0));   // log d!, tabulated for 0 <= d < kLogFact
    }
    red[threadIdx.x] = s;
    nb[threadIdx.x] = nbad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            nb[threadIdx.x] += nb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[(size_t)b * nblk + blk] = red[0];
        bad[(size_t)b * nblk + blk] = nb[0];
        __threadfence();                                   // the block sum is visible before the count
        last = atomicAdd(&done[b], 1u) == (unsigned)(nblk - 1);
    }
    __syncthreads();
    if (!last || threadIdx.x >= 64) return;
    __threadfence();                                       // every block's sum is visible to this one
    const volatile double *vp = part + (size_t)b * nblk;
    const volatile int32_t *vb = bad + (size_t)b * nblk;
    const int lane = threadIdx.x;
    double t = 0.0;
    int tb = 0;
    for (int q = lane; q < nblk; q += 64) {
        t += vp[q];
        tb += vb[q];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        t += __shfl_xor(t, o, 64);
        tb += __shfl_xor(tb, o, 64);
    }
    if (lane == 0) {
        if (tb || stars[b].status != PPM_INST_OK) t = -INFINITY;
        logl[b] = t;
        done[b] = 0u;
    }
}

__global__ void k_status(const StarRec *stars, int B, int32_t *out)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = stars[b].status;
}

// ---------------------------------------------------------------------------
// launch wrappers (host)
// ---------------------------------------------------------------------------
int loglike_blocks(int PC) { return (PC + kLLChunk - 1) / kLLChunk; }

int loglike_parts(int P, int C)
{
    const int fused = P * ((C + 15) / 16), blocks = loglike_blocks(P * C);
    return fused > blocks ? fused : blocks;
}

size_t accum_table_lds(const DevSpec &S)
{
    if (S.fast)
        return sizeof(double4) * (S.n_fp + 1) + sizeof(double) * ((S.nmu + 1) & ~1)
             + sizeof(float) * fast_tab_floats(S) + sizeof(float4) * kFwdWaves * 64 + sizeof(float4) * kFwdWaves * 64
             + sizeof(float) * kFwdWaves * ((S.E + 63) / 64 <= 1 ? 1 : ((S.E + 63) / 64 <= 2 ? 2 : ((S.E + 63) / 64 <= 4 ? 4 : 8))) * 64
             + sizeof(double) * 2 * (S.n_fp + 1) + sizeof(double) * 4 * S.nmu
             + sizeof(int16_t) * (2 * S.n_fp + S.mu_nb) + sizeof(float) * 2 * S.E;
    return sizeof(double4) * (S.n_fp + 1) + sizeof(double) * S.nmu + sizeof(float) * S.nmu * S.nx
         + sizeof(float) * 4 * S.nx;
}

void launch_setup(const DevSpec &S, const Workspace &W, const double *params, const int32_t *ncells_dev, int B,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_setup, dim3((S.R_tot + 63) / 64, B), dim3(64 * kSetupWaves), 0, st, S, params, ncells_dev, W.stars,
                       W.rings, W.vis_pairs, W.diag);
}

void launch_table_trace(const DevSpec &S, const Workspace &W, const int32_t *list, int n_list, hipStream_t st)
{
    const int nodes_per_block = 256 / kTableSplit;
    hipLaunchKernelGGL(k_table, dim3(n_list, (S.n_alpha + nodes_per_block - 1) / nodes_per_block), dim3(256), 0, st, S,
                       list, W.stars, W.rings, W.table);
    size_t lds_tr = sizeof(double4) * (S.n_alpha + S.n_fp + 1);
    hipLaunchKernelGGL(k_trace, dim3(n_list), dim3(kTraceThreads), lds_tr, st, S, list, W.stars, W.rings, W.table,
                       W.trace, W.sub, W.diag);
}

// FP32 ring-group partials -> per-instance FP64 sum, absorption, MFMA fold,
// and with data the likelihood in the fold's epilogue
void launch_reduce_fold32(const DevSpec &S, const Workspace &W, const int32_t *list, int B, hipStream_t st,
                          double *flux_out, double *counts_out, const int32_t *data, double *logl)
{
    if ((S.E & 3) == 0)
        hipLaunchKernelGGL(k_reduce4, dim3(S.P, (S.E + 127) / 128, B), dim3(32 * kReduceGroups), S.R_tot, st, S,
                           W.stars, W.rings, list, W.glist, W.grange, W.partial32, flux_out, W.fold_in32);
    else
        hipLaunchKernelGGL((k_reduce<float, float>), dim3(S.P, (S.E + 63) / 64, B), dim3(256), S.R_tot, st, S,
                           W.stars, W.rings, list, W.glist, W.grange, W.partial32, flux_out, W.fold_in32);
    launch_fold32(S, W, B, st, counts_out, data, logl);
}

void launch_fold32(const DevSpec &S, const Workspace &W, int B, hipStream_t st, double *counts_out,
                   const int32_t *data, double *logl)
{
    const dim3 grid((S.C + 15) / 16, (B * S.P + 15) / 16);
    if (data) {
        hipLaunchKernelGGL(k_fold_ll, grid, dim3(256), 0, st, W.fold_in32, S.rsp32, counts_out, B * S.P, S.C, S.E,
                           S.P, S.bkg, data, W.lfact, W.ll_part, W.ll_bad);
        hipLaunchKernelGGL(k_ll_sum, dim3(B), dim3(256), 0, st, S.P * (int)grid.x, W.stars, W.ll_part, W.ll_bad,
                           logl);
    } else {
        hipLaunchKernelGGL(k_fold_f32, grid, dim3(256), 0, st, W.fold_in32, S.rsp32, counts_out, B * S.P, S.C, S.E);
    }
}

// The windowed kernel runs over the ring groups of the pass (W.glist), the
// generic and blackbody kernels over its rings (groups of one ring: the
// group list is then the identity, n_groups == n_list).
hipError_t launch_forward(const DevSpec &S, const Workspace &W, const double *params,
                          const int32_t *ncells_dev, int B, const int32_t *list, int n_list, int n_groups,
                          hipStream_t st, double *flux_out, double *counts_out, const int32_t *data, double *logl,
                          hipEvent_t ev_hot0, hipEvent_t ev_hot1)
{
    const bool want_flux_f64 = flux_out != nullptr;
    launch_setup(S, W, params, ncells_dev, B, st);
    launch_table_trace(S, W, list, n_list, st);
    const int PT = S.pt_fwd;
    const int n_tile = (S.P + PT - 1) / PT;
    const size_t PE = (size_t)S.P * S.E;
    if (S.intensity == PPM_I_TABLE) {
        size_t lds = accum_table_lds(S);
        if (ev_hot0) (void)hipEventRecord(ev_hot0, st);
        int epl = (S.E + 63) / 64;
        if (S.fast) {
            const int step = max_list_per_launch(n_tile, 64 * kFwdWaves);
            for (int off = 0; off < n_groups; off += step) {
                const int32_t *gl = W.glist + 2 * (size_t)off;
                float *pt = W.partial32 + (size_t)off * PE;
                const int n = n_groups - off < step ? n_groups - off : step;
                dim3 grid(xcd_grid(n, n_tile));
#define PPM_FAST(E_, G_)                                                                                          \
    hipLaunchKernelGGL((k_accum_fast<E_, kFwdWaves, G_>), grid, dim3(64 * kFwdWaves), lds, st, S, list, gl,       \
                       W.rings, W.trace, W.sub, pt, W.vis_pairs, W.diag, PT, n)
#define PPM_FAST_E(G_)                     \
    do {                                   \
        if (epl <= 1) PPM_FAST(1, G_);     \
        else if (epl <= 2) PPM_FAST(2, G_); \
        else if (epl <= 4) PPM_FAST(4, G_); \
        else PPM_FAST(8, G_);              \
    } while (0)
                if (S.ring_group > 1) PPM_FAST_E(true);
                else PPM_FAST_E(false);
#undef PPM_FAST_E
#undef PPM_FAST
            }
        } else {
            const int step = max_list_per_launch(n_tile, 256);
            for (int off = 0; off < n_list; off += step) {
                const int32_t *sl = list + off;
                float *pt = W.partial32 + (size_t)off * PE;
                const int n = n_list - off < step ? n_list - off : step;
                dim3 grid(xcd_grid(n, n_tile));
#define PPM_TAB(E_)                                                                                               \
    hipLaunchKernelGGL(k_accum_table<E_>, grid, dim3(256), lds, st, S, sl, W.rings, W.trace, W.sub, pt,          \
                       W.vis_pairs, W.diag, PT, n)
                if (epl <= 1) PPM_TAB(1);
                else if (epl <= 2) PPM_TAB(2);
                else if (epl <= 4) PPM_TAB(4);
                else PPM_TAB(8);
#undef PPM_TAB
            }
        }
        if (ev_hot1) (void)hipEventRecord(ev_hot1, st);
        launch_reduce_fold32(S, W, list, B, st, want_flux_f64 ? flux_out : nullptr, counts_out, data, logl);
    } else {
        size_t lds = sizeof(double4) * (S.n_fp + 1);
        int epl = (S.E + 63) / 64;
        if (ev_hot0) (void)hipEventRecord(ev_hot0, st);
        const int step = max_list_per_launch(n_tile, 256);
        for (int off = 0; off < n_list; off += step) {
            const int32_t *sl = list + off;
            double *pt = W.partial64 + (size_t)off * PE;
            const int n = n_list - off < step ? n_list - off : step;
            dim3 grid(xcd_grid(n, n_tile));
#define PPM_BB(E_) \
    hipLaunchKernelGGL(k_accum_bb<E_>, grid, dim3(256), lds, st, S, sl, W.rings, W.trace, pt, W.vis_pairs, PT, n)
            if (epl <= 1) PPM_BB(1);
            else if (epl <= 2) PPM_BB(2);
            else if (epl <= 4) PPM_BB(4);
            else PPM_BB(8);
#undef PPM_BB
        }
        if (ev_hot1) (void)hipEventRecord(ev_hot1, st);
        double *fx = want_flux_f64 ? flux_out : nullptr;
        if (S.rsp64) {
            hipLaunchKernelGGL((k_reduce<double, double>), dim3(S.P, (S.E + 63) / 64, B), dim3(256), S.R_tot, st, S,
                               W.stars, W.rings, list, W.glist, W.grange, W.partial64, fx, W.fold_in64);
            hipLaunchKernelGGL(k_fold_f64, dim3((S.C + 255) / 256, B * S.P), dim3(256), 0, st,
                               W.fold_in64, S.rsp64, counts_out, B * S.P, S.C, S.E);
            if (data) {
                const int nblk = loglike_blocks(S.P * S.C);
                hipLaunchKernelGGL(k_loglike, dim3(nblk, B), dim3(256), 0, st, W.stars, counts_out, S.bkg, data,
                                   W.lfact, S.P * S.C, W.ll_part, W.ll_bad, W.ll_done, logl);
            }
        } else {
            hipLaunchKernelGGL((k_reduce<double, float>), dim3(S.P, (S.E + 63) / 64, B), dim3(256), S.R_tot, st, S,
                               W.stars, W.rings, list, W.glist, W.grange, W.partial64, fx, W.fold_in32);
            launch_fold32(S, W, B, st, counts_out, data, logl);
        }
    }
    return hipGetLastError();
}

hipError_t launch_status(const Workspace &W, int B, int32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_status, dim3((B + 255) / 256), dim3(256), 0, st, W.stars, B, out);
    return hipGetLastError();
}

}  // namespace ppm
