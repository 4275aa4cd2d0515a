// Internal records shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppm {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;
constexpr double kHalfPi = 0.5 * kPi;

// physical constants, CGS + keV
constexpr double kC = 2.99792458e10;
constexpr double kGMsun = 1.3271244e26;
constexpr double kKB = 8.617333262e-8;
constexpr double kH = 4.135667696e-18;
constexpr double kPc = 3.0856775814913673e18;

constexpr int kMaxMu = 128;       // mu nodes held in constant memory

// Static model description as seen by the kernels (device pointers).
struct DevSpec {
    int mode, intensity, n_spots;
    int interp;           // atmosphere interpolation strategy (ppm_interp)
    int shape[2];
    double shape_a[2], shape_b[2];
    int n_fp, P, E, C;
    int nT, ng, nmu, nx;
    int n_alpha, n_quad;
    int fast;             // 1: windowed accumulation kernel applies (energy span <= 59 x-intervals)
    int W_max;            // x-node window of the per-ring sub-table
    int sub_stride;       // floats per ring in the sub-table buffer (multiple of 4)
    int pt_fwd, pt_adj;   // phases per block of the forward / adjoint accumulation kernels
    int ring_group;       // rings summed per block of the windowed forward accumulation
    int n_side;           // temperature-map plan: HEALPix resolution (0: spot model)
    int n_pix;            // patches of a map (12 n_side^2)
    int map_nb;           // temperature buckets of a map ring (logT steps, with margins)
    int map_wm;           // x nodes of a bucket's slab window
    double tb0, r_span;   // (log10 E_0 - x0)/hx and (log10 E_last - log10 E_0)/hx
    double ihx;           // 1 / hx
    float ixl;            // 1 / (hx ln 10): x nodes per unit of ln z
    double mu_lo, mu_hi;  // first and last mu node
    double Pd, fpb;       // n_phase and 2 n_fp (the phase buckets) as doubles
    const float *tbe;     // [E] (log10 E_e - log10 E_0)/hx, the energies' x offsets
    // gradient plans: the energies grouped by the unit x interval their offset
    // falls in, bucket h = [ebkt[h], ebkt[h + 1]) holding floor(tbe) = h, and
    // each offset's part above its bucket (etau[E] = 2 closes the array)
    const int32_t *ebkt;  // [65]
    const float *etau;    // [E + 1] tbe[e] - floor(tbe[e])
    int e_it;             // binary-search steps that cover the largest bucket
    int R_tot;            // ring slots per instance (spot 0 then spot 1)
    int rings_max[2];     // ring slots of each spot
    int n_rings_spec[2], n_phi_spec[2];   // default grid of each spot
    double t_exp;
    double T0, hT, g0, hg, x0, hx;   // uniform logT, log g, x axes
    double T_end[2], g_end[2];       // first and last node of the logT and log g axes (clamp counting)
    const double *energy;   // [E] keV
    const double *sigma;    // [E] cm^2 (nullptr: no absorption)
    const float *rsp32;     // [E][C]
    const double *rsp64;    // [E][C]
    const double *rspT64;   // [C][E] (gradient plans: backward fold)
    const double *bkg;      // [P][C] background counts per bin (nullptr: none)
    const float *atm;       // [nT][ng][nmu][nx] linear I/T^3
    const double *ax_mu;    // [nmu]
    // mu-axis lookup of the windowed kernel: per interval l (a_l <= mu < a_{l+1})
    // the linear 1/(a_{l+1} - a_l) (l < 3, l = nmu - 2) or the four inverse
    // denominators of the cubic Lagrange weights on nodes l-1 .. l+2; and
    // mu_nb equal buckets over [a_0, a_{nmu-1}], each with the largest l
    // whose node lies at or below the bucket's lower edge
    const double *mu_coef;  // [nmu][4]
    const int16_t *mu_bucket;   // [mu_nb]
    int mu_nb;
    double mu_ibw;          // mu_nb / (a_{nmu-1} - a_0)
    const double *glx, *glw;  // Gauss-Legendre on [0, 1], n_quad nodes
};

// LDS copy of a ring's sub-table in the windowed kernel: x-major, the nmu
// values of one x node adjacent, node stride nmu | 1 (odd, so 64 lanes on
// consecutive nodes hit distinct banks); floats, rounded up to 16 bytes
__host__ __device__ inline int fast_tab_stride(int nmu) { return nmu | 1; }
__host__ __device__ inline int fast_tab_floats(const DevSpec &S)
{
    return (fast_tab_stride(S.nmu) * S.W_max + 3) & ~3;
}

struct StarRec {
    double GM, Rs, Re, x, Obar, o2, g0, D, nu, si, ci, NH;
    int status;
    int pad;
};

struct RingRec {
    double theta, dcos, R, u, sq1u, f, coseta, sineta, logg, beta, gamma;
    double dphi_out, dphi_in, dphi_cell, w_cell;
    double alpha_max, cdt_obl;   // c dt(R)/R of Eq. (16)
    double phi_spot;             // -2 pi (Phi + dphi_s)
    double logT, T, kT;
    double tm, cos_zm;           // crescent mask centre colatitude, cos(mask radius)
    int spot, shape, n_cells, active;
    int visible, inv_min, inv_max, interior;   // interior: the ring never reaches the x-axis edge intervals
    double zmin, zmax;           // range of the fine-phase redshift factor z
    int xw0, xw;                 // x-node window [xw0, xw0 + xw) of the ring's sub-table
    double tbk;                  // (log10(E_0 / kT) - x0)/hx: x position of E_0 at z = 1
};

// One active patch of a temperature-map ring, sorted by temperature bucket:
// cell index on the ring, logT interpolation weight between the bucket's
// two table nodes, (T / 10^6 K)^3, log10(k T / keV) and whether its logT
// was clamped to the table.
struct MapCell {
    double lkT;
    float t, T3;
    int j, clamped;   // clamped: the patch's logT lies outside the table's logT axis
};

// Temperature buckets of map rings: bucket q holds logT in
// [T0 + (q - kMapLow) hT, T0 + (q - kMapLow + 1) hT).
constexpr int kMapLow = 64;

// Ring-level tangents along the five local directions of a ring's geometry
// (M, R_e, inclination, the ring's spot colatitude and angular radius).
struct RingTan {
    double dlogg[5], dw[5];      // log g of the ring, cell weight
    double ddout[5], ddin[5];    // arc half-widths (outer, inner)
};

}  // namespace ppm
