/*
 * FP64 CPU oracle of the energy-resolved pulse-profile forward model and its
 * Poisson likelihood (Zhou & Huang, "GPU-accelerated X-ray pulse profile
 * modeling", arXiv:2510.07764).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP implementation: both consume the same seeded inputs.
 *
 * Every step is the paper's recipe written out plainly in double precision:
 * adaptive quadrature for the light-bending and time-delay integrals
 * (Eqs. 32, 35) evaluated exactly at each ray (no lookup table), Brent root
 * finding for the inverse map psi -> alpha, the pseudo-patch fine-phase
 * trace with invisible-segment fill (Sect. 2.8.3, Eqs. 38-44), shift-and-add
 * with linear phase interpolation (Eqs. 45-47), the naive 2x2x4x4 tensor
 * stencil of the mixed-order atmosphere interpolator (Sect. 4), absorption
 * (Eq. 22), response fold (Eq. 55) and the Poisson log-likelihood.
 */
#ifndef PPM_ORACLE_H
#define PPM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NPARAM 16

typedef struct {
    int mode;          /* 0: spherical + Doppler (S+D), 1: oblate Schwarzschild (OS) */
    int intensity;     /* 0: isotropic blackbody, 1: atmosphere table */
    int n_spots;       /* 1 or 2 */
    int shape[2];      /* 0 cap, 1 annulus, 2 crescent */
    int n_rings[2];
    int n_phi[2];
    double shape_a[2]; /* annulus: zeta_in/zeta ; crescent: mask radius/zeta */
    double shape_b[2]; /* crescent: mask-centre offset/zeta, towards the equator */
    int n_fp, n_phase, n_energy, n_chan;
    const double *energy;  /* [E] keV */
    const double *sigma;   /* [E] cm^2 */
    const double *rsp;     /* [E][C] cm^2 keV */
    double t_exp;          /* s */
    int nT, ng, nmu, nx;
    const double *ax_T, *ax_g, *ax_mu, *ax_x;
    const double *logI;    /* [nT][ng][nmu][nx] log10(I/T^3) */
    int interp;            /* atmosphere interpolation strategy of Sect. 4: 0 (d) mixed,
                              1 (a) cubic, 2 (b) cubic clipped at zero, 3 (c) cubic with
                              linear protected small-mu zone */
} orc_spec;

typedef struct {
    long long n_clamp_T, n_clamp_g, n_x_outside, n_multi_image, n_visible_pairs;
    int status;
    long long n_negative;  /* interpolated intensities below zero (before any clipping) */
} orc_diag;

typedef struct {
    double GM, Rs, Re, x, Obar, o2, g0, D, nu, incl, NH;
} orc_star;

typedef struct {
    double theta, dcos, R, u, f, coseta, sineta, logg, beta, gamma;
    double dphi_out, dphi_in, dphi_cell, w_cell;
    double alpha_max, psi_top;
    int n_cells;
} orc_ring;

/* light bending / delay primitives (Sect. 2.3, 2.8.2) */
double orc_psi(double u, double alpha);          /* both branches */
double orc_dpsi_dalpha(double u, double alpha);  /* both branches */
double orc_tp(double u, double alpha);           /* c dt_p / R, both branches */
double orc_rho(double u, double alpha);          /* Eq. (14) */
double orc_alpha_capture(double u);
/* inverse map: psi -> alpha, cos(alpha), d cos(alpha)/d cos(psi), sin(alpha)/sin(psi) */
int orc_invert(double u, double alpha_max, double psi, double out[4]);

void orc_star_setup(const orc_spec *s, const double *p, orc_star *st);
int orc_rings(const orc_spec *s, const double *p, int spot, orc_ring *rings);
double orc_cdt_oblate(const orc_star *st, double R);   /* Eq. (16) */
double orc_total_delay(const orc_star *st, double R, double u, double alpha); /* c dt / R */

/* fine-phase trace of one ring: arrays of length n_fp+1; returns 1 if the
   ring is visible at phi = 0, else 0 (ring skipped) */
int orc_trace_ring(const orc_spec *s, const double *p, const orc_ring *rg,
                   double *F, double *z, double *phio, double *mu, int *inv_range,
                   orc_diag *diag);

double orc_atmo(const orc_spec *s, const double *linI, double logT, double logg,
                double mu, double x, orc_diag *diag);
double orc_atmo_interp_mode(const orc_spec *s, const double *linI, double logT, double logg,
                            double mu, double x, int mode, orc_diag *diag);
double orc_blackbody(double E_kev, double T_kelvin);

/* full model: Ft[P][E] photon flux (ph cm^-2 s^-1 keV^-1, no absorption),
   counts[P][C] (NULL to skip). */
int orc_forward(const orc_spec *s, const double *p, double *Ft, double *counts, orc_diag *diag);
double orc_loglike_counts(const double *counts, const int *data, long long n);

/* HEALPix ring i = 1 .. 4 nside - 1 (Sect. 2.8.1): cos(colatitude), pixels
   on the ring, azimuth of its first pixel (pixels are 2 pi / nphi apart). */
void orc_healpix_ring(int nside, int i, double *z, int *nphi, double *phi_first);
/* Forward model of a full-surface temperature map (Sects. 2.6, 2.8.1):
   logT_map[12 nside^2] holds log10 T [K] per HEALPix patch in ring order
   (rings from the north pole, pixels by increasing azimuth); a value that is
   not finite or not positive marks an inactive patch.  Parameter slots 0-6
   as for spots; the spot slots are ignored.  Returns 0, -1 for nside < 1. */
int orc_forward_map(const orc_spec *s, const double *p, int nside, const double *logT_map, double *Ft,
                    double *counts, orc_diag *diag);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
