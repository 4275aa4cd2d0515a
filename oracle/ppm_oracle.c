/*
 * FP64 CPU oracle — TEST INFRASTRUCTURE (see ppm_oracle.h).
 *
 * Plain, slow, double-precision implementation of the paper's forward model.
 * Section / equation numbers refer to arXiv:2510.07764.
 */
#include "ppm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define TWO_PI (2.0 * PI)
#define HALF_PI (0.5 * PI)

/* constants, CGS + keV */
static const double C_CGS = 2.99792458e10;
static const double GM_SUN = 1.3271244e26;
static const double K_B = 8.617333262e-8;
static const double H_KEVS = 4.135667696e-18;
static const double PC_CM = 3.0856775814913673e18;

/* ------------------------------------------------------------------------ */
/* Global-adaptive Gauss-Kronrod (7,15) quadrature.                          */
/* ------------------------------------------------------------------------ */
typedef double (*orc_fn)(double x, const void *ctx);

static const double GK_X[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double GK_WK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double GK_WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

static void gk15(orc_fn f, const void *ctx, double a, double b, double *res, double *err)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = f(c, ctx);
    double rk = fc * GK_WK[7], rg = fc * GK_WG[3];
    for (int j = 0; j < 7; ++j) {
        double dx = h * GK_X[j];
        double f1 = f(c - dx, ctx), f2 = f(c + dx, ctx);
        rk += GK_WK[j] * (f1 + f2);
        if (j & 1) rg += GK_WG[j / 2] * (f1 + f2);
    }
    *res = rk * h;
    *err = fabs((rk - rg) * h);
}

#define QMAX 4000
static double integrate(orc_fn f, const void *ctx, double a, double b, double epsrel)
{
    double lo[QMAX], hi[QMAX], r[QMAX], e[QMAX];
    int n = 1;
    lo[0] = a; hi[0] = b;
    gk15(f, ctx, a, b, &r[0], &e[0]);
    for (;;) {
        double tot = 0.0, terr = 0.0;
        int worst = 0;
        for (int i = 0; i < n; ++i) {
            tot += r[i]; terr += e[i];
            if (e[i] > e[worst]) worst = i;
        }
        if (terr <= epsrel * fabs(tot) || terr < 1e-300 || n >= QMAX - 1) return tot;
        double m = 0.5 * (lo[worst] + hi[worst]);
        if (m <= lo[worst] || m >= hi[worst]) return tot;
        lo[n] = m; hi[n] = hi[worst];
        hi[worst] = m;
        gk15(f, ctx, lo[worst], hi[worst], &r[worst], &e[worst]);
        gk15(f, ctx, lo[n], hi[n], &r[n], &e[n]);
        ++n;
    }
}

/* ------------------------------------------------------------------------ */
/* Light bending and time delay, outgoing rays (Sect. 2.8.2, Eqs. 32-33, 35) */
/* ------------------------------------------------------------------------ */
typedef struct { double c, s, u; } bend_ctx;

/* q(x)/sin^2(alpha) of Eq. (33) */
static double q_over_s2(double x, double u)
{
    double t = 1.0 - x * x;
    return 2.0 - x * x - u * t * t / (1.0 - u);
}

static double f_psi(double x, const void *vp)
{
    const bend_ctx *b = (const bend_ctx *)vp;
    double D = b->c * b->c + x * x * b->s * b->s * q_over_s2(x, b->u);
    return x / sqrt(D);
}

static double f_dpsi(double x, const void *vp)
{
    const bend_ctx *b = (const bend_ctx *)vp;
    double D = b->c * b->c + x * x * b->s * b->s * q_over_s2(x, b->u);
    return x / (D * sqrt(D));
}

static double f_tp(double x, const void *vp)
{
    const bend_ctx *b = (const bend_ctx *)vp;
    double D = b->c * b->c + x * x * b->s * b->s * q_over_s2(x, b->u);
    double r = sqrt(D);
    return x / (r * (1.0 + r));
}

static const double QTOL = 1e-14;

/* Eq. (32): psi(u, alpha) for 0 <= alpha <= pi/2 */
static double psi_out(double u, double alpha)
{
    if (alpha <= 0.0) return 0.0;
    bend_ctx b = {cos(alpha), sin(alpha), u};
    if (alpha >= HALF_PI) b.c = 0.0;
    return 2.0 * b.s / sqrt(1.0 - u) * integrate(f_psi, &b, 0.0, 1.0, QTOL);
}

/* d psi / d alpha of Eq. (32), differentiated under the integral sign:
   with D = cos^2 a + x^2 q, d(sin a D^-1/2)/da = cos a D^-3/2, so
   psi' = 2 cos a / sqrt(1-u) * int_0^1 x D^-3/2 dx.  At alpha = pi/2 the
   product tends to 2 / (sqrt(1-u) q(0)). */
static double dpsi_out(double u, double alpha)
{
    if (alpha >= HALF_PI) return 2.0 / (sqrt(1.0 - u) * q_over_s2(0.0, u));
    bend_ctx b = {cos(alpha), sin(alpha), u};
    return 2.0 * b.c / sqrt(1.0 - u) * integrate(f_dpsi, &b, 0.0, 1.0, QTOL);
}

/* Eq. (35): c dt_p / R for 0 <= alpha <= pi/2 */
static double tp_out(double u, double alpha)
{
    if (alpha <= 0.0) return 0.0;
    bend_ctx b = {cos(alpha), sin(alpha), u};
    if (alpha >= HALF_PI) b.c = 0.0;
    return 2.0 * b.s * b.s / (1.0 - u) * integrate(f_tp, &b, 0.0, 1.0, QTOL);
}

/* Eq. (14): periastron radius in units of the emission radius */
double orc_rho(double u, double alpha)
{
    double sa = sin(alpha);
    double k = sqrt(3.0 * (1.0 - u));
    double arg = 3.0 * u * k / (2.0 * sa);
    if (arg > 1.0) arg = 1.0;
    return -2.0 * sa / k * cos((acos(arg) + TWO_PI) / 3.0);
}

/* largest emission angle whose ray still has a periastron outside the
   photon sphere: sin(alpha) = 3u sqrt(3(1-u))/2 on the inward side */
double orc_alpha_capture(double u)
{
    double v = 1.5 * u * sqrt(3.0 * (1.0 - u));
    if (v >= 1.0) return HALF_PI;
    return PI - asin(v);
}

/* psi over both branches: Eqs. (32) and (34) (equivalently (13)) */
double orc_psi(double u, double alpha)
{
    if (alpha <= HALF_PI) return psi_out(u, alpha);
    double rho = orc_rho(u, alpha);
    return 2.0 * psi_out(u / rho, HALF_PI) - psi_out(u, PI - alpha);
}

/* c dt_p/R over both branches, Eqs. (35)-(36).  On the inward branch the
   periastron leg is measured in units of the periastron radius rho R, so it
   is scaled by rho when expressed in units of R (the time-unit form of
   Eq. 17). */
double orc_tp(double u, double alpha)
{
    if (alpha <= HALF_PI) return tp_out(u, alpha);
    double rho = orc_rho(u, alpha);
    return 2.0 * rho * tp_out(u / rho, HALF_PI) - tp_out(u, PI - alpha);
}

double orc_dpsi_dalpha(double u, double alpha)
{
    if (alpha <= HALF_PI) return dpsi_out(u, alpha);
    /* inward branch: five-point central difference of the (smooth) psi */
    double h = 1e-4;
    double amax = orc_alpha_capture(u);
    if (alpha + 2 * h >= amax) h = 0.25 * (amax - alpha);
    return (orc_psi(u, alpha - 2 * h) - 8 * orc_psi(u, alpha - h) + 8 * orc_psi(u, alpha + h)
            - orc_psi(u, alpha + 2 * h)) / (12 * h);
}

/* ------------------------------------------------------------------------ */
/* Brent root finding on [a, b] for g(x) - target.                           */
/* ------------------------------------------------------------------------ */
typedef struct { double u, target; } inv_ctx;

static double brent(double (*g)(double, const inv_ctx *), const inv_ctx *ctx, double a, double b)
{
    double fa = g(a, ctx) - ctx->target, fb = g(b, ctx) - ctx->target;
    if (fa == 0.0) return a;
    if (fb == 0.0) return b;
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 200; ++it) {
        if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) { c = a; fc = fa; d = e = b - a; }
        if (fabs(fc) < fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
        double tol = 2.0 * 2.2e-16 * fabs(b) + 1e-300;
        double m = 0.5 * (c - b);
        if (fabs(m) <= tol || fb == 0.0) return b;
        if (fabs(e) >= tol && fabs(fa) > fabs(fb)) {
            double s = fb / fa, p, q;
            if (a == c) { p = 2.0 * m * s; q = 1.0 - s; }
            else {
                double qq = fa / fc, r = fb / fc;
                p = s * (2.0 * m * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) q = -q; else p = -p;
            if (2.0 * p < fmin(3.0 * m * q - fabs(tol * q), fabs(e * q))) { e = d; d = p / q; }
            else { d = m; e = m; }
        } else { d = m; e = m; }
        a = b; fa = fb;
        b += (fabs(d) > tol) ? d : (m > 0 ? tol : -tol);
        fb = g(b, ctx) - ctx->target;
    }
    return b;
}

static double g_psi(double a, const inv_ctx *c) { return orc_psi(c->u, a); }

/* Inverse of the bending map (Sect. 2.3): the emission angle alpha whose ray
   reaches the observer at angle psi from the radial direction, with
   LF = d cos(alpha) / d cos(psi) = (sin a / sin psi) / (d psi / d alpha)
   and s = sin(alpha)/sin(psi) (limit d alpha/d psi at psi = 0).
   Returns 0 when psi exceeds psi(alpha_max). */
int orc_invert(double u, double alpha_max, double psi, double out[4])
{
    const double psi_small = 1e-7;
    if (psi < psi_small) {
        /* sub-observer limit: alpha = psi sqrt(1-u) + O(psi^3) */
        double dadpsi = sqrt(1.0 - u);
        double a = psi * dadpsi;
        out[0] = a; out[1] = cos(a); out[2] = dadpsi * dadpsi; out[3] = dadpsi;
        return 1;
    }
    double ptop = orc_psi(u, alpha_max);
    if (psi > ptop) return 0;
    inv_ctx ctx = {u, psi};
    double phalf = psi_out(u, HALF_PI);
    double a;
    if (alpha_max <= HALF_PI || psi <= phalf)
        a = brent(g_psi, &ctx, 0.0, fmin(HALF_PI, alpha_max));
    else
        a = brent(g_psi, &ctx, HALF_PI, alpha_max);
    double sr = sin(a) / sin(psi);
    out[0] = a; out[1] = cos(a); out[2] = sr / orc_dpsi_dalpha(u, a); out[3] = sr;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Star and rings (Sects. 2.1, 2.2, 2.4)                                      */
/* ------------------------------------------------------------------------ */
void orc_star_setup(const orc_spec *s, const double *p, orc_star *st)
{
    st->GM = p[0] * GM_SUN;
    st->Re = p[1] * 1e5;
    st->Rs = 2.0 * st->GM / (C_CGS * C_CGS);
    st->x = st->GM / (C_CGS * C_CGS * st->Re);                    /* Eq. (8) */
    st->Obar = TWO_PI * p[5] * sqrt(st->Re * st->Re * st->Re / st->GM);
    st->o2 = (s->mode == 1) ? st->Obar * st->Obar * (-0.788 + 1.030 * st->x) : 0.0; /* Eq. (7) */
    st->g0 = st->GM / (st->Re * st->Re) / sqrt(1.0 - st->Rs / st->Re);       /* Eq. (11) */
    st->D = p[6] * PC_CM;
    st->nu = p[5];
    st->incl = p[2];
    st->NH = p[4] * 1e20;
}

/* Eq. (10): effective gravity over g0 on the OS surface (1 for S+D) */
static double gravity_ratio(const orc_star *st, int mode, double th)
{
    if (mode != 1) return 1.0;
    double x = st->x, O2 = st->Obar * st->Obar, O4 = O2 * O2, O6 = O4 * O2;
    double s2 = sin(th) * sin(th), c = cos(th), c2 = c * c;
    double e4 = O4 * (13.47 * x - 27.13 * x * x);
    return 1.0
        + s2 * (O2 * (-0.791 + 0.776 * x) + O4 * (-1.315 * x + 2.431 * x * x) + O6 * (-1.172 * x))
        + c2 * (O2 * (1.138 - 1.431 * x) + O4 * (0.653 * x - 2.864 * x * x) + O6 * (0.975 * x) - e4)
        + fabs(c) * e4;
}

/* half-width in azimuth of the intersection of the ring at colatitude th with
   the cap of angular radius z centred at colatitude tc: pi when the ring lies
   inside the cap, 0 when it misses it */
static double arc_halfwidth(double th, double tc, double z)
{
    double den = sin(th) * sin(tc);
    double num = cos(z) - cos(th) * cos(tc);
    if (den <= 0.0) return (num <= 0.0) ? PI : 0.0;
    double a = num / den;
    if (a <= -1.0) return PI;
    if (a >= 1.0) return 0.0;
    return acos(a);
}

/* Spot-local iso-colatitude rings: N_r rings with uniform edges in theta
   over the spot's colatitude span, N_phi cells per ring over the emitting
   arc(s).  The area element is Eq. (9) (Eq. 6 for a sphere); the per-ring
   quantities are Eqs. (2)-(3), (7), (10)-(11), (18). */
/* Geometry of the ring at colatitude th (Eqs. 2, 3, 7, 9-11, 18): radius,
   compactness, surface tilt, log g, surface speed and the largest emission
   angle of its deflection table. */
static void ring_geometry(const orc_spec *s, const orc_star *st, double th, orc_ring *g)
{
    g->theta = th;
    double ct = cos(th), sn = sin(th);
    g->R = st->Re * (1.0 + st->o2 * ct * ct);
    double dR = -2.0 * st->Re * st->o2 * ct * sn;
    g->u = st->Rs / g->R;
    g->f = dR / (g->R * sqrt(1.0 - g->u));
    g->coseta = 1.0 / sqrt(1.0 + g->f * g->f);
    g->sineta = g->f / sqrt(1.0 + g->f * g->f);
    g->logg = log10(st->g0 * gravity_ratio(st, s->mode, th));
    g->beta = TWO_PI * st->nu * g->R * sn / (C_CGS * sqrt(1.0 - g->u));
    g->gamma = 1.0 / sqrt(1.0 - g->beta * g->beta);
    double amax = HALF_PI + fabs(atan(g->f));
    double acap = orc_alpha_capture(g->u);
    if (amax > acap - 1e-6) amax = acap - 1e-6;
    g->alpha_max = amax;
    g->psi_top = orc_psi(g->u, amax);
}

int orc_rings(const orc_spec *s, const double *p, int spot, orc_ring *rings)
{
    orc_star st;
    orc_star_setup(s, p, &st);
    double tc = p[8 + 4 * spot], z = p[9 + 4 * spot];
    int nr = s->n_rings[spot], nphi = s->n_phi[spot];
    double lo = fmax(0.0, tc - z), hi = fmin(PI, tc + z);
    for (int r = 0; r < nr; ++r) {
        orc_ring *g = &rings[r];
        double e0 = lo + (hi - lo) * r / nr, e1 = lo + (hi - lo) * (r + 1) / nr;
        double th = 0.5 * (e0 + e1);
        ring_geometry(s, &st, th, g);
        g->dcos = cos(e0) - cos(e1);
        if (s->shape[spot] == 1) {
            g->dphi_out = arc_halfwidth(th, tc, z);
            g->dphi_in = arc_halfwidth(th, tc, s->shape_a[spot] * z);
            g->dphi_cell = (g->dphi_out - g->dphi_in) / (0.5 * nphi);
        } else {
            g->dphi_out = arc_halfwidth(th, tc, z);
            g->dphi_in = 0.0;
            g->dphi_cell = 2.0 * g->dphi_out / nphi;
        }
        g->w_cell = g->R * g->R * sqrt(1.0 + g->f * g->f) * g->dcos * g->dphi_cell / (st.D * st.D);
        g->n_cells = nphi;
    }
    return nr;
}

/* HEALPix ring i = 1 .. 4 nside - 1 (Sect. 2.8.1): cosine of its
   colatitude, its number of pixels and the azimuth of its first pixel; the
   pixels of a ring are 2 pi / nphi apart.  Rings south of the equator mirror
   those north of it. */
void orc_healpix_ring(int nside, int i, double *z, int *nphi, double *phi_first)
{
    int m = i > 2 * nside ? 4 * nside - i : i;   /* northern counterpart */
    double n = nside;
    double zz;
    if (m < nside) {
        zz = 1.0 - (double)m * m / (3.0 * n * n);
        *nphi = 4 * m;
        *phi_first = PI / (2.0 * m) * 0.5;
    } else {
        zz = 4.0 / 3.0 - 2.0 * m / (3.0 * n);
        *nphi = 4 * nside;
        *phi_first = PI / (2.0 * n) * (1.0 - ((m - nside + 1) % 2) / 2.0);
    }
    *z = i > 2 * nside ? -zz : zz;
}

/* azimuth offset of cell j on ring g relative to the spot centre */
static double cell_offset(const orc_spec *s, int spot, const orc_ring *g, int j)
{
    int nphi = s->n_phi[spot];
    if (s->shape[spot] == 1) {
        int h = nphi / 2;
        if (j < h) return -(g->dphi_in + (h - 1 - j + 0.5) * g->dphi_cell);
        return g->dphi_in + (j - h + 0.5) * g->dphi_cell;
    }
    return -g->dphi_out + (j + 0.5) * g->dphi_cell;
}

/* crescent: cells whose centre lies inside the masking cap emit nothing */
static int cell_masked(const orc_spec *s, const double *p, int spot, const orc_ring *g, double dphi)
{
    if (s->shape[spot] != 2) return 0;
    double tc = p[8 + 4 * spot], z = p[9 + 4 * spot];
    double sgn = (tc >= HALF_PI) ? 1.0 : -1.0;
    double tm = tc - sgn * s->shape_b[spot] * z;
    double zm = s->shape_a[spot] * z;
    double cd = cos(g->theta) * cos(tm) + sin(g->theta) * sin(tm) * cos(dphi);
    return cd > cos(zm);
}

/* Eq. (16): extra light-travel distance from radius R out to R_e */
double orc_cdt_oblate(const orc_star *st, double R)
{
    return st->Re - R + st->Rs * log((st->Re - st->Rs) / (R - st->Rs));
}

/* Total delay c dt / R: Eq. (35) plus Eq. (16) for outgoing rays, Eq. (17)
   for inward rays (periastron leg scaled by rho, see orc_tp). */
double orc_total_delay(const orc_star *st, double R, double u, double alpha)
{
    if (alpha <= HALF_PI) return orc_tp(u, alpha) + orc_cdt_oblate(st, R) / R;
    double rho = orc_rho(u, alpha);
    return orc_tp(u, alpha) + (2.0 * orc_cdt_oblate(st, rho * R) - orc_cdt_oblate(st, R)) / R;
}

/* ------------------------------------------------------------------------ */
/* Pseudo-patch fine-phase trace (Sect. 2.8.3, Eqs. 38-44)                   */
/* ------------------------------------------------------------------------ */
int orc_trace_ring(const orc_spec *s, const double *p, const orc_ring *g,
                   double *F, double *z, double *phio, double *mu, int *inv_range,
                   orc_diag *diag)
{
    orc_star st;
    orc_star_setup(s, p, &st);
    int nfp = s->n_fp;
    double si = sin(st.incl), ci = cos(st.incl);
    double sth = sin(g->theta), cth = cos(g->theta);
    double sq = sqrt(1.0 - g->u);
    int imin = nfp, imax = 0;
    int ring_visible = 1;
    for (int ifp = 0; ifp <= nfp; ++ifp) {
        double phi = TWO_PI * ifp / nfp;
        double cpsi = si * sth * cos(phi) + ci * cth;                 /* Table 2 */
        if (cpsi > 1.0) cpsi = 1.0;
        if (cpsi < -1.0) cpsi = -1.0;
        double psi = acos(cpsi);
        double inv[4];
        int vis = orc_invert(g->u, g->alpha_max, psi, inv);
        double cs = -1.0, delta = 0.0, cxi = 0.0;
        if (vis) {
            double ca = inv[1], lf = inv[2], sr = inv[3];
            /* Eq. (4) / (39) */
            cs = ca * g->coseta + sr * g->sineta * (ci * sth - si * cth * cos(phi));
            if (cs > 0.0) {
                cxi = -sr * si * sin(phi);                              /* Table 2 */
                delta = 1.0 / (g->gamma * (1.0 - g->beta * cxi));       /* Eq. (19) */
                double m = delta * cs;                                  /* Eq. (20) */
                F[ifp] = sq * delta * delta * delta * m * lf * g->gamma; /* Eq. (40) */
                z[ifp] = 1.0 / (delta * sq);
                double cdt = g->R * orc_total_delay(&st, g->R, g->u, inv[0]);
                phio[ifp] = phi / TWO_PI + st.nu * cdt / C_CGS;
                mu[ifp] = m;
                if (diag && g->psi_top > PI && psi > TWO_PI - g->psi_top) diag->n_multi_image++;
            }
        }
        if (!vis || cs <= 0.0) {
            if (ifp == 0) ring_visible = 0;
            if (ifp < imin) imin = ifp;
            if (ifp > imax) imax = ifp;
            F[ifp] = 0.0; z[ifp] = 0.0; phio[ifp] = 0.0; mu[ifp] = 0.0;
        }
    }
    inv_range[0] = imin; inv_range[1] = imax;
    if (!ring_visible) return 0;
    if (imin <= imax) {
        /* Eqs. (41)-(44): zero flux and mu, linear fill of z and phi_o */
        int a = imin - 1, b = imax + 1 > nfp ? nfp : imax + 1;   /* sample n_fp repeats sample 0 */
        for (int i = imin; i <= imax; ++i) {
            double t = (double)(i - a) / (double)(b - a);
            F[i] = 0.0; mu[i] = 0.0;
            z[i] = z[a] + (z[b] - z[a]) * t;
            phio[i] = phio[a] + (phio[b] - phio[a]) * t;
        }
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Intensities                                                                */
/* ------------------------------------------------------------------------ */
/* App. C, Eq. (C.5): blackbody photon-energy intensity in the comoving frame */
double orc_blackbody(double E, double T)
{
    return 2.0 * E * E * E / (H_KEVS * H_KEVS * H_KEVS * C_CGS * C_CGS) / expm1(E / (K_B * T));
}

/* linear weights, value clamped into the axis range */
static int lin_w(const double *ax, int n, double v, double w[2], long long *clamp)
{
    if (v <= ax[0]) { if (v < ax[0] && clamp) (*clamp)++; w[0] = 1.0; w[1] = 0.0; return 0; }
    if (v >= ax[n - 1]) { if (v > ax[n - 1] && clamp) (*clamp)++; w[0] = 0.0; w[1] = 1.0; return n - 2; }
    int i = 0;
    while (ax[i + 1] <= v) ++i;
    double t = (v - ax[i]) / (ax[i + 1] - ax[i]);
    w[0] = 1.0 - t; w[1] = t;
    return i;
}

/* cubic Lagrange weights on nodes ax[i-1..i+2] */
static void lagrange4(const double *ax, int i, double v, double w[4])
{
    for (int a = 0; a < 4; ++a) {
        double num = 1.0, den = 1.0;
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
            num *= v - ax[i - 1 + b];
            den *= ax[i - 1 + a] - ax[i - 1 + b];
        }
        w[a] = num / den;
    }
}

/* interval index with ax[i] <= v < ax[i+1] (v inside the axis) */
static int find_interval(const double *ax, int n, double v)
{
    if (v >= ax[n - 1]) return n - 2;
    int i = 0;
    while (ax[i + 1] <= v) ++i;
    return i;
}

/* Four-node Lagrange weights on nodes ax[s0 .. s0+3] at v. */
static void lagrange_at(const double *ax, int s0, double v, double w[4])
{
    for (int a = 0; a < 4; ++a) {
        double num = 1.0, den = 1.0;
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
            num *= v - ax[s0 + b];
            den *= ax[s0 + a] - ax[s0 + b];
        }
        w[a] = num / den;
    }
}

/* Cubic stencil of one axis for v inside it: the four nodes around the
 * bracketing interval, shifted inward at the two ends of the axis.
 * Returns the first node. */
static int cubic_w(const double *ax, int n, double v, double w[4])
{
    int i = find_interval(ax, n, v);
    int s0 = i - 1;
    if (s0 < 0) s0 = 0;
    if (s0 > n - 4) s0 = n - 4;
    lagrange_at(ax, s0, v, w);
    return s0;
}

/* Clamp v to the axis, counting values outside it. */
static double clamp_axis(const double *ax, int n, double v, long long *clamp)
{
    if (v < ax[0]) { if (clamp) (*clamp)++; return ax[0]; }
    if (v > ax[n - 1]) { if (clamp) (*clamp)++; return ax[n - 1]; }
    return v;
}

/* Atmosphere interpolation (Sect. 4), in linear space (I/T^3); returns I/T^3.
 * mode 0, strategy (d), mixed order (the default):
 *   logT, log g : linear, clamped at the table edges;
 *   mu          : cubic Lagrange, linear in the protected zone spanned by the
 *                 four smallest-mu nodes and in the last interval; mu clamped
 *                 to [mu_0, mu_last];
 *   x=log(E/kT) : cubic Lagrange, linear in the first and last interval;
 *                 outside the axis the intensity is zero.
 * mode 1, strategy (a): cubic Lagrange on all four axes (logT, log g and mu
 *   clamped), the four-node stencil shifted inward at every axis end;
 * mode 2, strategy (b): mode 1 with negative results set to zero;
 * mode 3, strategy (c): mode 1 but linear in the protected small-mu zone.
 * In every mode x outside its axis gives zero. */
double orc_atmo_interp_mode(const orc_spec *s, const double *linI, double logT, double logg,
                            double mu, double x, int mode, orc_diag *diag)
{
    int nT = s->nT, ng = s->ng, nmu = s->nmu, nx = s->nx;
    double wT[4] = {0, 0, 0, 0}, wg[4] = {0, 0, 0, 0}, wm[4] = {0, 0, 0, 0}, wx[4] = {0, 0, 0, 0};
    int iT, ig;
    if (mode == 0) {
        iT = lin_w(s->ax_T, nT, logT, wT, diag ? &diag->n_clamp_T : NULL);
        ig = lin_w(s->ax_g, ng, logg, wg, diag ? &diag->n_clamp_g : NULL);
    } else {
        iT = cubic_w(s->ax_T, nT, clamp_axis(s->ax_T, nT, logT, diag ? &diag->n_clamp_T : NULL), wT);
        ig = cubic_w(s->ax_g, ng, clamp_axis(s->ax_g, ng, logg, diag ? &diag->n_clamp_g : NULL), wg);
    }
    if (x < s->ax_x[0] || x > s->ax_x[nx - 1]) {
        if (diag) diag->n_x_outside++;
        return 0.0;
    }
    double m = mu;
    if (m < s->ax_mu[0]) m = s->ax_mu[0];
    if (m > s->ax_mu[nmu - 1]) m = s->ax_mu[nmu - 1];
    int im = find_interval(s->ax_mu, nmu, m);
    int m0;
    int lin_mu = (mode == 0) ? (im < 3 || im == nmu - 2) : (mode == 3 ? im < 3 : 0);
    if (lin_mu) {
        double t = (m - s->ax_mu[im]) / (s->ax_mu[im + 1] - s->ax_mu[im]);
        m0 = im; wm[0] = 1.0 - t; wm[1] = t;
    } else if (mode == 0) {
        m0 = im - 1; lagrange4(s->ax_mu, im, m, wm);
    } else {
        m0 = cubic_w(s->ax_mu, nmu, m, wm);
    }
    int ix = find_interval(s->ax_x, nx, x);
    int x0;
    if (mode == 0 && (ix == 0 || ix == nx - 2)) {
        double t = (x - s->ax_x[ix]) / (s->ax_x[ix + 1] - s->ax_x[ix]);
        x0 = ix; wx[0] = 1.0 - t; wx[1] = t;
    } else if (mode == 0) {
        x0 = ix - 1; lagrange4(s->ax_x, ix, x, wx);
    } else {
        x0 = cubic_w(s->ax_x, nx, x, wx);
    }
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) {
        if (wT[a] == 0.0) continue;
        for (int b = 0; b < 4; ++b) {
            if (wg[b] == 0.0) continue;
            for (int c = 0; c < 4; ++c) {
                if (wm[c] == 0.0) continue;
                for (int d = 0; d < 4; ++d) {
                    if (wx[d] == 0.0) continue;
                    long long idx = (((long long)(iT + a) * ng + (ig + b)) * nmu + (m0 + c)) * nx + (x0 + d);
                    acc += wT[a] * wg[b] * wm[c] * wx[d] * linI[idx];
                }
            }
        }
    }
    if (acc < 0.0 && diag) diag->n_negative++;
    if (mode == 2 && acc < 0.0) acc = 0.0;
    return acc;
}

double orc_atmo(const orc_spec *s, const double *linI, double logT, double logg,
                double mu, double x, orc_diag *diag)
{
    return orc_atmo_interp_mode(s, linI, logT, logg, mu, x, s->interp, diag);
}

/* ------------------------------------------------------------------------ */
/* Forward model                                                             */
/* ------------------------------------------------------------------------ */
static void neumaier_add(double *sum, double *comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else *comp += (v - t) + *sum;
    *sum = t;
}

/* Shift-and-add of one ring (Eqs. 45-47) into Ft_sum/Ft_comp [P][E]. */
/* Shift-and-add of one ring (Eqs. 45-47) over the cells given by their
   azimuths phic[j] (the spot or map longitude including -2 pi Phi) and
   log10 temperatures logTc[j]: one fine-phase trace for the ring, then per
   cell, output phase and energy the phase lookup, the intensity at the
   cell's temperature and a compensated sum into Ft. */
static void ring_accumulate_cells(const orc_spec *s, const double *p, const orc_ring *g, int ncell,
                                  const double *phic, const double *logTc, const double *linI,
                                  double *sum, double *comp, orc_diag *diag)
{
    int nfp = s->n_fp, P = s->n_phase, E = s->n_energy;
    double *F = malloc(sizeof(double) * 4 * (nfp + 1));
    double *z = F + (nfp + 1), *phio = z + (nfp + 1), *mu = phio + (nfp + 1);
    int inv[2];
    orc_diag local = {0, 0, 0, 0, 0, 0, 0};
    if (ncell == 0 || !orc_trace_ring(s, p, g, F, z, phio, mu, inv, &local) || g->w_cell <= 0.0) {
        free(F);
        if (diag) {
#pragma omp atomic
            diag->n_multi_image += local.n_multi_image;
        }
        return;
    }
    for (int j = 0; j < ncell; ++j) {
        double logT = logTc[j];
        double T = pow(10.0, logT);
        double kT = K_B * T;
        for (int k = 0; k < P; ++k) {
            double Phik = (k + 0.5) / P;
            double a = Phik + phic[j] / TWO_PI + 1.0 - phio[0];
            double php = (a - floor(a)) + phio[0];                     /* Eq. (45) */
            int lo = 0, hi = nfp;                                      /* phio[lo] <= php */
            while (hi - lo > 1) {
                int mid = (lo + hi) / 2;
                if (phio[mid] <= php) lo = mid; else hi = mid;
            }
            if (lo > nfp - 1) lo = nfp - 1;
            double w = (php - phio[lo]) / (phio[lo + 1] - phio[lo]);
            if (w < 0.0) w = 0.0;
            if (w > 1.0) w = 1.0;
            double Fp = F[lo] + w * (F[lo + 1] - F[lo]);               /* Eq. (46) */
            if (Fp == 0.0) continue;
            double zp = z[lo] + w * (z[lo + 1] - z[lo]);
            double mup = mu[lo] + w * (mu[lo + 1] - mu[lo]);
            local.n_visible_pairs++;
            for (int e = 0; e < E; ++e) {
                double Ee = s->energy[e];
                double Ep = zp * Ee;
                double I;
                if (s->intensity == 0) I = orc_blackbody(Ep, T);
                else I = T * T * T * orc_atmo(s, linI, logT, g->logg, mup, log10(Ep / kT), &local);
                neumaier_add(&sum[(long long)k * E + e], &comp[(long long)k * E + e],
                             g->w_cell * Fp * I / Ee);                  /* Eq. (47) */
            }
        }
    }
    free(F);
    if (diag) {
#pragma omp critical(orc_diag)
        {
            diag->n_clamp_T += local.n_clamp_T;
            diag->n_clamp_g += local.n_clamp_g;
            diag->n_x_outside += local.n_x_outside;
            diag->n_multi_image += local.n_multi_image;
            diag->n_visible_pairs += local.n_visible_pairs;
            diag->n_negative += local.n_negative;
        }
    }
}

/* One spot ring: the unmasked cells at their offsets from the spot centre,
   all at the spot's temperature. */
static void ring_accumulate(const orc_spec *s, const double *p, int spot, const orc_ring *g,
                            const double *linI, double *sum, double *comp, orc_diag *diag)
{
    double *phic = malloc(sizeof(double) * 2 * (g->n_cells + 1));
    double *logTc = phic + g->n_cells + 1;
    double phis = -TWO_PI * (p[3] + (spot == 1 ? p[15] : 0.0));
    int n = 0;
    for (int j = 0; j < g->n_cells; ++j) {
        double off = cell_offset(s, spot, g, j);
        if (cell_masked(s, p, spot, g, off)) continue;
        phic[n] = phis + off;
        logTc[n] = p[10 + 4 * spot];
        ++n;
    }
    ring_accumulate_cells(s, p, g, n, phic, logTc, linI, sum, comp, diag);
    free(phic);
}

/* Runs ring(ctx, r, sum, comp) for r = 0 .. nring-1 (in parallel over
   rings) and adds the per-ring partials to Ft in a fixed ring order, so that
   the result does not depend on the thread count. */
typedef void (*ring_fn)(void *ctx, int r, double *sum, double *comp);

static void sum_rings(const orc_spec *s, int nring, ring_fn ring, void *ctx, double *Ft)
{
    int P = s->n_phase, E = s->n_energy;
    long long PE = (long long)P * E;
    double *tot = calloc(2 * PE, sizeof(double));
    const int CH = 32;
    double *part = malloc(sizeof(double) * 2 * PE * CH);
    for (int r0 = 0; r0 < nring; r0 += CH) {
        int nc = (nring - r0 < CH) ? nring - r0 : CH;
        memset(part, 0, sizeof(double) * 2 * PE * nc);
#pragma omp parallel for schedule(dynamic, 1)
        for (int r = 0; r < nc; ++r) ring(ctx, r0 + r, part + 2 * PE * r, part + 2 * PE * r + PE);
        for (int r = 0; r < nc; ++r)
            for (long long i = 0; i < PE; ++i) {
                neumaier_add(&tot[i], &tot[PE + i], part[2 * PE * r + i]);
                neumaier_add(&tot[i], &tot[PE + i], part[2 * PE * r + PE + i]);
            }
    }
    for (long long i = 0; i < PE; ++i) Ft[i] = tot[i] + tot[PE + i];
    free(part);
    free(tot);
}

/* Eq. (22) absorption and Eq. (55) fold, T_exp / P seconds per phase bin. */
static void fold_counts(const orc_spec *s, const double *p, const double *Ft, double *counts)
{
    int P = s->n_phase, E = s->n_energy, C = s->n_chan;
    double NH = p[4] * 1e20;
    for (int k = 0; k < P; ++k)
        for (int c = 0; c < C; ++c) {
            double acc = 0.0;
            for (int e = 0; e < E; ++e) {
                double att = s->sigma ? exp(-NH * s->sigma[e]) : 1.0;
                acc += Ft[(long long)k * E + e] * att * s->rsp[(long long)e * C + c];
            }
            counts[(long long)k * C + c] = s->t_exp / P * acc;
        }
}

static double *linear_table(const orc_spec *s)
{
    if (s->intensity != 1) return NULL;
    long long n = (long long)s->nT * s->ng * s->nmu * s->nx;
    double *linI = malloc(sizeof(double) * n);
    for (long long i = 0; i < n; ++i) linI[i] = pow(10.0, s->logI[i]);
    return linI;
}

typedef struct {
    const orc_spec *s;
    const double *p, *linI;
    const orc_ring *rings;
    const int *rspot;
    orc_diag *diag;
} spot_ctx;

static void spot_ring(void *c, int r, double *sum, double *comp)
{
    spot_ctx *x = (spot_ctx *)c;
    ring_accumulate(x->s, x->p, x->rspot[r], &x->rings[r], x->linI, sum, comp, x->diag);
}

int orc_forward(const orc_spec *s, const double *p, double *Ft, double *counts, orc_diag *diag)
{
    double *linI = linear_table(s);
    /* ring list over all spots */
    int nring = 0;
    for (int sp = 0; sp < s->n_spots; ++sp) nring += s->n_rings[sp];
    orc_ring *rings = malloc(sizeof(orc_ring) * nring);
    int *rspot = malloc(sizeof(int) * nring);
    int off = 0;
    for (int sp = 0; sp < s->n_spots; ++sp) {
        orc_rings(s, p, sp, rings + off);
        for (int r = 0; r < s->n_rings[sp]; ++r) rspot[off + r] = sp;
        off += s->n_rings[sp];
    }
    spot_ctx ctx = {s, p, linI, rings, rspot, diag};
    sum_rings(s, nring, spot_ring, &ctx, Ft);
    if (counts) fold_counts(s, p, Ft, counts);
    free(rings); free(rspot); free(linI);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Full-surface temperature map on HEALPix (Sects. 2.6, 2.8.1)              */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_spec *s;
    const double *p, *linI, *map;
    int nside;
    const orc_ring *rings;
    const long long *first_pix;
    orc_diag *diag;
} map_ctx;

static void map_ring(void *c, int r, double *sum, double *comp)
{
    map_ctx *x = (map_ctx *)c;
    const orc_ring *g = &x->rings[r];
    double zr, phi0;
    int nphi;
    orc_healpix_ring(x->nside, r + 1, &zr, &nphi, &phi0);
    double *phic = malloc(sizeof(double) * 2 * nphi);
    double *logTc = phic + nphi;
    int n = 0;
    for (int j = 0; j < nphi; ++j) {
        double lt = x->map[x->first_pix[r] + j];
        if (!(isfinite(lt) && lt > 0.0)) continue;                    /* inactive patch */
        phic[n] = -TWO_PI * x->p[3] + phi0 + j * (TWO_PI / nphi);
        logTc[n] = lt;
        ++n;
    }
    ring_accumulate_cells(x->s, x->p, g, n, phic, logTc, x->linI, sum, comp, x->diag);
    free(phic);
}

int orc_forward_map(const orc_spec *s, const double *p, int nside, const double *logT_map, double *Ft,
                    double *counts, orc_diag *diag)
{
    if (nside < 1) return -1;
    orc_star st;
    orc_star_setup(s, p, &st);
    double *linI = linear_table(s);
    int nring = 4 * nside - 1;
    orc_ring *rings = malloc(sizeof(orc_ring) * nring);
    long long *first = malloc(sizeof(long long) * nring);
    long long pix = 0;
    const double area = PI / (3.0 * (double)nside * nside);   /* d cos(theta) d phi of one patch */
    for (int r = 0; r < nring; ++r) {
        double zr, phi0;
        int nphi;
        orc_healpix_ring(nside, r + 1, &zr, &nphi, &phi0);
        orc_ring *g = &rings[r];
        ring_geometry(s, &st, acos(zr), g);
        g->dcos = 0.0;
        g->dphi_out = g->dphi_in = 0.0;
        g->dphi_cell = TWO_PI / nphi;
        g->w_cell = g->R * g->R * sqrt(1.0 + g->f * g->f) * area / (st.D * st.D);   /* Eq. (9) */
        g->n_cells = nphi;
        first[r] = pix;
        pix += nphi;
    }
    map_ctx ctx = {s, p, linI, logT_map, nside, rings, first, diag};
    sum_rings(s, nring, map_ring, &ctx, Ft);
    if (counts) fold_counts(s, p, Ft, counts);
    free(rings); free(first); free(linI);
    return 0;
}

/* Threads of the ring loop of orc_forward (timing only; results do not
 * depend on it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Poisson log-likelihood  sum d ln m - m - ln Gamma(d + 1). */
double orc_loglike_counts(const double *m, const int *d, long long n)
{
    double acc = 0.0;
    for (long long i = 0; i < n; ++i) {
        if (d[i] == 0) { acc -= m[i]; continue; }
        if (m[i] <= 0.0) return -INFINITY;
        acc += d[i] * log(m[i]) - m[i] - lgamma(d[i] + 1.0);
    }
    return acc;
}
