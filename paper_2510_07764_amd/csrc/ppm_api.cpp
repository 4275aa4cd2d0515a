// C-ABI of libppm: plan management, argument validation, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <initializer_list>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "../../include/ppm.h"
#include "ppm_internal.h"
#include "ppm_launch.h"

using namespace ppm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return PPM_ERR_HIP;
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on P_n).
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   // (2/((1-z^2) P'^2)) / 2
    }
}

bool uniform_axis(const double *a, int n, double &x0, double &h)
{
    if (n < 2) return false;
    x0 = a[0];
    h = (a[n - 1] - a[0]) / (n - 1);
    if (!(h > 0.0)) return false;
    for (int i = 0; i < n; ++i)
        if (std::fabs(a[i] - (x0 + h * i)) > 1e-9 * std::fabs(h) * n) return false;
    return true;
}

}  // namespace

namespace ppm {
// error reporting shared with the other host sources of the library
int api_fail(int code, const char *msg) { return fail(code, msg); }
int api_hip_fail(hipError_t e, const char *where) { return hip_fail(e, where); }
}  // namespace ppm

// Work lists of one batch layout (B, per-instance grids, ring-group size):
// the live (instance, ring) slots and the ring groups of every workspace
// pass, resident in device memory.  A plan keeps kListSlots of them; a call
// whose layout is resident reuses it, another one is built on the host and
// uploaded on the caller's stream into the least recently used slot.  A
// slot used while the stream is being captured into a HIP graph is pinned:
// never rewritten, so that the graph keeps reading the lists it was
// captured with.
constexpr int kListSlots = 8;

struct ListPass {
    int inst0, nb;            // instances [inst0, inst0 + nb) of the batch
    int ring_off, n_ring;     // their live rings in d_ring (pass-local instance index * R_tot + ring)
    int grp_off, n_grp;       // their ring groups in d_glist (first pass-local ring position, count)
};

struct ListSlot {
    int32_t *d_ring = nullptr;    // [max_batch * R_tot]
    int32_t *d_glist = nullptr;   // [max_batch * R_tot][2]
    int32_t *d_grange = nullptr;  // [max_batch][2] per instance: its groups [first, end) within its pass
    int32_t *d_ncells = nullptr;  // [max_batch] per-instance grids (override layouts)
    std::vector<ListPass> pass;
    std::vector<int32_t> key;     // per-instance grids (empty: the spec's own)
    int B = -1, group = 0;
    bool override_grid = false;
    bool pinned = false;
    uint64_t used = 0;
};

struct ppm_plan {
    DevSpec S;
    Workspace W;
    int max_batch = 0;
    int max_cells = 0;
    int device = -1;               // the device the plan's memory lives on
    int chunk = 0;                 // largest number of instances per workspace pass (ring scratch)
    size_t gcap = 0;               // ring-group partial spectra the workspace holds per pass
    int precision = PPM_F32;
    bool grad = false;             // gradient buffers allocated
    bool count_negative = false;   // the forward counts negative interpolated intensities
    std::vector<void *> allocs;
    ListSlot slot[kListSlots];
    ListSlot *cur = nullptr;       // layout of the last call
    int32_t *h_stage = nullptr;    // pinned staging of list uploads
    size_t stage_ints = 0;
    hipEvent_t stage_ev = nullptr; // recorded after the last upload from h_stage
    bool stage_pending = false;
    uint64_t clock = 0;
    int last_B = 0;
    // hot-kernel timing: one event pair per recorded call
    std::vector<hipEvent_t> ev;
    int prof_cap = 0, prof_n = 0;
    bool prof_on = false;

    template <typename T>
    T *dalloc(size_t n)
    {
        if (n == 0) return nullptr;
        void *p = nullptr;
        if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return static_cast<T *>(p);
    }
    template <typename T>
    T *upload(const T *host, size_t n)
    {
        T *d = dalloc<T>(n);
        if (d && hipMemcpy(d, host, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        return d;
    }
    void events(hipEvent_t &a, hipEvent_t &b)
    {
        a = b = nullptr;
        if (!prof_on || prof_n >= prof_cap) return;
        a = ev[2 * prof_n];
        b = ev[2 * prof_n + 1];
        ++prof_n;
    }
    ~ppm_plan()
    {
        if (stage_ev) {
            (void)hipEventSynchronize(stage_ev);
            (void)hipEventDestroy(stage_ev);
        }
        if (h_stage) (void)hipHostFree(h_stage);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }
};

bool ppm::plan_view(const ppm_plan *pl, const DevSpec **S, const Workspace **W, int *max_batch, int *device)
{
    if (!pl) return false;
    *S = &pl->S;
    *W = &pl->W;
    *max_batch = pl->max_batch;
    *device = pl->device;
    return true;
}

extern "C" {

int ppm_version(void) { return 2; }

const char *ppm_last_error(void) { return g_last_error.c_str(); }

const char *ppm_status_string(int code)
{
    switch (code) {
    case PPM_OK: return "ok";
    case PPM_ERR_ARG: return "invalid argument";
    case PPM_ERR_BATCH: return "batch size outside [1, max_batch]";
    case PPM_ERR_HIP: return "HIP runtime error";
    case PPM_ERR_UNSUPPORTED: return "unsupported spec";
    case PPM_ERR_ALLOC: return "device allocation failed";
    default: return "unknown status";
    }
}

int ppm_validate_params(const double *params_host, int B, int n_spots, int32_t *status_host)
{
    if (!params_host || !status_host || B < 1 || n_spots < 0 || n_spots > 2)
        return fail(PPM_ERR_ARG, "ppm_validate_params: bad arguments");
    for (int b = 0; b < B; ++b) status_host[b] = validate_params(params_host + (size_t)b * PPM_NPARAM, n_spots);
    return PPM_OK;
}

int ppm_plan_create(const ppm_spec *sp, int max_batch, int max_cells, ppm_plan **out)
{
    if (!sp || !out) return fail(PPM_ERR_ARG, "ppm_plan_create: null pointer");
    *out = nullptr;
    if (max_batch < 1) return fail(PPM_ERR_ARG, "max_batch must be >= 1");
    const bool map_plan = sp->n_side != 0;
    if (map_plan) {
        if (sp->n_side < 1 || sp->n_side > 512) return fail(PPM_ERR_ARG, "n_side must lie in [1, 512]");
        if (sp->intensity != PPM_I_TABLE || sp->precision != PPM_F32 || sp->interp != PPM_INTERP_MIXED
            || sp->grad)
            return fail(PPM_ERR_UNSUPPORTED,
                        "temperature maps need the atmosphere table, FP32, the mixed strategy and no gradient");
        if (max_cells != 0) return fail(PPM_ERR_ARG, "max_cells does not apply to temperature maps");
    }
    if (!map_plan && (sp->n_spots < 1 || sp->n_spots > 2)) return fail(PPM_ERR_ARG, "n_spots must be 1 or 2");
    if (sp->mode != PPM_MODE_SD && sp->mode != PPM_MODE_OS) return fail(PPM_ERR_ARG, "bad mode");
    if (sp->intensity != PPM_I_BLACKBODY && sp->intensity != PPM_I_TABLE) return fail(PPM_ERR_ARG, "bad intensity");
    if (sp->precision != PPM_F32 && sp->precision != PPM_F64) return fail(PPM_ERR_ARG, "bad precision");
    if (sp->precision == PPM_F64 && sp->intensity != PPM_I_BLACKBODY)
        return fail(PPM_ERR_UNSUPPORTED, "FP64 precision is implemented for the blackbody model only");
    for (int s = 0; s < (map_plan ? 0 : sp->n_spots); ++s) {
        if (sp->shape[s] < 0 || sp->shape[s] > 2) return fail(PPM_ERR_ARG, "bad spot shape");
        if (sp->n_rings[s] < 1 || sp->n_phi[s] < 1) return fail(PPM_ERR_ARG, "spot grid must be >= 1x1");
        if (sp->shape[s] == PPM_SHAPE_ANNULUS && (sp->n_phi[s] % 2))
            return fail(PPM_ERR_ARG, "annulus needs an even number of cells per ring");
        if (sp->shape[s] != PPM_SHAPE_CAP && !(sp->shape_a[s] > 0.0 && sp->shape_a[s] < 1.0))
            return fail(PPM_ERR_ARG, "annulus / crescent ratio must lie in (0, 1)");
        if (max_cells > 0 && sp->shape[s] == PPM_SHAPE_ANNULUS && (max_cells % 2))
            return fail(PPM_ERR_ARG, "max_cells must be even with an annulus");
    }
    if (sp->n_fp < 4 || sp->n_phase < 1 || sp->n_energy < 1 || sp->n_chan < 1)
        return fail(PPM_ERR_ARG, "n_fp >= 4, n_phase, n_energy, n_chan >= 1 required");
    if (!sp->energy_kev || !sp->rsp) return fail(PPM_ERR_ARG, "energy and rsp are required");
    for (int e = 0; e < sp->n_energy; ++e) {
        if (!(sp->energy_kev[e] > 0.0)) return fail(PPM_ERR_ARG, "energies must be positive");
        if (e && !(sp->energy_kev[e] > sp->energy_kev[e - 1])) return fail(PPM_ERR_ARG, "energies must increase");
    }
    if (!(sp->t_exp > 0.0)) return fail(PPM_ERR_ARG, "t_exp must be positive");
    if (sp->n_alpha < 64 || sp->n_alpha > 8192) return fail(PPM_ERR_ARG, "n_alpha must lie in [64, 8192]");
    if (sp->n_energy > 64 * 8) return fail(PPM_ERR_UNSUPPORTED, "at most 512 energies");
    if (sp->grad != 0 && sp->grad != 1) return fail(PPM_ERR_ARG, "grad must be 0 or 1");
    if (sp->count_negative != 0 && sp->count_negative != 1) return fail(PPM_ERR_ARG, "count_negative must be 0 or 1");
    if (sp->count_negative && (sp->grad || map_plan || sp->intensity != PPM_I_TABLE))
        return fail(PPM_ERR_UNSUPPORTED,
                    "count_negative applies to forward-only spot plans with the atmosphere table");
    if (sp->interp < PPM_INTERP_MIXED || sp->interp > PPM_INTERP_CUBIC_LINMU)
        return fail(PPM_ERR_ARG, "interp must be one of the four strategies");
    if (sp->interp != PPM_INTERP_MIXED) {
        if (sp->intensity != PPM_I_TABLE) return fail(PPM_ERR_ARG, "interp applies to the atmosphere table only");
        if (sp->grad) return fail(PPM_ERR_UNSUPPORTED, "gradients are implemented for the mixed strategy (d) only");
        if (sp->nT < 4 || sp->ng < 4 || sp->nmu < 4 || sp->nx < 4)
            return fail(PPM_ERR_ARG, "cubic strategies need at least four nodes on every table axis");
    }
    if (sp->grad && sp->intensity != PPM_I_TABLE)
        return fail(PPM_ERR_UNSUPPORTED, "gradients are implemented for the atmosphere-table model only");
    double tmp0, tmp1;
    if (sp->intensity == PPM_I_TABLE) {
        if (!sp->ax_T || !sp->ax_g || !sp->ax_mu || !sp->ax_x || !sp->log_intensity)
            return fail(PPM_ERR_ARG, "table intensity needs axes and values");
        if (sp->nT < 2 || sp->ng < 2 || sp->nmu < 6 || sp->nmu > kMaxMu || sp->nx < 4)
            return fail(PPM_ERR_ARG, "atmosphere table too small (or more than 128 mu nodes)");
        if (!uniform_axis(sp->ax_T, sp->nT, tmp0, tmp1) || !uniform_axis(sp->ax_g, sp->ng, tmp0, tmp1)
            || !uniform_axis(sp->ax_x, sp->nx, tmp0, tmp1))
            return fail(PPM_ERR_UNSUPPORTED, "logT, log g and x axes must be uniformly spaced");
        for (int i = 1; i < sp->nmu; ++i)
            if (!(sp->ax_mu[i] > sp->ax_mu[i - 1])) return fail(PPM_ERR_ARG, "mu axis must increase");
    }

    ppm_plan *pl = new (std::nothrow) ppm_plan();
    if (!pl) return fail(PPM_ERR_ALLOC, "host allocation failed");
    if (hipGetDevice(&pl->device) != hipSuccess) {
        delete pl;
        return fail(PPM_ERR_HIP, "ppm_plan_create: no current HIP device");
    }
    DevSpec &S = pl->S;
    std::memset(&S, 0, sizeof(S));
    S.mode = sp->mode;
    S.intensity = sp->intensity;
    S.interp = sp->interp;
    S.n_spots = map_plan ? 1 : sp->n_spots;
    for (int s = 0; s < 2; ++s) {
        bool on = s < sp->n_spots;
        S.shape[s] = on && !map_plan ? sp->shape[s] : 0;
        S.shape_a[s] = on && !map_plan ? sp->shape_a[s] : 0.0;
        S.shape_b[s] = on && !map_plan ? sp->shape_b[s] : 0.0;
        S.n_rings_spec[s] = on ? sp->n_rings[s] : 0;
        S.n_phi_spec[s] = on ? sp->n_phi[s] : 0;
        int mx = on ? sp->n_rings[s] : 0;
        if (on && max_cells > mx) mx = max_cells;
        S.rings_max[s] = mx;
    }
    if (map_plan) {
        // the HEALPix rings of the whole surface form one ring list
        S.n_side = sp->n_side;
        S.n_pix = 12 * sp->n_side * sp->n_side;
        S.rings_max[0] = S.n_rings_spec[0] = 4 * sp->n_side - 1;
        S.n_phi_spec[0] = 4 * sp->n_side;
        S.rings_max[1] = S.n_rings_spec[1] = S.n_phi_spec[1] = 0;
    }
    S.R_tot = S.rings_max[0] + S.rings_max[1];
    S.n_fp = sp->n_fp;
    S.P = sp->n_phase;
    S.E = sp->n_energy;
    S.C = sp->n_chan;
    S.t_exp = sp->t_exp;
    S.n_alpha = sp->n_alpha;
    S.pt_fwd = kPhaseTile;
    S.pt_adj = kPhaseTile;
    S.ring_group = 1;
    pl->max_batch = max_batch;
    pl->max_cells = max_cells;
    pl->precision = sp->precision;
    pl->grad = sp->grad != 0;
    pl->count_negative = sp->count_negative != 0;

    // Gauss-Legendre rules of 20, 24, 32, 48 and 64 nodes, back to back
    std::vector<double> glx, glw;
    for (int n : {20, 24, 32, 48, 64}) {
        std::vector<double> x, w;
        gauss_legendre01(n, x, w);
        glx.insert(glx.end(), x.begin(), x.end());
        glw.insert(glw.end(), w.begin(), w.end());
    }
    S.n_quad = (int)glx.size();
    S.Pd = (double)S.P;
    S.fpb = 2.0 * S.n_fp;
    S.glx = pl->upload(glx.data(), glx.size());
    S.glw = pl->upload(glw.data(), glw.size());
    S.energy = pl->upload(sp->energy_kev, S.E);
    if (sp->sigma_cm2) S.sigma = pl->upload(sp->sigma_cm2, S.E);
    if (sp->background) {
        for (size_t i = 0; i < (size_t)S.P * S.C; ++i)
            if (!(sp->background[i] >= 0.0) || !std::isfinite(sp->background[i])) {
                delete pl;
                return fail(PPM_ERR_ARG, "background counts must be finite and >= 0");
            }
        S.bkg = pl->upload(sp->background, (size_t)S.P * S.C);
        if (!S.bkg) {
            delete pl;
            return fail(PPM_ERR_ALLOC, "background upload failed");
        }
    }
    {
        size_t n = (size_t)S.E * S.C;
        std::vector<float> r32(n);
        for (size_t i = 0; i < n; ++i) r32[i] = (float)sp->rsp[i];
        S.rsp32 = pl->upload(r32.data(), n);
        if (sp->precision == PPM_F64) S.rsp64 = pl->upload(sp->rsp, n);
        if (sp->grad) {
            std::vector<double> rt(n);
            for (int e = 0; e < S.E; ++e)
                for (int c = 0; c < S.C; ++c) rt[(size_t)c * S.E + e] = sp->rsp[(size_t)e * S.C + c];
            S.rspT64 = pl->upload(rt.data(), n);
        }
    }
    if (sp->intensity == PPM_I_TABLE) {
        S.nT = sp->nT; S.ng = sp->ng; S.nmu = sp->nmu; S.nx = sp->nx;
        S.T_end[0] = sp->ax_T[0];
        S.T_end[1] = sp->ax_T[S.nT - 1];
        S.g_end[0] = sp->ax_g[0];
        S.g_end[1] = sp->ax_g[S.ng - 1];
        uniform_axis(sp->ax_T, S.nT, S.T0, S.hT);
        uniform_axis(sp->ax_g, S.ng, S.g0, S.hg);
        uniform_axis(sp->ax_x, S.nx, S.x0, S.hx);
        // windowed accumulation: the energy grid spans r_span x intervals; the
        // per-ring window adds the redshift spread (z ratio <= (1+b)/(1-b) = 4
        // for surface speeds below 0.6 c) and the cubic stencil.
        S.tb0 = (std::log10(sp->energy_kev[0]) - S.x0) / S.hx;
        S.r_span = (std::log10(sp->energy_kev[S.E - 1]) - std::log10(sp->energy_kev[0])) / S.hx;
        S.ihx = 1.0 / S.hx;
        S.ixl = (float)(1.0 / (S.hx * std::log(10.0)));
        {
            std::vector<float> tbe(S.E);
            for (int e = 0; e < S.E; ++e)
                tbe[e] = (float)((std::log10(sp->energy_kev[e]) - std::log10(sp->energy_kev[0])) * S.ihx);
            S.tbe = pl->upload(tbe.data(), tbe.size());
            if (!S.tbe) {
                delete pl;
                return fail(PPM_ERR_ALLOC, "device allocation or upload failed");
            }
        }
        S.W_max = (int)std::ceil(S.r_span + std::log10(4.0) / S.hx) + 8;
        if (S.W_max > S.nx) S.W_max = S.nx;
        // the windowed kernel; the generic one also counts negative
        // interpolated intensities, and runs when the plan asks for that count
        S.fast = (S.r_span <= 59.0 && S.interp == PPM_INTERP_MIXED && !sp->count_negative) ? 1 : 0;
        if (map_plan) {
            if (!S.fast) {
                delete pl;
                return fail(PPM_ERR_UNSUPPORTED, "temperature maps need an energy grid spanning at most 59 x intervals");
            }
            // temperature buckets: the logT intervals plus kMapLow steps either side;
            // x window: the spot window widened by one logT step of kT
            S.map_nb = S.nT - 1 + 2 * kMapLow;
            int wm = S.W_max + (int)std::ceil(S.hT / S.hx) + 2;
            S.map_wm = (wm + 3) & ~3;
        }
        if (sp->grad && !S.fast) {
            delete pl;
            return fail(PPM_ERR_UNSUPPORTED, "gradients need an energy grid spanning at most 59 x intervals");
        }
        if (sp->grad) {
            // unit x buckets of the energies' offsets (the adjoint sums energy
            // moments per x interval from per-bucket prefix sums)
            std::vector<float> tau(S.E + 1);
            std::vector<int32_t> bk(65, S.E);
            int nmax = 0;
            for (int e = 0, h = 0; e < S.E; ++e) {
                const float t = (float)((std::log10(sp->energy_kev[e]) - std::log10(sp->energy_kev[0])) * S.ihx);
                const int he = (int)std::floor(t);
                while (h <= he && h < 65) bk[h++] = e;
                tau[e] = t - (float)he;
            }
            tau[S.E] = 2.0f;
            for (int h = 0; h < 64; ++h) nmax = std::max(nmax, bk[h + 1] - bk[h]);
            S.e_it = 0;
            while ((1 << S.e_it) <= nmax) ++S.e_it;
            if (S.e_it > 4) {
                delete pl;
                return fail(PPM_ERR_UNSUPPORTED, "gradients need at most 15 energies per x interval of the table");
            }
            S.ebkt = pl->upload(bk.data(), bk.size());
            S.etau = pl->upload(tau.data(), tau.size());
            if (!S.ebkt || !S.etau) {
                delete pl;
                return fail(PPM_ERR_ALLOC, "device allocation or upload failed");
            }
        }
        S.sub_stride = S.fast ? ((S.nmu * S.W_max + 3) & ~3) : S.nmu * S.nx;
        size_t n = (size_t)S.nT * S.ng * S.nmu * S.nx;
        std::vector<float> lin(n);
        for (size_t i = 0; i < n; ++i) lin[i] = (float)std::pow(10.0, sp->log_intensity[i]);
        S.atm = pl->upload(lin.data(), n);
        S.ax_mu = pl->upload(sp->ax_mu, S.nmu);
        const double *a = sp->ax_mu;
        const int nm = S.nmu;
        std::vector<double> cf(4 * (size_t)nm, 0.0);
        for (int lo = 0; lo < nm - 1; ++lo) {
            double *c = &cf[4 * (size_t)lo];
            if (lo < 3 || lo == nm - 2) {
                c[0] = 1.0 / (a[lo + 1] - a[lo]);
                continue;
            }
            const int m0 = lo - 1;
            for (int q = 0; q < 4; ++q) {
                double den = 1.0;
                for (int s = 0; s < 4; ++s)
                    if (s != q) den *= a[m0 + q] - a[m0 + s];
                c[q] = 1.0 / den;
            }
        }
        S.mu_coef = pl->upload(cf.data(), cf.size());
        S.mu_nb = 4 * nm;
        S.mu_lo = a[0];
        S.mu_hi = a[nm - 1];
        S.mu_ibw = S.mu_nb / (a[nm - 1] - a[0]);
        std::vector<int16_t> mb(S.mu_nb);
        for (int b = 0, l = 0; b < S.mu_nb; ++b) {
            const double edge = a[0] + b / S.mu_ibw;
            while (l < nm - 2 && a[l + 1] <= edge) ++l;
            mb[b] = (int16_t)l;
        }
        S.mu_bucket = pl->upload(mb.data(), mb.size());
    }
    // workspace: per-instance outputs and counters for max_batch instances;
    // ring-level scratch for `chunk` instances per pass (a 64 GiB budget of
    // the 288 GB bounds the chunk); ring-group partial spectra for `gcap`
    // groups per pass: the chunk at groups of 4 rings (as fast as one ring
    // per group for large batches, with a quarter of the partials), and at
    // least one instance at one ring per group
    Workspace &W = pl->W;
    std::memset(&W, 0, sizeof(W));
    const size_t R = S.R_tot;
    {
        size_t per_ring = sizeof(RingRec) + sizeof(double4) * (S.n_alpha + S.n_fp + 1)
                        + (S.intensity == PPM_I_TABLE && !map_plan ? sizeof(float) * (size_t)S.sub_stride : 0);
        if (map_plan) per_ring += sizeof(int32_t) * (size_t)(S.map_nb + 1);
        if (sp->grad)
            per_ring += sizeof(double4) * ((size_t)S.n_alpha + (size_t)(S.n_fp + 1) * 5) + sizeof(RingTan)
                      + sizeof(float2) * (size_t)S.sub_stride
                      + sizeof(double) * kGradAcc * (size_t)((S.P + kMinTileGrad - 1) / kMinTileGrad);
        const size_t part_bytes = (S.intensity == PPM_I_TABLE ? sizeof(float) : sizeof(double)) * (size_t)S.P * S.E;
        const size_t groups4 = (R + 3) / 4;
        size_t per_inst = per_ring * R + part_bytes * groups4 + sizeof(double) * (size_t)S.P * S.E
                        + (sp->grad ? (sizeof(double) + sizeof(float)) * (size_t)S.P * S.E : 0)
                        + (map_plan ? sizeof(MapCell) * (size_t)S.n_pix : 0);
        size_t budget = (size_t)64 << 30;
        size_t c = budget / per_inst;
        if (c < 1) c = 1;
        // PPM_MAX_CHUNK caps the instances per workspace pass (tests use it to
        // exercise multi-pass batches on small workloads)
        if (const char *env = std::getenv("PPM_MAX_CHUNK")) {
            long v = std::strtol(env, nullptr, 10);
            if (v >= 1 && (size_t)v < c) c = (size_t)v;
        }
        pl->chunk = (int)(c < (size_t)max_batch ? c : (size_t)max_batch);
        pl->gcap = std::max((size_t)pl->chunk * groups4, R);
        // PPM_PARTIAL_GROUPS sets the ring-group partials per pass (launch-shape studies)
        if (const char *env = std::getenv("PPM_PARTIAL_GROUPS")) {
            long v = std::strtol(env, nullptr, 10);
            if (v >= (long)R) pl->gcap = (size_t)v;
        }
    }
    const size_t B = pl->chunk, BM = max_batch;
    W.stars = pl->dalloc<StarRec>(BM);
    W.rings = pl->dalloc<RingRec>(B * R);
    W.table = pl->dalloc<double4>(B * R * S.n_alpha);
    W.trace = pl->dalloc<double4>(B * R * (S.n_fp + 1));
    W.vis_pairs = pl->dalloc<int32_t>(BM * R);
    W.diag = pl->dalloc<int32_t>(BM * R * kDiagFields);
    W.counts = pl->dalloc<double>(BM * S.P * S.C);
    W.ll_part = pl->dalloc<double>(BM * loglike_parts(S.P, S.C));
    W.ll_bad = pl->dalloc<int32_t>(BM * loglike_parts(S.P, S.C));
    {
        std::vector<double> lf(kLogFact);
        for (int d = 0; d < kLogFact; ++d) lf[d] = std::lgamma(d + 1.0);
        W.lfact = pl->upload(lf.data(), lf.size());
        std::vector<unsigned> z(BM, 0u);
        W.ll_done = pl->upload(z.data(), z.size());
    }
    bool ok = W.stars && W.rings && W.table && W.trace && W.vis_pairs && W.diag && W.counts && W.ll_part && W.ll_bad
              && W.lfact && W.ll_done && S.glx && S.glw && S.energy && S.rsp32;
    for (ListSlot &ls : pl->slot) {
        ls.d_ring = pl->dalloc<int32_t>(BM * R);
        ls.d_glist = pl->dalloc<int32_t>(2 * BM * R);
        ls.d_grange = pl->dalloc<int32_t>(2 * BM);
        ls.d_ncells = pl->dalloc<int32_t>(BM);
        ok = ok && ls.d_ring && ls.d_glist && ls.d_grange && ls.d_ncells;
    }
    pl->stage_ints = 3 * BM * R + 3 * BM;
    if (hipHostMalloc((void **)&pl->h_stage, sizeof(int32_t) * pl->stage_ints, hipHostMallocDefault) != hipSuccess)
        pl->h_stage = nullptr;
    if (hipEventCreateWithFlags(&pl->stage_ev, hipEventDisableTiming) != hipSuccess) pl->stage_ev = nullptr;
    ok = ok && pl->h_stage && pl->stage_ev;
    const size_t PEg = pl->gcap * S.P * S.E;
    if (S.intensity == PPM_I_TABLE) {
        if (map_plan) {
            W.mcell = pl->dalloc<MapCell>(B * (size_t)S.n_pix);
            W.mgrp = pl->dalloc<int32_t>(B * R * (size_t)(S.map_nb + 1));
            ok = ok && W.mcell && W.mgrp;
        } else {
            W.sub = pl->dalloc<float>(B * R * (size_t)S.sub_stride);
            ok = ok && W.sub;
        }
        W.partial32 = pl->dalloc<float>(PEg);
        W.fold_in32 = pl->dalloc<float>(B * S.P * S.E);
        ok = ok && W.partial32 && W.fold_in32 && S.atm && S.ax_mu && S.mu_coef && S.mu_bucket;
    } else {
        W.partial64 = pl->dalloc<double>(PEg);
        if (sp->precision == PPM_F64) {
            W.fold_in64 = pl->dalloc<double>(B * S.P * S.E);
            ok = ok && W.fold_in64 && S.rsp64;
        } else {
            W.fold_in32 = pl->dalloc<float>(B * S.P * S.E);
            ok = ok && W.fold_in32;
        }
        ok = ok && W.partial64;
    }
    if (sp->grad) {
        const size_t n_tile = (S.P + kMinTileGrad - 1) / kMinTileGrad;
        W.table_u = pl->dalloc<double4>(B * R * S.n_alpha);
        W.tangent = pl->dalloc<double4>(B * R * (S.n_fp + 1) * 5);
        W.ringtan = pl->dalloc<RingTan>(B * R);
        W.subtg = pl->dalloc<float2>(B * R * (size_t)S.sub_stride);
        W.flux = pl->dalloc<double>(B * S.P * S.E);
        W.gtil = pl->dalloc<float>(B * S.P * S.E);
        W.nh_part = pl->dalloc<double>(B * S.P * ((S.E + 15) / 16));
        W.gpart = pl->dalloc<double>(B * R * n_tile * kGradAcc);
        ok = ok && W.table_u && W.tangent && W.ringtan && W.subtg && W.flux && W.gtil && W.nh_part && W.gpart
           && S.rspT64;
    }
    if (!ok) {
        delete pl;
        return fail(PPM_ERR_ALLOC, "device allocation or upload failed");
    }
    if (map_plan && accum_map_lds(S) > 160 * 1024) {
        delete pl;
        return fail(PPM_ERR_UNSUPPORTED, "temperature-map working set does not fit in LDS");
    }
    if (S.intensity == PPM_I_TABLE && !map_plan) {
        size_t lds = accum_table_lds(S);
        if (lds > 160 * 1024) {
            delete pl;
            return fail(PPM_ERR_UNSUPPORTED, "atmosphere sub-table does not fit in LDS");
        }
        if (sp->grad && accum_adj_lds(S) > 160 * 1024) {
            delete pl;
            return fail(PPM_ERR_UNSUPPORTED, "adjoint working set does not fit in LDS");
        }
    }
    *out = pl;
    return PPM_OK;
}

void ppm_plan_destroy(ppm_plan *plan) { delete plan; }

// Rings the windowed spot accumulation sums per block; the generic,
// blackbody and map kernels take one ring per block.
static int plan_group(const ppm_plan *pl)
{
    const DevSpec &S = pl->S;
    return (S.intensity == PPM_I_TABLE && S.fast && S.n_side == 0) ? S.ring_group : 1;
}

static bool stream_capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs == hipStreamCaptureStatusActive;
}

// Validates the batch and makes its work lists resident (pl->cur): the
// live (instance, ring) slots and ring groups of every workspace pass, with
// the instances of a pass ordered larger grids first so that the longest
// blocks start early.  A pass holds at most pl->chunk instances and
// pl->gcap ring groups.  Uploads go on the caller's stream from pinned
// staging; the host waits only when the previous upload from the staging
// buffer has not run yet.
static int prepare(ppm_plan *pl, const double *params, int B, const int32_t *ncells_host, hipStream_t st,
                   bool map_call = false)
{
    if (!pl || !params) return fail(PPM_ERR_ARG, "null plan or params");
    if ((pl->S.n_side > 0) != map_call)
        return fail(PPM_ERR_ARG, map_call ? "plan has no temperature map (spec n_side = 0)"
                                          : "temperature-map plan: use the *_map entry points");
    if (B < 1 || B > pl->max_batch) return fail(PPM_ERR_BATCH, "batch outside [1, max_batch]");
    const DevSpec &S = pl->S;
    if (ncells_host) {
        for (int b = 0; b < B; ++b) {
            int n = ncells_host[b];
            if (n < 1) return fail(PPM_ERR_ARG, "per-instance grid must be >= 1");
            for (int s = 0; s < S.n_spots; ++s) {
                if (n > S.rings_max[s]) return fail(PPM_ERR_ARG, "per-instance grid exceeds the plan's max_cells");
                if (S.shape[s] == PPM_SHAPE_ANNULUS && (n % 2))
                    return fail(PPM_ERR_ARG, "annulus needs an even per-instance grid");
            }
        }
    }
    const int G = plan_group(pl);
    const bool over = ncells_host != nullptr;
    for (ListSlot &ls : pl->slot) {
        if (ls.B != B || ls.group != G || ls.override_grid != over) continue;
        if (over && std::memcmp(ls.key.data(), ncells_host, sizeof(int32_t) * B) != 0) continue;
        if (stream_capturing(st)) ls.pinned = true;
        ls.used = ++pl->clock;
        pl->cur = &ls;
        pl->last_B = B;
        return PPM_OK;
    }
    if (stream_capturing(st))
        return fail(PPM_ERR_ARG, "the work lists of this batch layout are not resident while the stream is being "
                                 "captured: make one call with the same B and per-instance grids first");
    ListSlot *v = nullptr;
    for (ListSlot &ls : pl->slot)
        if (!ls.pinned && (!v || ls.used < v->used)) v = &ls;
    if (!v) return fail(PPM_ERR_UNSUPPORTED, "every work-list slot of the plan is held by a captured graph");
    auto live_rings = [&](int b) {
        int n = 0;
        for (int s = 0; s < S.n_spots; ++s) n += ncells_host ? ncells_host[b] : S.n_rings_spec[s];
        return n;
    };
    std::vector<int32_t> ring, glist, grange(2 * (size_t)B);
    ring.reserve((size_t)B * S.R_tot);
    v->pass.clear();
    for (int c0 = 0; c0 < B;) {
        ListPass ps;
        ps.inst0 = c0;
        ps.ring_off = (int)ring.size();
        ps.grp_off = (int)(glist.size() / 2);
        size_t ng = 0;
        int nb = 0;
        while (c0 + nb < B && nb < pl->chunk) {
            const size_t gb = (size_t)(live_rings(c0 + nb) + G - 1) / G;
            if (nb > 0 && ng + gb > pl->gcap) break;
            ng += gb;
            ++nb;
        }
        ps.nb = nb;
        std::vector<std::pair<int, int>> order;   // (-cells, pass-local instance)
        for (int b = 0; b < nb; ++b) order.push_back({ncells_host ? -ncells_host[c0 + b] : 0, b});
        std::stable_sort(order.begin(), order.end());
        int rpos = 0, gpos = 0;
        for (auto &o : order) {
            const int b = o.second;
            const int r_first = rpos;
            grange[2 * (size_t)(c0 + b)] = gpos;
            for (int s = 0; s < S.n_spots; ++s) {
                const int nr = ncells_host ? ncells_host[c0 + b] : S.n_rings_spec[s];
                const int base = s == 0 ? 0 : S.rings_max[0];
                for (int r = 0; r < nr; ++r, ++rpos) ring.push_back(b * S.R_tot + base + r);
            }
            for (int f = r_first; f < rpos; f += G, ++gpos) {
                glist.push_back(f);
                glist.push_back(rpos - f < G ? rpos - f : G);
            }
            grange[2 * (size_t)(c0 + b) + 1] = gpos;
        }
        ps.n_ring = rpos;
        ps.n_grp = gpos;
        v->pass.push_back(ps);
        c0 += nb;
    }
    hipError_t e = hipSuccess;
    if (pl->stage_pending) {
        e = hipEventSynchronize(pl->stage_ev);
        if (e != hipSuccess) return hip_fail(e, "work-list staging");
        pl->stage_pending = false;
    }
    int32_t *h = pl->h_stage;
    const size_t nr = ring.size(), ngl = glist.size(), ngr = grange.size(), nnc = over ? (size_t)B : 0;
    std::memcpy(h, ring.data(), sizeof(int32_t) * nr);
    std::memcpy(h + nr, glist.data(), sizeof(int32_t) * ngl);
    std::memcpy(h + nr + ngl, grange.data(), sizeof(int32_t) * ngr);
    if (over) std::memcpy(h + nr + ngl + ngr, ncells_host, sizeof(int32_t) * nnc);
    // the slot is being rewritten: invalid until the uploads are queued
    v->B = -1;
    e = hipMemcpyAsync(v->d_ring, h, sizeof(int32_t) * nr, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(v->d_glist, h + nr, sizeof(int32_t) * ngl, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(v->d_grange, h + nr + ngl, sizeof(int32_t) * ngr, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && over)
        e = hipMemcpyAsync(v->d_ncells, h + nr + ngl + ngr, sizeof(int32_t) * nnc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(pl->stage_ev, st);
    if (e != hipSuccess) return hip_fail(e, "upload of the work lists");
    pl->stage_pending = true;
    if (over) v->key.assign(ncells_host, ncells_host + B);
    else v->key.clear();
    v->B = B;
    v->group = G;
    v->override_grid = over;
    v->pinned = false;
    v->used = ++pl->clock;
    pl->cur = v;
    pl->last_B = B;
    return PPM_OK;
}

// Workspace view of one pass of the current layout.
static Workspace pass_workspace(const ppm_plan *pl, const ListPass &ps)
{
    const DevSpec &S = pl->S;
    Workspace W = pl->W;
    W.stars += ps.inst0;
    W.vis_pairs += (size_t)ps.inst0 * S.R_tot;
    W.diag += (size_t)ps.inst0 * S.R_tot * kDiagFields;
    W.glist = pl->cur->d_glist + 2 * (size_t)ps.grp_off;
    W.grange = pl->cur->d_grange + 2 * (size_t)ps.inst0;
    W.ll_done += ps.inst0;
    return W;
}

// One forward pass over the batch, pass by pass; with data, the likelihood
// of every instance goes to logl (counts may then be NULL for FP32 plans).
static hipError_t run_forward(ppm_plan *pl, const double *params, hipStream_t st, double *flux, double *counts,
                              const int32_t *data = nullptr, double *logl = nullptr)
{
    const DevSpec &S = pl->S;
    const ListSlot &L = *pl->cur;
    for (const ListPass &ps : L.pass) {
        Workspace W = pass_workspace(pl, ps);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        pl->events(e0, e1);
        hipError_t e = launch_forward(S, W, params + (size_t)ps.inst0 * PPM_NPARAM,
                                      L.override_grid ? L.d_ncells + ps.inst0 : nullptr, ps.nb,
                                      L.d_ring + ps.ring_off, ps.n_ring, ps.n_grp, st,
                                      flux ? flux + (size_t)ps.inst0 * S.P * S.E : nullptr,
                                      counts ? counts + (size_t)ps.inst0 * S.P * S.C : nullptr, data,
                                      logl ? logl + ps.inst0 : nullptr, e0, e1);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One forward pass of a temperature-map plan over the batch, pass by pass.
static hipError_t run_forward_map(ppm_plan *pl, const double *params, const double *map, hipStream_t st,
                                  double *flux, double *counts, const int32_t *data = nullptr,
                                  double *logl = nullptr)
{
    const DevSpec &S = pl->S;
    const ListSlot &L = *pl->cur;
    for (const ListPass &ps : L.pass) {
        Workspace W = pass_workspace(pl, ps);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        pl->events(e0, e1);
        hipError_t e = launch_forward_map(S, W, params + (size_t)ps.inst0 * PPM_NPARAM,
                                          map + (size_t)ps.inst0 * S.n_pix, ps.nb, L.d_ring + ps.ring_off,
                                          ps.n_ring, ps.n_grp, st,
                                          flux ? flux + (size_t)ps.inst0 * S.P * S.E : nullptr,
                                          counts ? counts + (size_t)ps.inst0 * S.P * S.C : nullptr, data,
                                          logl ? logl + ps.inst0 : nullptr, e0, e1);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Model counts the likelihood path writes: the caller's buffer, else none
// for FP32 plans (the fold's epilogue computes logL from registers) and the
// plan's buffer for FP64 plans (their likelihood kernel reads counts).
static double *loglike_counts(ppm_plan *pl, double *counts_dev)
{
    return counts_dev ? counts_dev : (pl->S.rsp64 ? pl->W.counts : nullptr);
}

int ppm_forward_map(ppm_plan *pl, const double *params_dev, int B, const double *map_dev, double *counts_dev,
                    void *stream)
{
    int rc = prepare(pl, params_dev, B, nullptr, (hipStream_t)stream, true);
    if (rc) return rc;
    if (!map_dev || !counts_dev) return fail(PPM_ERR_ARG, "null map or counts buffer");
    hipError_t e = run_forward_map(pl, params_dev, map_dev, (hipStream_t)stream, nullptr, counts_dev);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_forward_map launch");
}

int ppm_flux_map(ppm_plan *pl, const double *params_dev, int B, const double *map_dev, double *flux_dev,
                 void *stream)
{
    int rc = prepare(pl, params_dev, B, nullptr, (hipStream_t)stream, true);
    if (rc) return rc;
    if (!map_dev || !flux_dev) return fail(PPM_ERR_ARG, "null map or flux buffer");
    hipError_t e = run_forward_map(pl, params_dev, map_dev, (hipStream_t)stream, flux_dev, pl->W.counts);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_flux_map launch");
}

int ppm_loglike_map(ppm_plan *pl, const double *params_dev, int B, const double *map_dev, const int32_t *data_dev,
                    double *logl_dev, double *counts_dev, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = prepare(pl, params_dev, B, nullptr, st, true);
    if (rc) return rc;
    if (!map_dev || !data_dev || !logl_dev) return fail(PPM_ERR_ARG, "null map, data or logl buffer");
    hipError_t e = run_forward_map(pl, params_dev, map_dev, st, nullptr, loglike_counts(pl, counts_dev), data_dev,
                                   logl_dev);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_loglike_map launch");
}

int ppm_forward(ppm_plan *pl, const double *params_dev, int B, const int32_t *n_cells_host,
                double *counts_dev, void *stream)
{
    int rc = prepare(pl, params_dev, B, n_cells_host, (hipStream_t)stream);
    if (rc) return rc;
    if (!counts_dev) return fail(PPM_ERR_ARG, "null counts buffer");
    hipError_t e = run_forward(pl, params_dev, (hipStream_t)stream, nullptr, counts_dev);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_forward launch");
}

int ppm_flux(ppm_plan *pl, const double *params_dev, int B, const int32_t *n_cells_host, double *flux_dev,
             void *stream)
{
    int rc = prepare(pl, params_dev, B, n_cells_host, (hipStream_t)stream);
    if (rc) return rc;
    if (!flux_dev) return fail(PPM_ERR_ARG, "null flux buffer");
    hipError_t e = run_forward(pl, params_dev, (hipStream_t)stream, flux_dev, pl->W.counts);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_flux launch");
}

int ppm_loglike(ppm_plan *pl, const double *params_dev, int B, const int32_t *n_cells_host,
                const int32_t *data_dev, double *logl_dev, double *counts_dev, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = prepare(pl, params_dev, B, n_cells_host, st);
    if (rc) return rc;
    if (!data_dev || !logl_dev) return fail(PPM_ERR_ARG, "null data or logl buffer");
    hipError_t e = run_forward(pl, params_dev, st, nullptr, loglike_counts(pl, counts_dev), data_dev, logl_dev);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_loglike launch");
}

// One forward + adjoint pass over the batch: per workspace pass the forward
// (keeping the pre-absorption flux), then the adjoint of the same instances
// while their ring scratch is live.  Model counts go to pl->W.counts.
static hipError_t run_grad(ppm_plan *pl, const double *params, const int32_t *data, double *logl, double *grad,
                           hipStream_t st, const char **what)
{
    const DevSpec &S = pl->S;
    const ListSlot &L = *pl->cur;
    for (const ListPass &ps : L.pass) {
        Workspace W = pass_workspace(pl, ps);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        pl->events(e0, e1);
        const double *pc = params + (size_t)ps.inst0 * PPM_NPARAM;
        const int32_t *ncc = L.override_grid ? L.d_ncells + ps.inst0 : nullptr;
        double *cc = pl->W.counts + (size_t)ps.inst0 * S.P * S.C;
        const int32_t *list = L.d_ring + ps.ring_off;
        hipError_t e = launch_forward(S, W, pc, ncc, ps.nb, list, ps.n_ring, ps.n_grp, st, W.flux, cc, data,
                                      logl + ps.inst0, e0, e1);
        if (e != hipSuccess) {
            *what = "ppm_loglike_grad forward";
            return e;
        }
        e = launch_grad(S, W, pc, ncc, ps.nb, list, ps.n_ring, cc, data, grad + (size_t)ps.inst0 * PPM_NGRAD, st);
        if (e != hipSuccess) {
            *what = "ppm_loglike_grad adjoint";
            return e;
        }
    }
    return hipSuccess;
}

int ppm_loglike_grad(ppm_plan *pl, const double *params_dev, int B, const int32_t *n_cells_host,
                     const int32_t *data_dev, double *logl_dev, double *grad_dev, void *stream)
{
    if (!pl) return fail(PPM_ERR_ARG, "null plan");
    if (!pl->grad) return fail(PPM_ERR_UNSUPPORTED, "plan created without gradient buffers (spec->grad = 0)");
    hipStream_t st = (hipStream_t)stream;
    int rc = prepare(pl, params_dev, B, n_cells_host, st);
    if (rc) return rc;
    if (!data_dev || !logl_dev || !grad_dev) return fail(PPM_ERR_ARG, "null data, logl or grad buffer");
    const char *what = "";
    hipError_t e = run_grad(pl, params_dev, data_dev, logl_dev, grad_dev, st, &what);
    return e == hipSuccess ? PPM_OK : hip_fail(e, what);
}

int ppm_get_diagnostics(ppm_plan *pl, int B, ppm_diag *total, ppm_diag *per_instance, void *stream)
{
    if (!pl || (!total && !per_instance)) return fail(PPM_ERR_ARG, "ppm_get_diagnostics: null argument");
    if (B < 1 || B > pl->max_batch) return fail(PPM_ERR_BATCH, "batch outside [1, max_batch]");
    const DevSpec &S = pl->S;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ppm_get_diagnostics sync");
    const size_t n = (size_t)B * S.R_tot;
    std::vector<int32_t> vp(n), dg(n * kDiagFields);
    e = hipMemcpy(vp.data(), pl->W.vis_pairs, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(dg.data(), pl->W.diag, sizeof(int32_t) * dg.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "ppm_get_diagnostics copy");
    // negative intensities are counted by the generic table kernel only
    const bool neg = S.intensity == PPM_I_TABLE && !S.fast;
    ppm_diag tot;
    std::memset(&tot, 0, sizeof(tot));
    for (int b = 0; b < B; ++b) {
        ppm_diag d;
        std::memset(&d, 0, sizeof(d));
        for (int r = 0; r < S.R_tot; ++r) {
            const size_t i = (size_t)b * S.R_tot + r;
            const int32_t *g = &dg[i * kDiagFields];
            const int64_t evals = (int64_t)vp[i] * S.E;
            d.n_visible_pairs += vp[i];
            if (g[0] & 1) d.n_clamp_T += evals;
            if (g[0] & 2) d.n_clamp_g += evals;
            d.n_clamp_T += (int64_t)g[4] * S.E;
            d.n_multi_image += g[1];
            d.n_x_outside += g[2];
            d.n_negative += g[3];
        }
        if (!neg) d.n_negative = -1;
        if (per_instance) per_instance[b] = d;
        tot.n_visible_pairs += d.n_visible_pairs;
        tot.n_clamp_T += d.n_clamp_T;
        tot.n_clamp_g += d.n_clamp_g;
        tot.n_x_outside += d.n_x_outside;
        tot.n_multi_image += d.n_multi_image;
        tot.n_negative += d.n_negative;
    }
    if (!neg) tot.n_negative = -1;
    if (total) *total = tot;
    return PPM_OK;
}

int ppm_get_tiles(const ppm_plan *pl, ppm_tiles *out)
{
    if (!pl || !out) return fail(PPM_ERR_ARG, "ppm_get_tiles: null argument");
    out->phase_tile = pl->S.pt_fwd;
    out->phase_tile_grad = pl->S.pt_adj;
    out->ring_group = pl->S.ring_group;
    return PPM_OK;
}

int ppm_set_tiles(ppm_plan *pl, const ppm_tiles *t)
{
    if (!pl || !t) return fail(PPM_ERR_ARG, "ppm_set_tiles: null argument");
    if (t->phase_tile < 1 || t->phase_tile > kMaxTile)
        return fail(PPM_ERR_ARG, "phase_tile must lie in [1, 256]");
    if (t->phase_tile_grad < kMinTileGrad || t->phase_tile_grad > kMaxTile)
        return fail(PPM_ERR_ARG, "phase_tile_grad must lie in [8, 256]");
    if (t->ring_group < 1 || t->ring_group > kMaxRingGroup)
        return fail(PPM_ERR_ARG, "ring_group must lie in [1, 64]");
    pl->S.pt_fwd = t->phase_tile;
    pl->S.pt_adj = t->phase_tile_grad;
    pl->S.ring_group = t->ring_group;
    return PPM_OK;
}

}  // extern "C"

namespace {

struct EventSet {
    std::vector<hipEvent_t> ev;
    ~EventSet()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

// Per-candidate medians of `reps` timed calls of run() (set(c) selects
// candidate c).  The device is first kept busy for about 100 ms with the
// first candidate (its clock ramps up under load, and drops again when idle),
// and the candidates are then timed in turn, repetition by repetition, so that
// any remaining drift reaches every candidate alike.
template <typename Set, typename Run>
int time_candidates(const std::vector<int> &cands, Set &&set, Run &&run, int reps, hipStream_t st,
                    std::vector<double> &med)
{
    const int nc = (int)cands.size();
    EventSet es;
    es.ev.assign(2 * (size_t)nc * reps + 2, nullptr);
    for (auto &e : es.ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return hip_fail(r, "autotune event");
    }
    const char *what = "autotune";
    set(cands[0]);
    hipError_t e = hipEventRecord(es.ev[0], st);
    if (e == hipSuccess) e = run(&what);
    if (e == hipSuccess) e = hipEventRecord(es.ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(es.ev[1]);
    if (e != hipSuccess) return hip_fail(e, what);
    float t0 = 0.0f;
    e = hipEventElapsedTime(&t0, es.ev[0], es.ev[1]);
    if (e != hipSuccess) return hip_fail(e, "autotune elapsed");
    int warm = t0 > 0.0f ? (int)std::ceil(100.0 / t0) : 1;
    warm = warm < 1 ? 1 : (warm > 500 ? 500 : warm);
    for (int i = 0; i < warm; ++i) {
        e = run(&what);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    for (int r = 0; r < reps; ++r)
        for (int c = 0; c < nc; ++c) {
            set(cands[c]);
            hipEvent_t *ev = &es.ev[2 + 2 * ((size_t)r * nc + c)];
            e = hipEventRecord(ev[0], st);
            if (e == hipSuccess) e = run(&what);
            if (e == hipSuccess) e = hipEventRecord(ev[1], st);
            if (e != hipSuccess) return hip_fail(e, what);
        }
    e = hipEventSynchronize(es.ev.back());
    if (e != hipSuccess) return hip_fail(e, "autotune sync");
    med.assign(nc, 0.0);
    std::vector<float> t(reps);
    for (int c = 0; c < nc; ++c) {
        for (int r = 0; r < reps; ++r) {
            hipEvent_t *ev = &es.ev[2 + 2 * ((size_t)r * nc + c)];
            e = hipEventElapsedTime(&t[r], ev[0], ev[1]);
            if (e != hipSuccess) return hip_fail(e, "autotune elapsed");
        }
        std::sort(t.begin(), t.end());
        med[c] = reps % 2 ? t[reps / 2] : 0.5 * (t[reps / 2 - 1] + t[reps / 2]);
    }
    return PPM_OK;
}

// Candidates in increasing order, dropping those that tile n_phase into as
// many tiles as a smaller candidate already does.
std::vector<int> tile_candidates(std::initializer_list<int> all, int P)
{
    std::vector<int> out;
    int last_tiles = -1;
    for (int t : all) {
        int n = (P + t - 1) / t;
        if (n == last_tiles) continue;
        out.push_back(t);
        last_tiles = n;
    }
    return out;
}

}  // namespace

extern "C" {

int ppm_autotune(ppm_plan *pl, const double *params_dev, int B, const int32_t *n_cells_host, int reps,
                 void *stream, ppm_tune_report *report)
{
    if (reps < 1 || reps > 1000) return fail(PPM_ERR_ARG, "ppm_autotune: reps must lie in [1, 1000]");
    if (!pl || !params_dev) return fail(PPM_ERR_ARG, "ppm_autotune: null plan or params");
    hipStream_t st = (hipStream_t)stream;
    if (stream_capturing(st)) return fail(PPM_ERR_ARG, "ppm_autotune: the stream is being captured");
    DevSpec &S = pl->S;
    const int pt0 = S.pt_fwd, pa0 = S.pt_adj, rg0 = S.ring_group;
    ppm_tune_report rep;
    std::memset(&rep, 0, sizeof(rep));
    auto restore = [&](int code) {
        S.pt_fwd = pt0;
        S.pt_adj = pa0;
        S.ring_group = rg0;
        return code;
    };
    // every candidate runs the batch as a caller's call would: the layout
    // (work lists of the candidate's ring group) is made resident first
    auto fwd = [&](const char **what) {
        int r = prepare(pl, params_dev, B, n_cells_host, st);
        if (r) {
            *what = ppm_last_error();
            return hipErrorInvalidValue;
        }
        *what = "ppm_autotune forward";
        return run_forward(pl, params_dev, st, nullptr, pl->W.counts);
    };
    int rc = prepare(pl, params_dev, B, n_cells_host, st);
    if (rc) return rc;
    // forward tile at the plan's ring group
    const std::vector<int> fc = tile_candidates({4, 8, 12, 16, 20, 24, 28, 32, 48, 64, 96, 128}, S.P);
    std::vector<double> fms;
    rc = time_candidates(fc, [&](int t) { S.pt_fwd = t; }, fwd, reps, st, fms);
    if (rc) return restore(rc);
    double best = 0.0;
    int best_t = pt0;
    for (size_t c = 0; c < fc.size(); ++c) {
        rep.fwd_tile[rep.n_fwd] = fc[c];
        rep.fwd_ms[rep.n_fwd++] = fms[c];
        if (c == 0 || fms[c] < best) {
            best = fms[c];
            best_t = fc[c];
        }
    }
    S.pt_fwd = best_t;
    // rings per block of the windowed kernel at that tile: 1, 2, 4, 8, 16,
    // 32 (candidates beyond the rings of one instance are skipped)
    if (S.intensity == PPM_I_TABLE && S.fast && S.n_side == 0) {
        std::vector<int> gc;
        for (int g : {1, 2, 4, 8, 16, 32})
            if (g == 1 || g <= S.n_rings_spec[0] + S.n_rings_spec[1]) gc.push_back(g);
        std::vector<double> gms;
        rc = time_candidates(gc, [&](int g) { S.ring_group = g; }, fwd, reps, st, gms);
        if (rc) return restore(rc);
        double bg = 0.0;
        int best_g = rg0;
        for (size_t c = 0; c < gc.size(); ++c) {
            rep.group[rep.n_group] = gc[c];
            rep.group_ms[rep.n_group++] = gms[c];
            if (c == 0 || gms[c] < bg) {
                bg = gms[c];
                best_g = gc[c];
            }
        }
        S.ring_group = best_g;
        rc = prepare(pl, params_dev, B, n_cells_host, st);
        if (rc) return restore(rc);
    }
    // adjoint tile (gradient plans)
    if (pl->grad) {
        DevBuf data, grad, logl;
        hipError_t e = hipMalloc(&data.p, sizeof(int32_t) * (size_t)S.P * S.C);
        if (e == hipSuccess) e = hipMalloc(&grad.p, sizeof(double) * (size_t)B * PPM_NGRAD);
        if (e == hipSuccess) e = hipMalloc(&logl.p, sizeof(double) * (size_t)B);
        if (e == hipSuccess) e = hipMemsetAsync(data.p, 0, sizeof(int32_t) * (size_t)S.P * S.C, st);
        if (e != hipSuccess) return restore(hip_fail(e, "ppm_autotune temporary buffers"));
        int best_a = pa0;
        const std::vector<int> gc = tile_candidates({8, 16, 24, 32}, S.P);
        std::vector<double> gms;
        rc = time_candidates(gc, [&](int t) { S.pt_adj = t; }, [&](const char **what) {
            return run_grad(pl, params_dev, (const int32_t *)data.p, (double *)logl.p, (double *)grad.p, st, what);
        }, reps, st, gms);
        if (rc) return restore(rc);
        for (size_t c = 0; c < gc.size(); ++c) {
            rep.grad_tile[rep.n_grad] = gc[c];
            rep.grad_ms[rep.n_grad++] = gms[c];
            if (c == 0 || gms[c] < best) {
                best = gms[c];
                best_a = gc[c];
            }
        }
        S.pt_adj = best_a;
        // the temporaries are freed on return: finish the work that uses them
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return restore(hip_fail(e, "ppm_autotune sync"));
    }
    rep.chosen.phase_tile = S.pt_fwd;
    rep.chosen.phase_tile_grad = S.pt_adj;
    rep.chosen.ring_group = S.ring_group;
    if (report) *report = rep;
    return PPM_OK;
}

int ppm_autotune_map(ppm_plan *pl, const double *params_dev, int B, const double *map_dev, int reps, void *stream,
                     ppm_tune_report *report)
{
    if (reps < 1 || reps > 1000) return fail(PPM_ERR_ARG, "ppm_autotune_map: reps must lie in [1, 1000]");
    if (!pl || !params_dev) return fail(PPM_ERR_ARG, "ppm_autotune_map: null plan or params");
    hipStream_t st = (hipStream_t)stream;
    if (stream_capturing(st)) return fail(PPM_ERR_ARG, "ppm_autotune_map: the stream is being captured");
    int rc = prepare(pl, params_dev, B, nullptr, st, true);
    if (rc) return rc;
    if (!map_dev) return fail(PPM_ERR_ARG, "null map");
    DevSpec &S = pl->S;
    const int pt0 = S.pt_fwd;
    ppm_tune_report rep;
    std::memset(&rep, 0, sizeof(rep));
    const std::vector<int> mc = tile_candidates({8, 16, 32}, S.P);
    std::vector<double> mms;
    rc = time_candidates(mc, [&](int t) { S.pt_fwd = t; }, [&](const char **what) {
        *what = "ppm_autotune_map forward";
        return run_forward_map(pl, params_dev, map_dev, st, nullptr, pl->W.counts);
    }, reps, st, mms);
    if (rc) {
        S.pt_fwd = pt0;
        return rc;
    }
    double best = 0.0;
    int best_t = pt0;
    for (size_t c = 0; c < mc.size(); ++c) {
        rep.fwd_tile[rep.n_fwd] = mc[c];
        rep.fwd_ms[rep.n_fwd++] = mms[c];
        if (c == 0 || mms[c] < best) {
            best = mms[c];
            best_t = mc[c];
        }
    }
    S.pt_fwd = best_t;
    rep.chosen.phase_tile = S.pt_fwd;
    rep.chosen.phase_tile_grad = S.pt_adj;
    rep.chosen.ring_group = S.ring_group;
    if (report) *report = rep;
    return PPM_OK;
}

int ppm_instance_status(ppm_plan *pl, int B, int32_t *status_dev, void *stream)
{
    if (!pl || !status_dev) return fail(PPM_ERR_ARG, "null argument");
    if (B < 1 || B > pl->max_batch) return fail(PPM_ERR_BATCH, "batch outside [1, max_batch]");
    hipError_t e = launch_status(pl->W, B, status_dev, (hipStream_t)stream);
    return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_instance_status");
}

int ppm_debug_ring(ppm_plan *pl, int b, int r, double *table_out, double *info_out, double *trace_out,
                   int32_t *trace_info, void *stream)
{
    if (!pl) return fail(PPM_ERR_ARG, "null plan");
    if (!pl->cur || pl->cur->pass.empty()) return fail(PPM_ERR_ARG, "ppm_debug_ring: no evaluation yet");
    const ListPass &lp = pl->cur->pass.back();   // the ring scratch holds the last pass
    if (b < lp.inst0 || b >= lp.inst0 + lp.nb || r < 0 || r >= pl->S.R_tot)
        return fail(PPM_ERR_ARG, "ring out of range (instances of the last evaluation's last workspace pass only)");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "ppm_debug_ring sync");
    const size_t ring = (size_t)(b - lp.inst0) * pl->S.R_tot + r;
    RingRec g;
    e = hipMemcpy(&g, pl->W.rings + ring, sizeof(g), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "ppm_debug_ring copy");
    if (table_out) {
        e = hipMemcpy(table_out, pl->W.table + ring * pl->S.n_alpha, sizeof(double4) * pl->S.n_alpha,
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "ppm_debug_ring table copy");
    }
    if (info_out) {
        double4 last;
        e = hipMemcpy(&last, pl->W.table + ring * pl->S.n_alpha + pl->S.n_alpha - 1, sizeof(last),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "ppm_debug_ring info copy");
        info_out[0] = g.alpha_max;
        info_out[1] = last.x;
        info_out[2] = g.u;
        info_out[3] = g.R;
    }
    if (trace_out) {
        e = hipMemcpy(trace_out, pl->W.trace + ring * (pl->S.n_fp + 1), sizeof(double4) * (pl->S.n_fp + 1),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "ppm_debug_ring trace copy");
    }
    if (trace_info) {
        trace_info[0] = g.visible;
        trace_info[1] = g.inv_min;
        trace_info[2] = g.inv_max;
    }
    return PPM_OK;
}

int ppm_profile_begin(ppm_plan *pl, int max_calls)
{
    if (!pl || max_calls < 1) return fail(PPM_ERR_ARG, "ppm_profile_begin: bad arguments");
    if ((int)pl->ev.size() < 2 * max_calls) {
        for (hipEvent_t e : pl->ev) (void)hipEventDestroy(e);
        pl->ev.assign(2 * max_calls, nullptr);
        for (auto &e : pl->ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return hip_fail(r, "ppm_profile_begin event");
        }
    }
    pl->prof_cap = max_calls;
    pl->prof_n = 0;
    pl->prof_on = true;
    return PPM_OK;
}

int ppm_profile_end(ppm_plan *pl, double *hot_ms_total, int *n_calls)
{
    if (!pl || !hot_ms_total || !n_calls) return fail(PPM_ERR_ARG, "ppm_profile_end: null argument");
    double tot = 0.0;
    for (int i = 0; i < pl->prof_n; ++i) {
        hipError_t r = hipEventSynchronize(pl->ev[2 * i + 1]);
        if (r != hipSuccess) return hip_fail(r, "ppm_profile_end sync");
        float ms = 0.0f;
        r = hipEventElapsedTime(&ms, pl->ev[2 * i], pl->ev[2 * i + 1]);
        if (r != hipSuccess) return hip_fail(r, "ppm_profile_end elapsed");
        tot += ms;
    }
    *hot_ms_total = tot;
    *n_calls = pl->prof_n;
    pl->prof_on = false;
    pl->prof_n = 0;
    return PPM_OK;
}

int ppm_get_passes(const ppm_plan *pl, int *n_passes)
{
    if (!pl || !n_passes) return fail(PPM_ERR_ARG, "ppm_get_passes: null argument");
    *n_passes = pl->cur ? (int)pl->cur->pass.size() : 0;
    return PPM_OK;
}

int ppm_visible_pairs(ppm_plan *pl, int B, long long *out, void *stream)
{
    if (!pl || !out) return fail(PPM_ERR_ARG, "null argument");
    if (B < 1 || B > pl->max_batch) return fail(PPM_ERR_BATCH, "batch outside [1, max_batch]");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ppm_visible_pairs sync");
    std::vector<int32_t> v((size_t)B * pl->S.R_tot);
    e = hipMemcpy(v.data(), pl->W.vis_pairs, sizeof(int32_t) * v.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "ppm_visible_pairs copy");
    long long s = 0;
    for (int32_t x : v) s += x;
    *out = s;
    return PPM_OK;
}

}  // extern "C"
