// GPU-resident parallel-tempered Metropolis sampler over the batched
// likelihood (the inference layer of Sect. 6 of arXiv:2510.07764).  Every
// step: one proposal kernel (thread per chain and temperature), one batched
// likelihood evaluation of all proposals, one acceptance kernel (thread per
// chain: its T Metropolis decisions, then the swap round).  Random numbers
// come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC11), a
// counter-based generator, so no generator state is stored or carried.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>
#include <new>

#include "ppm_internal.h"
#include "ppm_launch.h"
#include "../../include/ppm.h"

namespace ppm {

namespace {

// the configuration as a kernel argument
struct PTDev {
    int C, T, n_free, swap_every;
    int free_slot[16];
    double lo[16], hi[16], step[16];
    double beta[PPM_PT_MAX_TEMPS];
    uint32_t key0, key1;
};

// Philox4x32 with ten rounds: words 0 and 2 multiplied by the two round
// multipliers; new words (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)); the key bumped by the two Weyl constants between rounds.
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// uniform on [0, 1) from the top 53 bits of the 64-bit word hi:lo
__device__ inline double uniform53(uint32_t hi, uint32_t lo)
{
    const uint64_t w = ((uint64_t)hi << 21) | (lo >> 11);
    return (double)w * 0x1.0p-53;
}

__device__ inline uint4 pt_counter(int64_t step, int slot, int purpose, int k)
{
    return make_uint4((uint32_t)step, (uint32_t)((uint64_t)step >> 32), (uint32_t)slot,
                      ((uint32_t)purpose << 16) | (uint32_t)k);
}

__global__ __launch_bounds__(64) void k_pt_propose(PTDev cfg, const double *state, double *prop, int64_t step)
{
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;   // t * C + c
    if (slot >= cfg.T * cfg.C) return;
    const int t = slot / cfg.C;
    const double *src = state + (size_t)slot * PPM_NPARAM;
    double *dst = prop + (size_t)slot * PPM_NPARAM;
    double v[PPM_NPARAM];
    for (int j = 0; j < PPM_NPARAM; ++j) v[j] = src[j];
    const double isb = 1.0 / sqrt(cfg.beta[t]);
    for (int pr = 0; 2 * pr < cfg.n_free; ++pr) {
        const uint4 w = philox4x32_10(pt_counter(step, slot, 0, pr), cfg.key0, cfg.key1);
        const double ua = uniform53(w.x, w.y), ub = uniform53(w.z, w.w);
        const double r = sqrt(-2.0 * log(1.0 - ua));
        double sb, cb;
        sincos(2.0 * kPi * ub, &sb, &cb);
        const double z[2] = {r * cb, r * sb};
        for (int q = 0; q < 2; ++q) {
            const int j = 2 * pr + q;
            if (j >= cfg.n_free) break;
            const int s = cfg.free_slot[j];
            v[s] = v[s] + (cfg.step[j] * isb) * z[q];
        }
    }
    for (int j = 0; j < PPM_NPARAM; ++j) dst[j] = v[j];
}

// thread per chain c: the T Metropolis decisions, the swap round when due,
// then the cold state into the chain record
__global__ __launch_bounds__(64) void k_pt_accept(PTDev cfg, double *state, double *logl, const double *prop,
                                                  const double *prop_logl, int32_t *n_acc, int32_t *n_swap,
                                                  int64_t step, double *chain_row, double *chain_logl_row)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cfg.C) return;
    const int C = cfg.C, T = cfg.T;
    for (int t = 0; t < T; ++t) {
        const int slot = t * C + c;
        const double *pp = prop + (size_t)slot * PPM_NPARAM;
        bool in_box = true;
        for (int j = 0; j < cfg.n_free; ++j) {
            const double x = pp[cfg.free_slot[j]];
            in_box = in_box && x >= cfg.lo[j] && x <= cfg.hi[j];
        }
        const double Lp = prop_logl[slot], L = logl[slot];
        const uint4 w = philox4x32_10(pt_counter(step, slot, 1, 0), cfg.key0, cfg.key1);
        const double u = uniform53(w.x, w.y);
        const double log_alpha = cfg.beta[t] * (Lp - L);
        if (in_box && isfinite(Lp) && log(u) < log_alpha) {
            double *dst = state + (size_t)slot * PPM_NPARAM;
            for (int j = 0; j < PPM_NPARAM; ++j) dst[j] = pp[j];
            logl[slot] = Lp;
            n_acc[slot] += 1;
        }
    }
    if (cfg.swap_every > 0 && T > 1 && (step + 1) % cfg.swap_every == 0) {
        const int parity = (int)((step / cfg.swap_every) % 2);
        for (int t = parity; t + 1 < T; t += 2) {
            const int sa = t * C + c, sb = (t + 1) * C + c;
            const uint4 w = philox4x32_10(pt_counter(step, sa, 2, 0), cfg.key0, cfg.key1);
            const double u = uniform53(w.x, w.y);
            const double log_r = (cfg.beta[t] - cfg.beta[t + 1]) * (logl[sb] - logl[sa]);
            if (log(u) < log_r) {
                double *a = state + (size_t)sa * PPM_NPARAM, *b = state + (size_t)sb * PPM_NPARAM;
                for (int j = 0; j < PPM_NPARAM; ++j) {
                    const double tmp = a[j];
                    a[j] = b[j];
                    b[j] = tmp;
                }
                const double tl = logl[sa];
                logl[sa] = logl[sb];
                logl[sb] = tl;
                n_swap[sa] += 1;   // pair t of chain c
            }
        }
    }
    if (chain_row)
        for (int j = 0; j < PPM_NPARAM; ++j) chain_row[(size_t)c * PPM_NPARAM + j] = state[(size_t)c * PPM_NPARAM + j];
    if (chain_logl_row) chain_logl_row[c] = logl[c];
}

__global__ void k_pt_set(int n, const double *params_in, const double *logl_in, double *state, double *logl,
                         int32_t *n_acc, int32_t *n_swap)
{
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n) return;
    for (int j = 0; j < PPM_NPARAM; ++j) state[(size_t)slot * PPM_NPARAM + j] = params_in[(size_t)slot * PPM_NPARAM + j];
    logl[slot] = logl_in ? logl_in[slot] : -INFINITY;
    n_acc[slot] = 0;
    n_swap[slot] = 0;
}

}  // namespace

}  // namespace ppm

using namespace ppm;

struct ppm_pt {
    PTDev cfg;
    int64_t step = 0;
    double *state = nullptr, *logl = nullptr, *prop = nullptr, *prop_logl = nullptr;
    int32_t *n_acc = nullptr, *n_swap = nullptr;
    ~ppm_pt()
    {
        for (void *p : {(void *)state, (void *)logl, (void *)prop, (void *)prop_logl, (void *)n_acc, (void *)n_swap})
            if (p) (void)hipFree(p);
    }
};

extern "C" {

int ppm_pt_create(const ppm_pt_config *c, ppm_pt **out)
{
    if (!c || !out) return api_fail(PPM_ERR_ARG, "ppm_pt_create: null argument");
    *out = nullptr;
    if (c->n_chains < 1) return api_fail(PPM_ERR_ARG, "n_chains must be >= 1");
    if (c->n_temps < 1 || c->n_temps > PPM_PT_MAX_TEMPS) return api_fail(PPM_ERR_ARG, "n_temps must lie in [1, 64]");
    if (c->n_free < 1 || c->n_free > 16) return api_fail(PPM_ERR_ARG, "n_free must lie in [1, 16]");
    if (c->swap_every < 0) return api_fail(PPM_ERR_ARG, "swap_every must be >= 0");
    if ((int64_t)c->n_chains * c->n_temps > (1 << 24)) return api_fail(PPM_ERR_ARG, "too many chains");
    unsigned seen = 0;
    for (int j = 0; j < c->n_free; ++j) {
        const int s = c->free_slot[j];
        if (s < 0 || s >= PPM_NPARAM || (seen >> s & 1u)) return api_fail(PPM_ERR_ARG, "free slots must be distinct, 0..15");
        seen |= 1u << s;
        if (!(c->lo[j] < c->hi[j])) return api_fail(PPM_ERR_ARG, "prior box needs lo < hi");
        if (!(c->step[j] > 0.0) || !std::isfinite(c->step[j])) return api_fail(PPM_ERR_ARG, "proposal steps must be > 0");
    }
    for (int t = 0; t < c->n_temps; ++t) {
        if (!(c->beta[t] > 0.0 && c->beta[t] <= 1.0)) return api_fail(PPM_ERR_ARG, "beta must lie in (0, 1]");
        if (t && !(c->beta[t] < c->beta[t - 1])) return api_fail(PPM_ERR_ARG, "beta must decrease strictly");
    }
    ppm_pt *pt = new (std::nothrow) ppm_pt();
    if (!pt) return api_fail(PPM_ERR_ALLOC, "host allocation failed");
    PTDev &d = pt->cfg;
    d.C = c->n_chains;
    d.T = c->n_temps;
    d.n_free = c->n_free;
    d.swap_every = c->swap_every;
    for (int j = 0; j < 16; ++j) {
        const bool on = j < c->n_free;
        d.free_slot[j] = on ? c->free_slot[j] : 0;
        d.lo[j] = on ? c->lo[j] : 0.0;
        d.hi[j] = on ? c->hi[j] : 0.0;
        d.step[j] = on ? c->step[j] : 0.0;
    }
    for (int t = 0; t < PPM_PT_MAX_TEMPS; ++t) d.beta[t] = t < c->n_temps ? c->beta[t] : 1.0;
    d.key0 = (uint32_t)c->seed;
    d.key1 = (uint32_t)(c->seed >> 32);
    const size_t n = (size_t)d.T * d.C;
    bool ok = hipMalloc(&pt->state, sizeof(double) * n * PPM_NPARAM) == hipSuccess
           && hipMalloc(&pt->prop, sizeof(double) * n * PPM_NPARAM) == hipSuccess
           && hipMalloc(&pt->logl, sizeof(double) * n) == hipSuccess
           && hipMalloc(&pt->prop_logl, sizeof(double) * n) == hipSuccess
           && hipMalloc(&pt->n_acc, sizeof(int32_t) * n) == hipSuccess
           && hipMalloc(&pt->n_swap, sizeof(int32_t) * n) == hipSuccess;
    if (!ok) {
        delete pt;
        return api_fail(PPM_ERR_ALLOC, "device allocation of the sampler state failed");
    }
    *out = pt;
    return PPM_OK;
}

void ppm_pt_destroy(ppm_pt *pt) { delete pt; }

int ppm_pt_set_state(ppm_pt *pt, const double *params_dev, const double *logl_dev, int64_t step, void *stream)
{
    if (!pt || !params_dev) return api_fail(PPM_ERR_ARG, "ppm_pt_set_state: null argument");
    if (step < 0) return api_fail(PPM_ERR_ARG, "step must be >= 0");
    const int n = pt->cfg.T * pt->cfg.C;
    hipLaunchKernelGGL(k_pt_set, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, params_dev, logl_dev,
                       pt->state, pt->logl, pt->n_acc, pt->n_swap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return api_hip_fail(e, "ppm_pt_set_state");
    pt->step = step;
    return PPM_OK;
}

int ppm_pt_propose(ppm_pt *pt, double *prop_dev, void *stream)
{
    if (!pt || !prop_dev) return api_fail(PPM_ERR_ARG, "ppm_pt_propose: null argument");
    const int n = pt->cfg.T * pt->cfg.C;
    hipLaunchKernelGGL(k_pt_propose, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, pt->cfg, pt->state,
                       prop_dev, pt->step);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PPM_OK : api_hip_fail(e, "ppm_pt_propose");
}

static int pt_accept(ppm_pt *pt, const double *prop, const double *prop_logl, double *chain_row, double *chain_l,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_pt_accept, dim3((pt->cfg.C + 63) / 64), dim3(64), 0, st, pt->cfg, pt->state, pt->logl, prop,
                       prop_logl, pt->n_acc, pt->n_swap, pt->step, chain_row, chain_l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return api_hip_fail(e, "ppm_pt_accept");
    ++pt->step;
    return PPM_OK;
}

int ppm_pt_accept(ppm_pt *pt, const double *prop_dev, const double *prop_logl_dev, void *stream)
{
    if (!pt || !prop_dev || !prop_logl_dev) return api_fail(PPM_ERR_ARG, "ppm_pt_accept: null argument");
    return pt_accept(pt, prop_dev, prop_logl_dev, nullptr, nullptr, (hipStream_t)stream);
}

int ppm_pt_run(ppm_pt *pt, ppm_plan *plan, const int32_t *data_dev, int n_steps, double *chain_dev,
               double *chain_logl_dev, void *stream)
{
    if (!pt || !plan || !data_dev) return api_fail(PPM_ERR_ARG, "ppm_pt_run: null argument");
    if (n_steps < 0) return api_fail(PPM_ERR_ARG, "n_steps must be >= 0");
    const int n = pt->cfg.T * pt->cfg.C;
    for (int s = 0; s < n_steps; ++s) {
        int rc = ppm_pt_propose(pt, pt->prop, stream);
        if (rc) return rc;
        rc = ppm_loglike(plan, pt->prop, n, nullptr, data_dev, pt->prop_logl, nullptr, stream);
        if (rc) return rc;
        rc = pt_accept(pt, pt->prop, pt->prop_logl, chain_dev ? chain_dev + (size_t)s * pt->cfg.C * PPM_NPARAM : nullptr,
                       chain_logl_dev ? chain_logl_dev + (size_t)s * pt->cfg.C : nullptr, (hipStream_t)stream);
        if (rc) return rc;
    }
    return PPM_OK;
}

int ppm_pt_get_state(ppm_pt *pt, double *params_dev, double *logl_dev, int32_t *n_accept_dev, int32_t *n_swap_dev,
                     int64_t *step, void *stream)
{
    if (!pt) return api_fail(PPM_ERR_ARG, "ppm_pt_get_state: null sampler");
    const size_t n = (size_t)pt->cfg.T * pt->cfg.C;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (params_dev && e == hipSuccess)
        e = hipMemcpyAsync(params_dev, pt->state, sizeof(double) * n * PPM_NPARAM, hipMemcpyDeviceToDevice, st);
    if (logl_dev && e == hipSuccess) e = hipMemcpyAsync(logl_dev, pt->logl, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (n_accept_dev && e == hipSuccess)
        e = hipMemcpyAsync(n_accept_dev, pt->n_acc, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
    if (n_swap_dev && e == hipSuccess)
        e = hipMemcpyAsync(n_swap_dev, pt->n_swap, sizeof(int32_t) * (n - pt->cfg.C), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return api_hip_fail(e, "ppm_pt_get_state copy");
    if (step) *step = pt->step;
    return PPM_OK;
}

}  // extern "C"
