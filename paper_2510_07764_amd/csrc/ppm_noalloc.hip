// Allocation-free likelihood entry point (ppm_loglike_noalloc): the same
// kernels and launch sequence as ppm_loglike, with every per-call buffer
// (ring records, deflection tables, traces, sub-tables, ring-group partial
// spectra, fold input, model counts, likelihood partial sums, work lists)
// carved from one file-scope device array instead of the plan's workspace,
// and the work lists built on the device, so that a call makes no
// allocation and no host-to-device copy.  The plan still supplies its
// constant tables (atmosphere, response, energies, quadrature nodes, log d!
// table), set up once at plan creation.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "ppm_internal.h"
#include "ppm_launch.h"
#include "../../include/ppm.h"

namespace ppm {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// Per-call scratch of ppm_loglike_noalloc.  In host code this name is a
// host-side stand-in, not a device address: host code uses only the
// address registered per device below.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_mu;
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];
bool g_done[kMaxDevices];

// Device address of `scratch` on the current device dev: looked up with
// hipGetSymbolAddress on the entry point's first call on that device and
// kept (each device holds its own copy of the array at its own address).
hipError_t scratch_ptr(int dev, void **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[dev]) {
        void *p = nullptr;
        g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
        g_done[dev] = true;
    }
    *out = g_ptr[dev];
    return g_err[dev];
}
}  // namespace

// Work lists of B instances at the spec's own grids, built on the device:
// instance b's live rings (spot 0 rings, then spot 1 rings) at list
// positions b * n_live + i, its ring groups at b * n_grp + j, group j
// covering positions j G .. min(j G + G, n_live) - 1.  Also clears the
// likelihood's per-instance block counters, which must start at zero.
__global__ void k_default_lists(DevSpec S, int B, int G, int n_live, int n_grp, int32_t *list, int32_t *glist,
                                int32_t *grange, unsigned *ll_done)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nr0 = S.n_rings_spec[0];
    if (tid < B * n_live) {
        const int b = tid / n_live, i = tid - b * n_live;
        const int r = i < nr0 ? i : S.rings_max[0] + (i - nr0);
        list[tid] = b * S.R_tot + r;
    }
    if (tid < B * n_grp) {
        const int b = tid / n_grp, j = tid - b * n_grp;
        const int f = j * G;
        glist[2 * tid] = b * n_live + f;
        glist[2 * tid + 1] = n_live - f < G ? n_live - f : G;
    }
    if (tid < B) {
        grange[2 * tid] = tid * n_grp;
        grange[2 * tid + 1] = (tid + 1) * n_grp;
        ll_done[tid] = 0u;
    }
}

namespace {

// Carves the per-call buffers of B instances out of the scratch array;
// returns the bytes needed (a layout larger than the array is refused).
struct Carver {
    unsigned char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

size_t carve(const DevSpec &S, int B, int n_live, int n_grp, bool want_counts, unsigned char *base, Workspace &W,
             int32_t *&list)
{
    Carver c{base};
    const size_t R = S.R_tot, Bz = B;
    const bool table = S.intensity == PPM_I_TABLE;
    W.stars = c.take<StarRec>(Bz);
    W.rings = c.take<RingRec>(Bz * R);
    W.table = c.take<double4>(Bz * R * S.n_alpha);
    W.trace = c.take<double4>(Bz * R * (S.n_fp + 1));
    W.sub = table ? c.take<float>(Bz * R * (size_t)S.sub_stride) : nullptr;
    W.vis_pairs = c.take<int32_t>(Bz * R);
    W.diag = c.take<int32_t>(Bz * R * kDiagFields);
    W.counts = want_counts ? c.take<double>(Bz * S.P * S.C) : nullptr;
    const int nblk = loglike_parts(S.P, S.C);
    W.ll_part = c.take<double>(Bz * nblk);
    W.ll_bad = c.take<int32_t>(Bz * nblk);
    W.ll_done = c.take<unsigned>(Bz);
    const size_t pe = (size_t)n_grp * B * S.P * S.E;
    if (table) {
        W.partial32 = c.take<float>(pe);
        W.fold_in32 = c.take<float>(Bz * S.P * S.E);
    } else {
        W.partial64 = c.take<double>(pe);
        if (S.rsp64)
            W.fold_in64 = c.take<double>(Bz * S.P * S.E);
        else
            W.fold_in32 = c.take<float>(Bz * S.P * S.E);
    }
    list = c.take<int32_t>(Bz * n_live);
    W.glist = c.take<int32_t>(2 * Bz * n_grp);
    W.grange = c.take<int32_t>(2 * Bz);
    return c.off;
}

}  // namespace

}  // namespace ppm

using namespace ppm;

extern "C" int ppm_loglike_noalloc(ppm_plan *plan, const double *params_dev, int B, const int32_t *data_dev,
                                   double *logl_dev, double *counts_dev, void *stream)
{
    const DevSpec *Sp = nullptr;
    const Workspace *Wp = nullptr;
    int max_batch = 0, plan_dev = -1;
    if (!plan_view(plan, &Sp, &Wp, &max_batch, &plan_dev))
        return api_fail(PPM_ERR_ARG, "ppm_loglike_noalloc: null plan");
    const DevSpec &S = *Sp;
    if (S.n_side > 0)
        return api_fail(PPM_ERR_UNSUPPORTED, "ppm_loglike_noalloc: temperature-map plans are not supported");
    if (!params_dev || !data_dev || !logl_dev)
        return api_fail(PPM_ERR_ARG, "ppm_loglike_noalloc: null params, data or logl");
    if (B < 1 || B > max_batch) return api_fail(PPM_ERR_BATCH, "batch outside [1, max_batch]");
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return api_hip_fail(e, "ppm_loglike_noalloc device");
    if (dev != plan_dev) return api_fail(PPM_ERR_ARG, "ppm_loglike_noalloc: the current device is not the plan's");
    void *vbase = nullptr;
    e = scratch_ptr(dev, &vbase);
    if (e != hipSuccess) return api_hip_fail(e, "ppm_loglike_noalloc: address of the static scratch");
    unsigned char *base = static_cast<unsigned char *>(vbase);
    const int G = (S.intensity == PPM_I_TABLE && S.fast) ? S.ring_group : 1;
    const int n_live = S.n_rings_spec[0] + (S.n_spots > 1 ? S.n_rings_spec[1] : 0);
    const int n_grp = (n_live + G - 1) / G;
    Workspace W = *Wp;   // the plan's constant tables (log d!) are kept
    int32_t *list = nullptr;
    const size_t need = carve(S, B, n_live, n_grp, counts_dev == nullptr, nullptr, W, list);
    if (need > kNoAllocBytes)
        return api_fail(PPM_ERR_BATCH, "ppm_loglike_noalloc: the batch needs more than the 64 MiB static scratch");
    W = *Wp;
    carve(S, B, n_live, n_grp, counts_dev == nullptr, base, W, list);
    double *cnt = counts_dev ? counts_dev : W.counts;
    const int nt = B * (n_live > n_grp ? n_live : n_grp);
    hipLaunchKernelGGL(k_default_lists, dim3((nt + 255) / 256), dim3(256), 0, st, S, B, G, n_live, n_grp, list,
                       const_cast<int32_t *>(W.glist), const_cast<int32_t *>(W.grange), W.ll_done);
    e = launch_forward(S, W, params_dev, nullptr, B, list, B * n_live, B * n_grp, st, nullptr, cnt, data_dev,
                       logl_dev);
    return e == hipSuccess ? PPM_OK : api_hip_fail(e, "ppm_loglike_noalloc launch");
}
