// Device workspace of a plan and the host-side launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppm_internal.h"
#include "ppm_status.h"
#include "../../include/ppm.h"

namespace ppm {

struct Workspace {
    StarRec *stars;        // [B]
    RingRec *rings;        // [B][R_tot]
    double4 *table;        // [B][R_tot][n_alpha]
    double4 *trace;        // [B][R_tot][n_fp + 1]
    float *sub;            // [B][R_tot][nmu][nx]      (table intensity)
    float *partial32;      // [n_groups][P][E] ring-group partial sums (FP32 path), by group-list position
    double *partial64;     // [n_groups][P][E]         (FP64 path)
    float *fold_in32;      // [B][P][E]
    double *fold_in64;     // [B][P][E]
    double *counts;        // [B][P][C]
    int32_t *vis_pairs;    // [B][R_tot]
    int32_t *diag;         // [B][R_tot][5] per ring: clamp flags (bit 0 logT, bit 1 log g), multiple-image
                           // samples, intensity evaluations with x outside the table, negative intensities,
                           // visible pairs of map patches whose logT was clamped
    const int32_t *glist;  // [n_groups][2] ring groups of the pass: first work-list position, ring count
    const int32_t *grange; // [B][2] per instance of the pass: its groups [first, end) in glist
    double *ll_part;       // [B][loglike_parts] first-stage likelihood sums
    int32_t *ll_bad;       // [B][loglike_parts] bins with m <= 0 and d > 0
    double *lfact;         // [kLogFact] log d! for the first kLogFact counts
    unsigned *ll_done;     // [B] blocks of the likelihood kernel done per instance (zero between calls)
    // gradient plans only
    double4 *table_u;      // [B][R_tot][n_alpha] d/du (psi, psi', T, T') at fixed alpha
    double4 *tangent;      // [B][R_tot][n_fp + 1][5] tangents of (F, z, phi_o, mu)
    RingTan *ringtan;      // [B][R_tot]
    float2 *subtg;         // [B][R_tot][sub_stride] d sub / d logT, d sub / d log g
    double *flux;          // [B][P][E] flux before absorption
    float *gtil;           // [B][P][E] adjoint of the flux divided by E
    double *nh_part;       // [B][P][E/16] N_H gradient per phase and 16-energy tile
    double *gpart;         // [B][R_tot][n_tile][kGradAcc] per-block adjoint sums
    // temperature-map plans only
    MapCell *mcell;        // [B][n_pix] active patches, per ring sorted by temperature bucket
    int32_t *mgrp;         // [B][R_tot][map_nb + 1] bucket offsets within the ring's patches
};

constexpr int kPhaseTile = 8;    // default phases per block of the accumulation kernels
constexpr int kMinTileGrad = 8;  // smallest adjoint phase tile (sizes the per-block adjoint sums)
constexpr int kMaxTile = 256;    // largest phase tile either kernel accepts
constexpr int kGradAcc = 9;      // per-ring adjoint sums of the accumulation kernel
constexpr int kLogFact = 1024;   // counts whose log d! comes from a table
#ifndef PPM_FWD_WAVES
#define PPM_FWD_WAVES 12
#endif
constexpr int kFwdWaves = PPM_FWD_WAVES;  // waves per block of the forward accumulation kernel

constexpr int kDiagFields = 5;   // per-ring diagnostic counters (Workspace::diag)
constexpr int kMaxRingGroup = 64; // largest number of rings one accumulation block sums

__host__ __device__ int validate_params(const double *p, int n_spots);

// One workspace pass: B instances, their live rings (list, n_list entries,
// chunk-local instance index * R_tot + ring slot) and the ring groups of the
// accumulation (W.glist, n_groups entries; W.grange per instance).
// counts_out may be NULL when data is given (then only logL is kept); with
// data (int32 [P][C]) the pass's logL goes to logl[B] (Workspace::stars,
// ll_part, ll_bad, ll_done of the pass).
hipError_t launch_forward(const DevSpec &S, const Workspace &W, const double *params,
                          const int32_t *ncells_dev, int B, const int32_t *list, int n_list, int n_groups,
                          hipStream_t st, double *flux_out, double *counts_out, const int32_t *data = nullptr,
                          double *logl = nullptr, hipEvent_t ev_hot0 = nullptr, hipEvent_t ev_hot1 = nullptr);
void launch_setup(const DevSpec &S, const Workspace &W, const double *params, const int32_t *ncells_dev, int B,
                  hipStream_t st);
void launch_table_trace(const DevSpec &S, const Workspace &W, const int32_t *list, int n_list, hipStream_t st);
void launch_reduce_fold32(const DevSpec &S, const Workspace &W, const int32_t *list, int B, hipStream_t st,
                          double *flux_out, double *counts_out, const int32_t *data = nullptr,
                          double *logl = nullptr);
void launch_fold32(const DevSpec &S, const Workspace &W, int B, hipStream_t st, double *counts_out,
                   const int32_t *data, double *logl);
hipError_t launch_forward_map(const DevSpec &S, const Workspace &W, const double *params, const double *map, int B,
                              const int32_t *list, int n_list, int n_groups, hipStream_t st, double *flux_out,
                              double *counts_out, const int32_t *data = nullptr, double *logl = nullptr,
                              hipEvent_t ev_hot0 = nullptr, hipEvent_t ev_hot1 = nullptr);
size_t accum_map_lds(const DevSpec &S);
constexpr int kMapWaves = 8;     // waves per block of the map accumulation kernel, one phase each
hipError_t launch_status(const Workspace &W, int B, int32_t *out, hipStream_t st);
hipError_t launch_grad(const DevSpec &S, const Workspace &W, const double *params, const int32_t *ncells_dev,
                       int B, const int32_t *list, int n_list, const double *counts, const int32_t *data,
                       double *grad, hipStream_t st);
size_t accum_table_lds(const DevSpec &S);
size_t accum_adj_lds(const DevSpec &S);
int loglike_blocks(int PC);
int loglike_parts(int P, int C);   // per-instance likelihood partials (fused fold or block sums)
// read access to a plan's model, workspace, batch limit and device (host)
bool plan_view(const ppm_plan *pl, const DevSpec **S, const Workspace **W, int *max_batch, int *device);
int api_hip_fail(hipError_t e, const char *where);  // sets ppm_last_error, returns PPM_ERR_HIP

}  // namespace ppm
