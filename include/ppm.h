/*
 * libppm — MI355X (gfx950) implementation of the energy-resolved X-ray
 * pulse-profile forward model and its Poisson log-likelihood
 * (Zhou & Huang, "GPU-accelerated X-ray pulse profile modeling",
 * arXiv:2510.07764).
 *
 * C ABI.  All entry points return an int status (PPM_OK = 0, negative on
 * error) and never throw.  Device buffers are caller-owned and must hold
 * the sizes stated; the plan owns its tables and scratch.  Calls are
 * asynchronous on the given HIP stream (pass the stream handle as void*,
 * NULL = the default stream); no call synchronises the host except where
 * stated.  One plan must not be used from two streams at the same time.
 * Results are bitwise reproducible for fixed inputs.
 *
 * Parameter record: 16 doubles per instance, row-major [B][16]:
 *   0 M [M_sun]     1 R_e [km]     2 inclination [rad]   3 Phi [cycles]
 *   4 N_H [1e20 cm^-2]  5 nu [Hz]  6 D [pc]              7 unused
 *   8 theta_1 [rad] 9 zeta_1 [rad] 10 logT_1             11 unused
 *  12 theta_2 [rad] 13 zeta_2 [rad] 14 logT_2            15 dphi_2 [cycles]
 * The twelve differentiable slots, in gradient order, are
 *   0, 1, 2, 3, 4, 8, 9, 10, 12, 13, 14, 15.
 */
#ifndef PPM_H
#define PPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PPM_NPARAM 16
#define PPM_NGRAD 12

/* return codes */
#define PPM_OK 0
#define PPM_ERR_ARG (-1)        /* null pointer, size or layout the plan does not support */
#define PPM_ERR_BATCH (-2)      /* B larger than the plan's max_batch, or B < 1 */
#define PPM_ERR_HIP (-3)        /* a HIP runtime call failed (see ppm_last_error) */
#define PPM_ERR_UNSUPPORTED (-4)/* spec feature not implemented (e.g. non-uniform x axis) */
#define PPM_ERR_ALLOC (-5)      /* device allocation at plan creation failed */

/* per-instance status codes (written by every evaluation) */
#define PPM_INST_OK 0
#define PPM_INST_NONFINITE 1    /* a parameter is NaN or Inf */
#define PPM_INST_BAD_STAR 2     /* M <= 0, R_e <= 0, D <= 0, nu < 0, or R_e <= 1.5 R_S */
#define PPM_INST_COMPACT 3      /* GM/(R_e c^2) > 0.28: multiple images not modelled (Sect. 6) */
#define PPM_INST_BAD_SPOT 4     /* spot colatitude outside [0, pi] or radius outside (0, pi] */
#define PPM_INST_FAST_SPIN 5    /* surface speed beta >= 0.6 somewhere on the star */
#define PPM_INST_BAD_MAP 6      /* a temperature-map value more than 64 logT table steps
                                   outside the table's logT range */

enum ppm_mode { PPM_MODE_SD = 0, PPM_MODE_OS = 1 };
enum ppm_intensity { PPM_I_BLACKBODY = 0, PPM_I_TABLE = 1 };
enum ppm_shape { PPM_SHAPE_CAP = 0, PPM_SHAPE_ANNULUS = 1, PPM_SHAPE_CRESCENT = 2 };
enum ppm_precision { PPM_F32 = 0, PPM_F64 = 1 };
enum ppm_interp { PPM_INTERP_MIXED = 0, PPM_INTERP_CUBIC = 1, PPM_INTERP_CUBIC_CLIP = 2, PPM_INTERP_CUBIC_LINMU = 3 };

/*
 * Static description of the model (host memory; copied at plan creation).
 *
 *  mode        S+D (spherical star, Doppler) or OS (oblate Schwarzschild), Sect. 2.2
 *  intensity   isotropic blackbody (App. C) or a 4D atmosphere table (Sect. 2.5)
 *  n_spots     1 or 2; spot s uses params 8+4s .. 11+4s
 *  shape[s]    cap, annulus (inner radius shape_a*zeta) or crescent (mask cap of
 *              radius shape_a*zeta centred shape_b*zeta towards the equator)
 *  n_rings[s], n_phi[s]   spot grid: rings of equal colatitude width, cells of
 *              equal azimuth width per ring (annulus: n_phi even, half per arc)
 *  n_fp        fine rotation phases of the pseudo-patch light curve (Sect. 2.8.3)
 *  n_phase     output phase bins, centres (k + 1/2)/n_phase
 *  n_energy    model energies energy_kev[E] (keV), any increasing grid
 *  n_chan      response channels; rsp[E][C] in cm^2 keV (row-major)
 *  sigma_cm2   absorption cross-section per H atom [E] (NULL: no absorption)
 *  t_exp       exposure [s]; counts per bin = t_exp / n_phase * flux . rsp
 *  nT, ng, nmu, nx, ax_*, log_intensity
 *              atmosphere axes (logT, log g, mu, log(E/kT)) and table
 *              log10(I / T^3) [nT][ng][nmu][nx]; logT, log g and x axes must be
 *              uniformly spaced; ignored for the blackbody model
 *  n_alpha     nodes of the per-ring FP64 deflection table (>= 64)
 *  precision   PPM_F32: FP32 bulk intensity/accumulate, MFMA FP32 fold;
 *              PPM_F64: FP64 throughout (blackbody model only)
 *  grad        1: also allocate what ppm_loglike_grad needs (atmosphere-table
 *              model with the windowed accumulation only); 0: forward only
 *  interp      atmosphere interpolation strategy of Sect. 4: PPM_INTERP_MIXED
 *              (d, the default: linear in logT and log g, cubic in mu and x,
 *              linear in the protected small-mu zone and at the table edges),
 *              PPM_INTERP_CUBIC (a: cubic Lagrange on all four axes, stencils
 *              shifted inward at the axis ends), PPM_INTERP_CUBIC_CLIP (b: (a)
 *              with negative intensities set to zero), PPM_INTERP_CUBIC_LINMU
 *              (c: (a) but linear in the protected zone).  (a)-(c) need at
 *              least four nodes on every axis, run on the generic kernel and
 *              have no gradient.
 *  n_side      0: the spot model above.  > 0 (at most 512): a full-surface
 *              temperature-map plan (Sects. 2.6, 2.8.1): the surface is the
 *              12 n_side^2 equal-area HEALPix patches on 4 n_side - 1 rings,
 *              each with its own temperature given per call to the *_map
 *              entry points; the spot fields are ignored.  Needs the
 *              atmosphere table, PPM_F32, the mixed strategy, grad = 0 and an
 *              energy grid spanning at most 59 x intervals.
 *  background  NULL, or [n_phase][n_chan] expected background counts per bin
 *              (Sect. 6): the likelihood and its gradient use model counts
 *              plus background; ppm_forward's counts stay the model's own.
 *  count_negative
 *              1: count interpolated intensities below zero (the quantity
 *              Sect. 4 compares the strategies by) in ppm_get_diagnostics;
 *              the forward then runs on the generic kernel (slower).  Spot
 *              plans with the atmosphere table and grad = 0 only.  0: not
 *              counted (n_negative = -1).
 */
typedef struct {
    int32_t mode, intensity, n_spots;
    int32_t shape[2], n_rings[2], n_phi[2];
    double shape_a[2], shape_b[2];
    int32_t n_fp, n_phase, n_energy, n_chan;
    const double *energy_kev;
    const double *sigma_cm2;
    const double *rsp;
    double t_exp;
    int32_t nT, ng, nmu, nx;
    const double *ax_T, *ax_g, *ax_mu, *ax_x;
    const double *log_intensity;
    int32_t n_alpha;
    int32_t precision;
    int32_t grad;
    int32_t interp;
    int32_t n_side;
    const double *background;
    int32_t count_negative;
} ppm_spec;

typedef struct ppm_plan ppm_plan;

/* Creates a plan (Sect. 2.9: the tables are set up once and every
 * likelihood call reuses them): validates the spec, uploads tables
 * (atmosphere converted to linear FP32), allocates every device buffer an
 * evaluation of up to max_batch instances needs, and pinned host staging
 * for the work lists.  All device and pinned allocation happens here.
 * max_cells: largest per-spot grid side (rings = cells per ring) that a
 * per-instance resolution override may ask for (0: the spec's own).
 * Synchronises the host (table uploads).  PPM_ERR_ARG / PPM_ERR_UNSUPPORTED
 * for an invalid or unsupported spec, PPM_ERR_ALLOC when memory runs out;
 * *out is NULL on error.
 *
 * Work lists.  Every evaluation needs the list of live (instance, ring)
 * slots and ring groups of its batch layout (B, per-instance grids, ring
 * group).  The plan keeps the lists of eight layouts resident; a call with
 * another layout builds them on the host and uploads them on the call's
 * stream (asynchronously, from pinned staging; the host waits only if the
 * previous upload has not run yet).  A call made while its stream is being
 * captured into a HIP graph must find its layout resident (make one
 * uncaptured call with the same layout first; PPM_ERR_ARG otherwise) and
 * pins it: the lists a graph was captured with are never rewritten, so
 * direct calls with other layouts between replays leave the graph intact.
 * Once all eight slots are pinned, a call with a ninth layout fails with
 * PPM_ERR_UNSUPPORTED (pinned layouts keep working). */
int ppm_plan_create(const ppm_spec *spec, int max_batch, int max_cells, ppm_plan **out);
void ppm_plan_destroy(ppm_plan *plan);

/* Forward model (Sects. 2.3-2.8): counts_dev[B][n_phase][n_chan] (double,
 * device).  params_dev: [B][16] doubles (device).  n_cells_host: NULL, or
 * B ints (host) giving each instance's cells per side for both spots
 * (rings = cells per ring = n), at most the plan's max_cells. */
int ppm_forward(ppm_plan *plan, const double *params_dev, int B, const int32_t *n_cells_host,
                double *counts_dev, void *stream);

/* Photon flux before absorption and response: flux_dev[B][n_phase][n_energy]
 * (ph cm^-2 s^-1 keV^-1, double).  Same arguments as ppm_forward. */
int ppm_flux(ppm_plan *plan, const double *params_dev, int B, const int32_t *n_cells_host,
             double *flux_dev, void *stream);

/* Poisson log-likelihood sum d ln m - m - ln(d!) over all phase-channel bins
 * for each instance (the likelihood a sampler calls, Sect. 6; the model
 * counts are those of Sect. 2.8.4, the Poisson form is the standard one
 * for counted photons): logl_dev[B] (double, device).  data_dev:
 * [n_phase][n_chan] int32 counts shared by all instances (device).
 * counts_dev may be NULL; otherwise it receives the model counts.
 * An instance with a nonzero status gets logL = -inf. */
int ppm_loglike(ppm_plan *plan, const double *params_dev, int B, const int32_t *n_cells_host,
                const int32_t *data_dev, double *logl_dev, double *counts_dev, void *stream);

/* Allocation-free variant of ppm_loglike, for callers that cannot allocate
 * device memory during a call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments and results as
 * ppm_loglike with n_cells_host = NULL (the spec's own grids), computed by
 * the same kernels with the plan's tiles and ring group: logl_dev[B], and
 * counts_dev[B][n_phase][n_chan] unless NULL.  Every per-call buffer is
 * carved from one static device array of 64 MiB per device (held by each
 * device the library runs on until the process ends) and the work lists are
 * built on the device; the call makes no allocation, no host-device copy
 * and no host synchronisation.  The plan supplies its constant tables only.
 * All calls on one device share that array: calls that overlap on a device
 * (two streams, or two plans) race and must be serialised by the caller.
 * PPM_ERR_BATCH when the batch needs more than the 64 MiB (for the
 * 128x128-cell two-spot workload at 128 phases and 256 energies: one
 * instance with one ring per group, four with groups of 16 rings),
 * PPM_ERR_UNSUPPORTED for a temperature-map plan, PPM_ERR_ARG when the
 * current device is not the plan's. */
int ppm_loglike_noalloc(ppm_plan *plan, const double *params_dev, int B, const int32_t *data_dev,
                        double *logl_dev, double *counts_dev, void *stream);

/* Poisson log-likelihood and its gradient with respect to the twelve
 * differentiable parameters, in the order M, R_e, i, Phi, N_H, theta_1,
 * zeta_1, logT_1, theta_2, zeta_2, logT_2, dphi_2 (units of the parameter
 * record): logl_dev[B], grad_dev[B][12] (double, device).  The gradient is
 * the derivative of the discrete model of Sects. 2.3-2.8 as evaluated by
 * ppm_loglike (held fixed: interpolation stencils, visibility ranges, clamps,
 * table node positions in alpha; crescent masks are not differentiated).
 * Reverse mode through Eqs. (22), (55) and the likelihood, reverse mode over
 * energies of Eq. (47), forward-mode tangents of the ring geometry, the
 * deflection table and the fine-phase trace.  An instance with a nonzero
 * status gets logL = -inf and a NaN gradient.  Needs a plan created with
 * spec->grad = 1 (PPM_ERR_UNSUPPORTED otherwise).  Other arguments as
 * ppm_loglike. */
int ppm_loglike_grad(ppm_plan *plan, const double *params_dev, int B, const int32_t *n_cells_host,
                     const int32_t *data_dev, double *logl_dev, double *grad_dev, void *stream);

/* Forward model of a full-surface temperature map (Sects. 2.6, 2.8.1) for a
 * plan created with spec->n_side > 0.  map_dev: [B][12 n_side^2] doubles
 * (device), log10 T [K] per HEALPix patch in ring order (rings from the
 * north pole, pixels by increasing azimuth; patch j of ring i at azimuth
 * phi_first(i) + 2 pi j / n(i), rotated by -2 pi Phi); a value that is not
 * finite or not positive marks a patch that emits nothing.  Temperatures
 * outside the table's logT axis are clamped for the interpolation on that
 * axis (Sect. 4) while x = log10(E / kT) uses the patch's own T; a value more
 * than 64 table steps outside the axis gives the instance PPM_INST_BAD_MAP.
 * Parameter record slots 0-6 as for spots; the spot slots are ignored.
 * counts_dev[B][n_phase][n_chan], flux_dev[B][n_phase][n_energy] and the
 * likelihood as for ppm_forward, ppm_flux and ppm_loglike.  PPM_ERR_ARG on a
 * spot plan (and the spot entry points return it on a map plan). */
int ppm_forward_map(ppm_plan *plan, const double *params_dev, int B, const double *map_dev, double *counts_dev,
                    void *stream);
int ppm_flux_map(ppm_plan *plan, const double *params_dev, int B, const double *map_dev, double *flux_dev,
                 void *stream);
int ppm_loglike_map(ppm_plan *plan, const double *params_dev, int B, const double *map_dev, const int32_t *data_dev,
                    double *logl_dev, double *counts_dev, void *stream);

/* Diagnostic counters of the last evaluation (host; synchronises the
 * stream), summed over its first B instances (total) and per instance
 * (per_instance[B]; either pointer may be NULL, not both):
 *   n_visible_pairs   (cell, phase) pairs with nonzero flux (Eq. 46)
 *   n_clamp_T, n_clamp_g   intensity evaluations whose logT / log g lay
 *                     outside the atmosphere table and was clamped to its
 *                     edge (Sect. 4); a spot ring's values hold for all its
 *                     evaluations, a map patch's logT for its own
 *   n_x_outside       intensity evaluations with x = log10(E / kT) outside
 *                     the table's x axis (no contribution)
 *   n_multi_image     visible fine-phase samples of the ring traces with
 *                     psi > 2 pi - psi_top, i.e. points also seen along a
 *                     second ray, which the model leaves out (Sect. 6);
 *                     zero below GM/(R c^2) ~ 0.28
 *   n_negative        interpolated intensities below zero (Sect. 4), or -1
 *                     when the plan does not count them (spec count_negative)
 * The blackbody model has no table: its clamp, x and negative counts are 0.
 * PPM_ERR_BATCH for B outside [1, max_batch]. */
typedef struct ppm_diag {
    int64_t n_visible_pairs;
    int64_t n_clamp_T;
    int64_t n_clamp_g;
    int64_t n_x_outside;
    int64_t n_multi_image;
    int64_t n_negative;
} ppm_diag;
int ppm_get_diagnostics(ppm_plan *plan, int B, ppm_diag *total, ppm_diag *per_instance, void *stream);

/* Per-instance status codes of the last evaluation: status_dev[B] (device). */
int ppm_instance_status(ppm_plan *plan, int B, int32_t *status_dev, void *stream);

/* Host-side parameter validation with the same rules the device applies;
 * status_host[B].  n_spots 0 checks the star only (temperature maps). */
int ppm_validate_params(const double *params_host, int B, int n_spots, int32_t *status_host);

/* Introspection for tests: copies to host (synchronising the stream) the
 * per-ring FP64 deflection table of instance b, ring r of the last
 * evaluation (b among the instances of its last workspace pass): out[n_alpha][4] = (psi, dpsi/dalpha, c dt/R, d(c dt/R)/dalpha)
 * at alpha_j = alpha_max * j / (n_alpha - 1); info[4] = (alpha_max, psi_top,
 * u, R [cm]).  And the fine-phase trace out_tr[n_fp+1][4] = (F, z, phi_o, mu)
 * with trace_info[3] = (visible, inv_min, inv_max). */
int ppm_debug_ring(ppm_plan *plan, int b, int r, double *table_out, double *info_out,
                   double *trace_out, int32_t *trace_info, void *stream);

/* Number of (cell, phase) pairs with nonzero flux in the last evaluation,
 * summed over instances (host; synchronises the stream). */
int ppm_visible_pairs(ppm_plan *plan, int B, long long *out, void *stream);

/* Workspace passes of the last evaluation (host, no synchronisation): a
 * batch runs in passes of at most the instances whose ring scratch and
 * ring-group partial spectra the plan holds (0 before the first call). */
int ppm_get_passes(const ppm_plan *plan, int *n_passes);

/* Timing of the intensity-accumulation kernel (the hot loop) with HIP events
 * recorded on the caller's stream around each launch, for the next max_calls
 * evaluations.  ppm_profile_end synchronises on the recorded events and
 * returns the summed kernel time [ms] and the number of calls timed. */
int ppm_profile_begin(ppm_plan *plan, int max_calls);
int ppm_profile_end(ppm_plan *plan, double *hot_ms_total, int *n_calls);

/* Launch shape of the two accumulation kernels (the sum of Eq. (47) and its
 * adjoint): phase_tile output phases per work-group of the forward kernel
 * (1..256) and phase_tile_grad per work-group of the adjoint kernel
 * (8..256); ring_group rings summed per work-group of the windowed forward
 * kernel (1..64; one FP32 partial spectrum per group goes to the FP64 ring
 * reduction instead of one per ring).  Forward results do not depend on
 * phase_tile: every phase's sums run in the same order whatever the tile.
 * They depend on ring_group at the FP32 rounding level (a group's rings are
 * summed in FP32, groups in FP64); for a fixed ring_group they are bitwise
 * reproducible, and an instance gives the same bits alone as in a batch.
 * The gradient's per-block partial sums depend on phase_tile_grad, at the
 * rounding level.  Temperature-map plans use phase_tile rounded down to 8,
 * 16 or 32 (8 waves) and one ring per group.  Defaults 8, 8, 1.  A change
 * applies to later calls; a HIP graph captured earlier keeps the shape it
 * was captured with.  PPM_ERR_ARG for a null pointer or a value out of range
 * (the plan is then unchanged). */
typedef struct ppm_tiles {
    int32_t phase_tile;
    int32_t phase_tile_grad;
    int32_t ring_group;
} ppm_tiles;
int ppm_get_tiles(const ppm_plan *plan, ppm_tiles *out);
int ppm_set_tiles(ppm_plan *plan, const ppm_tiles *tiles);

/* Autotuner of the launch shape.  For each candidate phase tile (forward:
 * 4, 8, 12, 16, 20, 24, 28, 32, 48, 64, 96, 128; adjoint, gradient plans only: 8,
 * 16, 24, 32;
 * a candidate that gives the same number of tiles over n_phase as a smaller
 * one is skipped) it times whole evaluations of the given batch (params_dev,
 * B, n_cells_host as for ppm_forward), each between two HIP events on
 * `stream`: about 100 ms of untimed warm-up evaluations first (the device
 * clock ramps up under load), then every candidate once per repetition, in
 * turn, for `reps` repetitions (1..1000).  It keeps the candidate with the
 * smallest median time and sets it on the plan; the forward tile is
 * chosen first, then (windowed spot plans) the ring group among 1, 2, 4, 8,
 * 16 and 32 at that tile, and then the adjoint tile.  Adjoint calls
 * run on all-zero data (their cost does not depend on the data) and need
 * two temporary device buffers, allocated and freed here.  Synchronises the
 * stream; refused on a stream that is being captured.  Spot plans only.
 * On error the plan keeps its previous tiles.  report may be NULL;
 * otherwise it receives every candidate's median time [ms] and the choice. */
#define PPM_TUNE_MAX 16
typedef struct ppm_tune_report {
    int32_t n_fwd, n_grad, n_group;
    int32_t fwd_tile[PPM_TUNE_MAX];
    double fwd_ms[PPM_TUNE_MAX];
    int32_t grad_tile[PPM_TUNE_MAX];
    double grad_ms[PPM_TUNE_MAX];
    int32_t group[PPM_TUNE_MAX];
    double group_ms[PPM_TUNE_MAX];
    ppm_tiles chosen;
} ppm_tune_report;
int ppm_autotune(ppm_plan *plan, const double *params_dev, int B, const int32_t *n_cells_host, int reps,
                 void *stream, ppm_tune_report *report);
/* The same for a temperature-map plan over map_dev (as for ppm_forward_map):
 * candidates 8, 16 and 32 phases per work-group of the map kernel. */
int ppm_autotune_map(ppm_plan *plan, const double *params_dev, int B, const double *map_dev, int reps,
                     void *stream, ppm_tune_report *report);

/*
 * GPU-resident parallel-tempered Metropolis sampler (the inference layer
 * named in Sect. 6): C chains at each of T inverse temperatures, every step
 * one batched likelihood call of the T*C proposals, all on the device with
 * no host synchronisation.
 *   move     theta'_j = theta_j + step[j] / sqrt(beta_t) z_j on the free
 *            slots (z standard normal), accepted when theta' lies in the
 *            uniform prior box [lo, hi] and log u < beta_t (L' - L)
 *            (an invalid proposal has L' = -inf and is rejected);
 *   swap     after every swap_every-th step n, for each chain the pairs
 *            (t, t+1) with t of parity (n / swap_every) mod 2 exchange
 *            states when log u < (beta_t - beta_{t+1}) (L_{t+1} - L_t).
 * Random numbers: Philox4x32-10 (Salmon et al. 2011) with counter
 * (n mod 2^32, n div 2^32, t*C + c, purpose << 16 | k), key (seed mod 2^32,
 * seed div 2^32), purpose 0 proposal (k = pair of free slots, Box-Muller of
 * two 53-bit uniforms taken from words (0,1) and (2,3)), 1 acceptance, 2 swap.
 * Layouts (device, caller-owned): state and proposals [T][C][16] doubles
 * (slots not free are carried unchanged), log-likelihoods [T][C],
 * acceptance counts [T][C] int32, swap counts [T-1][C] int32 (pair t).
 * The sampler owns its state and scratch (allocated at creation); its calls
 * are asynchronous on the given stream, and it must not be used from two
 * streams at once.
 */
#define PPM_PT_MAX_TEMPS 64
typedef struct ppm_pt_config {
    int32_t n_chains;               /* C >= 1 */
    int32_t n_temps;                /* T in [1, 64] */
    int32_t n_free;                 /* free slots, 1 .. 16 */
    int32_t free_slot[16];          /* their places in the parameter record, distinct, 0 .. 15 */
    double lo[16], hi[16];          /* uniform prior box per free slot, lo < hi */
    double step[16];                /* proposal standard deviation at beta = 1, > 0 */
    double beta[PPM_PT_MAX_TEMPS];  /* inverse temperatures in (0, 1], strictly decreasing */
    uint64_t seed;
    int32_t swap_every;             /* swap round after every k-th step; 0: no swaps */
} ppm_pt_config;

typedef struct ppm_pt ppm_pt;

/* Creates a sampler (validates the configuration, allocates its device
 * state).  PPM_ERR_ARG on an invalid configuration. */
int ppm_pt_create(const ppm_pt_config *cfg, ppm_pt **out);
void ppm_pt_destroy(ppm_pt *pt);
/* Sets the state [T][C][16] and its log-likelihoods [T][C] (logl_dev NULL:
 * -inf, so that the first finite proposals are accepted), the step counter
 * n, and zeroes the acceptance and swap counts. */
int ppm_pt_set_state(ppm_pt *pt, const double *params_dev, const double *logl_dev, int64_t step, void *stream);
/* Proposals of the current step into prop_dev [T][C][16]. */
int ppm_pt_propose(ppm_pt *pt, double *prop_dev, void *stream);
/* Acceptance of the current step's proposals given their log-likelihoods
 * prop_logl_dev [T][C], then the swap round when due; advances the step
 * counter. */
int ppm_pt_accept(ppm_pt *pt, const double *prop_dev, const double *prop_logl_dev, void *stream);
/* n_steps steps of propose -> ppm_loglike(plan, T*C proposals, data_dev) ->
 * accept, all launched on the stream without synchronisation.  chain_dev
 * [n_steps][C][16] and chain_logl_dev [n_steps][C] (either may be NULL)
 * receive the cold chains (t = 0) after each step.  The plan must be a spot
 * plan with max_batch >= T*C. */
int ppm_pt_run(ppm_pt *pt, ppm_plan *plan, const int32_t *data_dev, int n_steps, double *chain_dev,
               double *chain_logl_dev, void *stream);
/* Copies the state, its log-likelihoods and the counts (device pointers,
 * each may be NULL) and returns the step counter (host). */
int ppm_pt_get_state(ppm_pt *pt, double *params_dev, double *logl_dev, int32_t *n_accept_dev, int32_t *n_swap_dev,
                     int64_t *step, void *stream);

/*
 * Instrument pipeline of Sect. 2.8.4 (host functions, no device work).
 * ppm_arf_read / ppm_rmf_read read OGIP FITS files (CAL/GEN/92-002): the
 * ARF's SPECRESP extension (ENERG_LO, ENERG_HI [keV], SPECRESP [cm^2]) and
 * the RMF's MATRIX (or SPECRESP MATRIX) extension (ENERG_LO, ENERG_HI, N_GRP,
 * F_CHAN, N_CHAN, MATRIX, fixed-width or variable-length columns; first
 * channel from TLMIN of F_CHAN, default 1; channel count from DETCHANS or the
 * EBOUNDS rows) and EBOUNDS (E_MIN, E_MAX).  Two calls: with every output
 * array NULL only the sizes are returned; then arrays of n_energy
 * (e_lo, e_hi, area), n_energy x n_chan row-major (matrix, dense probabilities)
 * and n_chan (ch_lo, ch_hi; may be NULL).  PPM_ERR_ARG for an unreadable file
 * or a missing extension or column (see ppm_last_error).
 *
 * ppm_response_build: RSP[i][c] = sum_e DS[i][e] A[e] R[e][c] for the model
 * energies e_model[n_model] (increasing), where DS[i][e] is the integral of
 * the piecewise-linear hat function of model energy i (constant beyond the
 * grid's ends) over the fine bin [e_lo[e], e_hi[e]]; area NULL means A = 1.
 * rsp[n_model][n_chan] in the units of A times keV, ready for
 * ppm_spec.rsp.  Absorption is not folded in: it stays exp(-N_H sigma) per
 * evaluation with N_H a parameter.
 *
 * ppm_sigma_from_table: the cross-section per H atom at energies e[n] from a
 * transmission table (e_tab increasing, att_tab in (0, 1]) at the reference
 * column nh_ref [cm^-2], linear in energy between table nodes and constant
 * beyond them: sigma = -ln(transmission) / nh_ref, so that exp(-N_H sigma) is
 * the table value to the power N_H / nh_ref.
 */
int ppm_arf_read(const char *path, int32_t *n_energy, double *e_lo, double *e_hi, double *area);
int ppm_rmf_read(const char *path, int32_t *n_energy, int32_t *n_chan, double *e_lo, double *e_hi, double *matrix,
                 double *ch_lo, double *ch_hi);
int ppm_response_build(int32_t n_model, const double *e_model, int32_t n_fine, const double *e_lo, const double *e_hi,
                       const double *area, int32_t n_chan, const double *matrix, double *rsp);
int ppm_sigma_from_table(int32_t n_tab, const double *e_tab, const double *att_tab, double nh_ref, int32_t n,
                         const double *e, double *sigma);

const char *ppm_status_string(int code);
const char *ppm_last_error(void);
int ppm_version(void);

#ifdef __cplusplus
}
#endif
#endif
