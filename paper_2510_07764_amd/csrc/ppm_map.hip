// Full-surface temperature maps on HEALPix (Sects. 2.6, 2.8.1): the whole
// stellar surface is divided into 12 n_side^2 equal-area patches on
// 4 n_side - 1 iso-latitude rings, each patch with its own temperature
// (inactive patches emit nothing).  The ring machinery of the spot model
// (setup, FP64 deflection table, fine-phase trace, ring reduction, fold)
// is shared; what differs is that the (logT, log g) collapse of the
// atmosphere table can no longer be done once per ring.
//
//   k_map_sort    per ring: buckets the active patches by logT table
//                 interval (stable counting sort), so that patches sharing
//                 the two logT nodes of their linear interpolation are
//                 processed together
//   k_accum_map   shift-and-add (Eq. 47) per (ring, 8, 16 or 32 phases),
//                 8 waves: for each bucket, the two logT slabs collapsed
//                 in log g over the bucket's x window go to LDS, then the
//                 windowed scheme of the spot kernel with the logT weight
//                 applied inside the mu contraction
// Section and equation numbers refer to arXiv:2510.07764.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ppm_internal.h"
#include "ppm_device.h"
#include "ppm_launch.h"
#include "../../include/ppm.h"

namespace ppm {

// bucket of a map value: -1 inactive patch (not finite or not positive),
// -2 further than kMapLow table steps outside the logT axis
__device__ inline int map_bucket(const DevSpec &S, double lt)
{
    if (!(isfinite(lt) && lt > 0.0)) return -1;
    const double u = floor((lt - S.T0) / S.hT);
    if (u < -kMapLow || u >= S.map_nb - kMapLow) return -2;
    return (int)u + kMapLow;
}

// ---------------------------------------------------------------------------
// k_map_sort: one block per (instance, ring).  Pass 1 histograms the ring's
// active patches over the temperature buckets, the offsets go to grp; pass 2
// places each patch at its bucket offset plus its rank among the earlier
// patches of the same bucket (stable, so the accumulation order over patches
// is fixed).  A ring without active patches is switched off (n_cells = 0)
// before the table and trace kernels run.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_map_sort(DevSpec S, const int32_t *list, const double *map, StarRec *stars,
                                                  RingRec *rings, MapCell *cells, int32_t *grp)
{
    const int ent = list[blockIdx.x], b = ent / S.R_tot, r = ent - b * S.R_tot;
    RingRec *gp = rings + (size_t)b * S.R_tot + r;
    const int n = gp->n_cells;   // pixels of the ring; 0 when the instance is not evaluated
    const int NB = S.map_nb;
    extern __shared__ int lds_i[];
    int *cnt = lds_i, *run = lds_i + NB, *qch = run + NB;   // NB, NB, blockDim.x
    __shared__ int bad, total;
    const int tid = threadIdx.x;
    for (int q = tid; q < NB; q += blockDim.x) cnt[q] = 0;
    if (tid == 0) bad = 0;
    __syncthreads();
    const long long pix0 = healpix_first_pixel(S.n_side, r + 1);
    const double *mrow = map + (size_t)b * S.n_pix + pix0;
    for (int j = tid; j < n; j += blockDim.x) {
        const int q = map_bucket(S, mrow[j]);
        if (q >= 0) atomicAdd(&cnt[q], 1);
        else if (q == -2) bad = 1;
    }
    __syncthreads();
    int32_t *gr = grp + ((size_t)b * S.R_tot + r) * (NB + 1);
    if (tid == 0) {
        int acc = 0;
        for (int q = 0; q < NB; ++q) {
            run[q] = acc;
            gr[q] = acc;
            acc += cnt[q];
        }
        gr[NB] = acc;
        total = acc;
    }
    __syncthreads();
    MapCell *out = cells + (size_t)b * S.n_pix + pix0;
    for (int j0 = 0; j0 < n; j0 += blockDim.x) {
        const int j = j0 + tid;
        const double lt = j < n ? mrow[j] : 0.0;
        const int q = j < n ? map_bucket(S, lt) : -1;
        qch[tid] = q;
        __syncthreads();
        if (q >= 0) {
            int rank = 0;
            for (int t = 0; t < tid; ++t) rank += qch[t] == q;
            const int u = q - kMapLow;
            const int it = u < 0 ? 0 : (u > S.nT - 2 ? S.nT - 2 : u);
            double w = (lt - S.T0) / S.hT - it;     // linear in logT, clamped at the axis ends
            w = fmin(1.0, fmax(0.0, w));
            MapCell c;
            c.lkT = log10(kKB) + lt;
            c.t = (float)w;
            c.T3 = (float)pow(10.0, 3.0 * (lt - 6.0));
            c.j = j;
            c.clamped = (lt < S.T_end[0] || lt > S.T_end[1]) ? 1 : 0;   // logT clamped for the table (Sect. 4)
            out[run[q] + rank] = c;
        }
        __syncthreads();
        for (int qq = tid; qq < NB; qq += blockDim.x) {
            int c = 0;
            for (int t = 0; t < (int)blockDim.x; ++t) c += qch[t] == qq;
            run[qq] += c;
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (total == 0) gp->n_cells = 0;
        if (bad && stars[b].status == PPM_INST_OK) stars[b].status = PPM_INST_BAD_MAP;
    }
}

// ---------------------------------------------------------------------------
// k_accum_map: block = (ring, 8 KPW output phases), 8 waves, wave w owns
// phases 8 KPW tile + w + 8 q (q < KPW) and EPL energies, 64 apart, per
// lane; the staged slabs of a bucket serve all of the block's phases.  The
// ring's active patches, sorted by temperature bucket, go through in groups
// of 64:
//   stage A  lane = patch of the group, for each of the wave's phases:
//            observed-phase lookup (Eqs. 45-46), mu weights of the mixed
//            scheme pre-scaled by F_p (T / 10^6 K)^3, logT weight, x position
//            of the first energy (kept in registers);
// then, for each bucket (logT nodes it, it + 1 after clamping) holding
// patches of the group, in order:
//   staging  (unless the bucket is still staged from the previous group) the
//            table slabs at logT nodes it and it + 1 (x-major, the two
//            interleaved), linear in the ring's log g, over the x window the
//            bucket's patches can reach (redshift range of the ring, bucket's
//            kT range, energy span and the cubic stencil);
//   stage B  per visible pair of the group in the bucket: mu contraction of
//            both slabs and their logT blend at x node I0 - 1 + lane, cubic
//            coefficients of interval I0 + lane (next nodes by DPP wave
//            shifts; linear in the first and last table interval, zero
//            outside), per energy one quad read and a Horner step.
// The pairs are summed in the order of the sorted patches.
// ---------------------------------------------------------------------------
// Stage B of k_accum_map for the visible pairs (mask) of one 64-patch group
// of a bucket.  INTERIOR: the bucket's x window stays one interval clear of
// the table's first and last intervals (every interval an energy can use is
// cubic and every stencil column lies in the staged window), so the bounds
// tests drop out; columns past the window are read but never reach a quad
// an energy uses.
template <int EPL, bool INTERIOR>
__device__ __forceinline__ void map_pairs(uint64_t mask, float w0f, float w1f, float w2f, float w3f, float fr,
                                          float tw, int pk, int lane, const float2 *slb, int NMP,
                                          int WM, int w0, int xw, int nx, float4 *Qw,
                                          const float (&tbr)[EPL], float (&acc)[EPL])
{
    while (mask) {
        const int p = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const float pw0 = readlane_f(w0f, p), pw1 = readlane_f(w1f, p), pw2 = readlane_f(w2f, p),
                    pw3 = readlane_f(w3f, p), pfr = readlane_f(fr, p), ptw = readlane_f(tw, p);
        const int ppk = __builtin_amdgcn_readlane(pk, p);
        const int pI0 = ppk >> 8, pm0 = ppk & 255;
        int col = pI0 - 1 + lane - w0;
        float Sv = 0.0f;
        if (INTERIOR || (col >= 0 && col < xw)) {
            if (INTERIOR) col = col < WM - 1 ? col : WM - 1;
            // the four mu rows of both slabs at this x node: adjacent pairs
            // (24-bit multiply-add on the byte offset)
            const float2 *t = (const float2 *)((const char *)(slb + pm0) + __umul24((unsigned)col, 8u * NMP));
            const float2 a = t[0], b = t[1], c = t[2], d = t[3];
            const float v0 = pw0 * a.x + pw1 * b.x + pw2 * c.x + pw3 * d.x;
            const float v1 = pw0 * a.y + pw1 * b.y + pw2 * c.y + pw3 * d.y;
            Sv = v0 + ptw * (v1 - v0);
        }
        const float s1 = wave_next_f(Sv), s2 = wave_next_f(s1), s3 = wave_next_f(s2);
        float4 qd = make_float4(0.f, 0.f, 0.f, 0.f);
        const int gi = pI0 + lane;
        if (INTERIOR || (gi >= 1 && gi <= nx - 3)) {
            const float c2 = 0.5f * (Sv + s2) - s1;
            const float c3 = (s3 - Sv) * (1.0f / 6.0f) + 0.5f * (s1 - s2);
            qd = make_float4(s1, s2 - s1 - c2 - c3, c2, c3);
        } else if (gi == 0 || gi == nx - 2) {
            qd = make_float4(s1, s2 - s1, 0.f, 0.f);
        }
        Qw[lane] = qd;
        wave_sync();
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            const float t = pfr + tbr[m];
            const float f = __builtin_amdgcn_fractf(t);
            const float4 qv = Qw[(int)t];
            acc[m] += qv.x + f * (qv.y + f * (qv.z + f * qv.w));
        }
        wave_sync();
    }
}

// The partial of work-list entry li goes to partial[li] (groups of one ring).
template <int EPL, int KPW>
__global__ __launch_bounds__(64 * kMapWaves) void k_accum_map(DevSpec S, const int32_t *list, const RingRec *rings,
                                                             const double4 *trace, const MapCell *cells,
                                                             const int32_t *grp, float *partial, int32_t *vis_pairs,
                                                             int32_t *diag, int n_list)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    constexpr int PT = kMapWaves * KPW;
    const int n_tile = (S.P + PT - 1) / PT;
    int li, tile;
    if (!xcd_block(n_list, n_tile, li, tile)) return;
    const int ent = list[li], b = ent / S.R_tot, r = ent - b * S.R_tot;
    const size_t slot = (size_t)b * S.R_tot + r;
    const RingRec g = rings[slot];
    if (!g.active) return;
    const int nfp = S.n_fp, nmu = S.nmu, nx = S.nx, E = S.E, P = S.P, WM = S.map_wm, NB = S.map_nb;
    double4 *tr = (double4 *)lds_raw;                          // nfp + 1
    double *po = (double *)(tr + nfp + 1);                     // nfp + 1, padded to even
    double *axmu = po + ((nfp + 2) & ~1);                      // nmu, padded to even
    // the two logT slabs, x-major and interleaved: (slab 0, slab 1) of mu row m
    // at x node c in slb[c NMP + m], node stride NMP = nmu | 1
    const int NMP = fast_tab_stride(nmu);
    float2 *slb = (float2 *)(axmu + ((nmu + 1) & ~1));         // NMP * WM
    float4 *Qb = (float4 *)(slb + ((NMP * WM + 1) & ~1));      // kMapWaves * 64 quads
    double *ipo = (double *)(Qb + kMapWaves * 64);             // nfp: 1 / (phi_o[i+1] - phi_o[i])
    double *mcf = ipo + nfp + 1;                               // nmu * 4 mu-interval coefficients
    int16_t *pbk = (int16_t *)(mcf + 4 * nmu);                 // 2 nfp phase buckets
    int16_t *mbk = pbk + 2 * nfp;                              // mu_nb mu buckets
    float *tbl = (float *)(mbk + ((S.mu_nb + 1) & ~1));        // E: the energies' x offsets
    // (bucket, first patch) of the non-empty buckets, 8-byte aligned
    int2 *nel = (int2 *)(lds_raw + ((((unsigned char *)(tbl + E) - lds_raw) + 7) & ~7));
    const int n_pb = 2 * nfp;
    const int tid = threadIdx.x;
    const double4 *gtr = trace + slot * (nfp + 1);
    // LDS trace per fine-phase sample i: (F, z_{i+1}/z_i - 1, x position of
    // E_0 at z_i and kT = 1 keV, mu); phi_o in po
    for (int i = tid; i <= nfp; i += blockDim.x) {
        const double4 v = gtr[i];
        const double zn = i < nfp ? gtr[i + 1].y : v.y;
        tr[i] = make_double4(v.x, zn / v.y - 1.0, log10(v.y) * S.ihx + S.tb0, v.w);
        po[i] = v.z;
    }
    for (int i = tid; i < nmu; i += blockDim.x) axmu[i] = S.ax_mu[i];
    for (int i = tid; i < 4 * nmu; i += blockDim.x) mcf[i] = S.mu_coef[i];
    for (int i = tid; i < S.mu_nb; i += blockDim.x) mbk[i] = S.mu_bucket[i];
    for (int e = tid; e < E; e += blockDim.x) tbl[e] = S.tbe[e];
    __syncthreads();
    // phase buckets and inverse spacings of phi_o, as in the spot kernel
    for (int q = tid; q < n_pb; q += blockDim.x) {
        const double edge = po[0] + (double)q / n_pb;
        int l0 = 0, h0 = nfp;
        while (h0 - l0 > 1) {
            int mid = (l0 + h0) >> 1;
            if (po[mid] <= edge) l0 = mid; else h0 = mid;
        }
        pbk[q] = (int16_t)l0;
    }
    for (int i = tid; i < nfp; i += blockDim.x) ipo[i] = 1.0 / (po[i + 1] - po[i]);
    const int wave = tid >> 6, lane = tid & 63;
    const int32_t *gr = grp + slot * (NB + 1);
    if (wave == 0) {
        // the non-empty buckets in order, with the sentinel (NB, active patches)
        int cnt = 0;
        for (int q0 = 0; q0 < NB; q0 += 64) {
            const int q = q0 + lane;
            const int a0 = gr[q < NB ? q : NB], a1 = gr[q < NB ? q + 1 : NB];
            const bool ne = q < NB && a1 > a0;
            const uint64_t m = __ballot(ne);
            if (ne) nel[cnt + __popcll(m & ((1ull << lane) - 1ull))] = make_int2(q, a0);
            cnt += __popcll(m);
        }
        if (lane == 0) nel[cnt] = make_int2(NB, gr[NB]);
    }
    __syncthreads();   // phase buckets, spacings and the bucket list are in place
    float4 *Qw = Qb + wave * 64;
    const double ihx = S.ihx;
    float tbr[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
        int e = lane + 64 * m;     // energies 64 apart: neighbouring lanes read neighbouring quads
        tbr[m] = e < E ? S.tbe[e] : 0.0f;
    }
    const double mu_lo = S.mu_lo, mu_hi = S.mu_hi;
    const double inv2pi = 1.0 / kTwoPi;
    const double phio0 = gtr[0].z;
    const int k_first = tile * PT + wave;
    double wg1;
    const int ig = lin_bracket(g.logg, S.g0, S.hg, S.ng, wg1);
    const float fg1 = (float)wg1, fg0 = (float)(1.0 - wg1);
    const double lz_lo = log10(g.zmin), lz_hi = log10(g.zmax);
    const double lkb = log10(kKB);
    const MapCell *cl = cells + (size_t)b * S.n_pix + healpix_first_pixel(S.n_side, r + 1);
    const size_t slab = (size_t)nmu * nx;
    float acc[KPW][EPL];
#pragma unroll
    for (int kq = 0; kq < KPW; ++kq)
#pragma unroll
        for (int m = 0; m < EPL; ++m) acc[kq][m] = 0.0f;
    int npairs = 0, nclamp = 0, nxout = 0;
    const int n_act = gr[NB];   // active patches of the ring, sorted by bucket
    int staged = -1, w0 = 0, xw = 0, iq = 0;
    bool interior = false;
    for (int c0 = 0; c0 < n_act; c0 += 64) {
        const int c1 = c0 + 64 < n_act ? c0 + 64 : n_act;
        // ---------------- stage A: lane = patch c0 + lane, for each of the
        // wave's phases (whatever the patch's bucket)
        const int cc = c0 + lane;
        const MapCell mc = cl[cc < c1 ? cc : c1 - 1];
        const double off = cell_offset(g, mc.j);
        float W0[KPW], W1[KPW], W2[KPW], W3[KPW], FR[KPW], TW[KPW];
        int PK[KPW];
        uint64_t MK[KPW];
#pragma unroll
        for (int kq = 0; kq < KPW; ++kq) {
            const int k = k_first + kMapWaves * kq;
            const double Phik = (k + 0.5) / S.Pd;
            bool vis = false, clamped = false;
            float w0f = 0.f, w1f = 0.f, w2f = 0.f, w3f = 0.f, fr = 0.f;
            int I0 = 0, m0 = 0;
            if (cc < c1 && k < P) {
                double a = Phik + (g.phi_spot + off) * inv2pi + 1.0 - phio0;
                double php = (a - floor(a)) + phio0;                    // Eq. (45)
                int qb = (int)((php - phio0) * S.fpb);                 // Eq. (46): bucket, bounded scan
                int l0 = pbk[qb < n_pb - 1 ? qb : n_pb - 1];
                while (l0 > 0 && po[l0] > php) --l0;
                while (l0 < nfp - 1 && po[l0 + 1] <= php) ++l0;
                const double4 A = tr[l0], Cn = tr[l0 + 1];
                double wp = (php - po[l0]) * ipo[l0];
                wp = fmin(1.0, fmax(0.0, wp));
                const double Fp = A.x + wp * (Cn.x - A.x);
                if (Fp != 0.0) {
                    vis = true;
                    const double mu = fmin(mu_hi, fmax(mu_lo, A.w + wp * (Cn.w - A.w)));
                    int qm = (int)((mu - mu_lo) * S.mu_ibw);               // bucket, bounded scan
                    int lo = mbk[qm < S.mu_nb - 1 ? qm : S.mu_nb - 1];
                    while (lo > 0 && axmu[lo] > mu) --lo;
                    while (lo < nmu - 2 && axmu[lo + 1] <= mu) ++lo;
                    const double *cf = mcf + 4 * lo;
                    double v0, v1, v2, v3;
                    if (lo < 3 || lo == nmu - 2) {
                        const double t = (mu - axmu[lo]) * cf[0];
                        m0 = lo < nmu - 4 ? lo : nmu - 4;
                        const int sl = lo - m0;
                        v0 = sl == 0 ? 1.0 - t : 0.0;
                        v1 = sl == 0 ? t : (sl == 1 ? 1.0 - t : 0.0);
                        v2 = sl == 1 ? t : (sl == 2 ? 1.0 - t : 0.0);
                        v3 = sl == 2 ? t : 0.0;
                    } else {
                        m0 = lo - 1;
                        const double d0 = mu - axmu[m0], d1 = mu - axmu[m0 + 1], d2 = mu - axmu[m0 + 2],
                                     d3 = mu - axmu[m0 + 3];
                        const double p01 = d0 * d1, p23 = d2 * d3;
                        v0 = d1 * p23 * cf[0];
                        v1 = d0 * p23 * cf[1];
                        v2 = p01 * d3 * cf[2];
                        v3 = p01 * d2 * cf[3];
                    }
                    const double sc = Fp * (double)mc.T3;
                    w0f = (float)(v0 * sc);
                    w1f = (float)(v1 * sc);
                    w2f = (float)(v2 * sc);
                    w3f = (float)(v3 * sc);
                    // x position at zp = z_A (1 + wp q_A) and the patch's kT
                    const double T0 = A.z + (double)x_shift(wp * A.y, S.ixl) - mc.lkT * ihx;
                    const double fl = floor(T0);
                    I0 = (int)fl;
                    fr = (float)(T0 - fl);
                    clamped = mc.clamped != 0;
                    // energies beyond the table's x range contribute nothing
                    // (counted; never the case in a bucket clear of the table's edges)
                    if (I0 < 0 || (float)I0 + fr + tbl[E - 1] >= (float)(nx - 2))
                        nxout += x_outside_count(I0, fr, tbl, E, nx);
                }
            }
            W0[kq] = w0f;
            W1[kq] = w1f;
            W2[kq] = w2f;
            W3[kq] = w3f;
            FR[kq] = fr;
            TW[kq] = mc.t;
            PK[kq] = (I0 << 8) | m0;
            MK[kq] = __ballot(vis);
            npairs += __popcll(MK[kq]);
            nclamp += __popcll(__ballot(clamped));
        }
        // ---------------- stage B: the buckets holding patches c0 .. c1 - 1,
        // in order; a bucket that goes on into the next group stays staged
        for (;;) {
            const int q = __builtin_amdgcn_readfirstlane(nel[iq].x);
            const int beg = __builtin_amdgcn_readfirstlane(nel[iq].y);
            const int end = __builtin_amdgcn_readfirstlane(nel[iq + 1].y);
            if (q != staged) {
                const int u = q - kMapLow;
                const int it = u < 0 ? 0 : (u > S.nT - 2 ? S.nT - 2 : u);
                // x window of the bucket: t = (log10(z E / kT) - x0) / hx over the
                // ring's z range, the bucket's kT range and the energy grid
                const double lkt_lo = lkb + S.T0 + u * S.hT, lkt_hi = lkt_lo + S.hT;
                const double tlo = (lz_lo - lkt_hi) * ihx + S.tb0, thi = (lz_hi - lkt_lo) * ihx + S.tb0 + S.r_span;
                w0 = (int)floor(tlo) - 2;
                int w1 = (int)floor(thi) + 3;
                w0 = w0 < 0 ? 0 : w0;
                w1 = w1 > nx - 1 ? nx - 1 : w1;
                xw = w1 - w0 + 1;
                xw = xw < 0 ? 0 : (xw > WM ? WM : xw);
                // every interval a pair of the bucket uses lies in [floor(tlo),
                // floor(thi)] up to one interval of slip (as for the spot rings)
                interior = floor(tlo) >= 2.0 && floor(thi) <= nx - 4 && w1 - w0 + 1 <= WM;
                __syncthreads();   // the previous bucket's slabs are no longer read
                const float *a00 = S.atm + ((size_t)it * S.ng + ig) * slab, *a01 = a00 + slab;
                const float *a10 = S.atm + ((size_t)(it + 1) * S.ng + ig) * slab, *a11 = a10 + slab;
                // wave w stages rows w, w + 8, ..., two rows and 128 columns per
                // round: the round's sixteen loads (at clamped, valid indices)
                // are issued before any of them is waited for
                for (int mA = wave; mA < nmu; mA += 2 * kMapWaves) {
                    const bool hasB = mA + kMapWaves < nmu;
                    const int mB = hasB ? mA + kMapWaves : mA;
                    const size_t oA = (size_t)mA * nx + w0, oB = (size_t)mB * nx + w0;
                    for (int cb = 0; cb < xw; cb += 128) {
                        const int c0 = cb + lane, c1 = cb + 64 + lane;
                        const int d0 = c0 < xw ? c0 : xw - 1, d1 = c1 < xw ? c1 : xw - 1;
                        const float p0 = a00[oA + d0], p1 = a01[oA + d0], p2 = a10[oA + d0], p3 = a11[oA + d0];
                        const float q0 = a00[oA + d1], q1 = a01[oA + d1], q2 = a10[oA + d1], q3 = a11[oA + d1];
                        const float r0 = a00[oB + d0], r1 = a01[oB + d0], r2 = a10[oB + d0], r3 = a11[oB + d0];
                        const float t0 = a00[oB + d1], t1 = a01[oB + d1], t2 = a10[oB + d1], t3 = a11[oB + d1];
                        const float2 vp = make_float2(fg0 * p0 + fg1 * p1, fg0 * p2 + fg1 * p3);
                        const float2 vq = make_float2(fg0 * q0 + fg1 * q1, fg0 * q2 + fg1 * q3);
                        const float2 vr = make_float2(fg0 * r0 + fg1 * r1, fg0 * r2 + fg1 * r3);
                        const float2 vt = make_float2(fg0 * t0 + fg1 * t1, fg0 * t2 + fg1 * t3);
                        if (c0 < xw) slb[c0 * NMP + mA] = vp;
                        if (c1 < xw) slb[c1 * NMP + mA] = vq;
                        if (hasB && c0 < xw) slb[c0 * NMP + mB] = vr;
                        if (hasB && c1 < xw) slb[c1 * NMP + mB] = vt;
                    }
                }
                __syncthreads();
                staged = q;
            }
            // lanes of this group whose patch lies in bucket q
            const int lo = (beg > c0 ? beg : c0) - c0, hi = (end < c1 ? end : c1) - c0;
            const uint64_t rng = (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~((1ull << lo) - 1ull);
#pragma unroll
            for (int kq = 0; kq < KPW; ++kq) {
                const uint64_t mask = MK[kq] & rng;
                if (!mask) continue;
                if (interior)
                    map_pairs<EPL, true>(mask, W0[kq], W1[kq], W2[kq], W3[kq], FR[kq], TW[kq], PK[kq], lane, slb,
                                         NMP, WM, w0, xw, nx, Qw, tbr, acc[kq]);
                else
                    map_pairs<EPL, false>(mask, W0[kq], W1[kq], W2[kq], W3[kq], FR[kq], TW[kq], PK[kq], lane, slb,
                                          NMP, WM, w0, xw, nx, Qw, tbr, acc[kq]);
            }
            if (end > c1) break;
            ++iq;
            if (end == c1) break;
        }
    }
    const double scale = g.w_cell * g.T * g.T * g.T;   // g.T = 10^6 K, the patches' reference
#pragma unroll
    for (int kq = 0; kq < KPW; ++kq) {
        const int k = k_first + kMapWaves * kq;
        if (k >= P) break;
        float *out = partial + ((size_t)li * P + k) * E;
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            int e = lane + 64 * m;
            if (e < E) out[e] = (float)(acc[kq][m] * (scale / S.energy[e]));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nxout += __shfl_xor(nxout, o, 64);
    if (lane == 0 && npairs) atomicAdd(&vis_pairs[slot], npairs);
    if (lane == 0 && nclamp) atomicAdd(&diag[slot * kDiagFields + 4], nclamp);
    if (lane == 0 && nxout) atomicAdd(&diag[slot * kDiagFields + 2], nxout);
}

size_t accum_map_lds(const DevSpec &S)
{
    return sizeof(double4) * (S.n_fp + 1) + sizeof(double) * ((S.n_fp + 2) & ~1) + sizeof(double) * ((S.nmu + 1) & ~1)
         + sizeof(float2) * (size_t)((fast_tab_stride(S.nmu) * S.map_wm + 1) & ~1) + sizeof(float4) * kMapWaves * 64
         + sizeof(double) * (S.n_fp + 1) + sizeof(double) * 4 * S.nmu
         + sizeof(int16_t) * (2 * S.n_fp + ((S.mu_nb + 1) & ~1)) + sizeof(float) * S.E + 8
         + sizeof(int2) * (S.map_nb + 1);
}

hipError_t launch_forward_map(const DevSpec &S, const Workspace &W, const double *params, const double *map, int B,
                              const int32_t *list, int n_list, int n_groups, hipStream_t st, double *flux_out,
                              double *counts_out, const int32_t *data, double *logl, hipEvent_t ev_hot0,
                              hipEvent_t ev_hot1)
{
    (void)n_groups;   // groups of one ring: the group list is the identity
    launch_setup(S, W, params, nullptr, B, st);
    hipLaunchKernelGGL(k_map_sort, dim3(n_list), dim3(256), sizeof(int) * (2 * S.map_nb + 256), st, S, list, map,
                       W.stars, W.rings, W.mcell, W.mgrp);
    launch_table_trace(S, W, list, n_list, st);
    const int kpw = S.pt_fwd >= 4 * kMapWaves ? 4 : (S.pt_fwd >= 2 * kMapWaves ? 2 : 1);
    const int n_tile = (S.P + kMapWaves * kpw - 1) / (kMapWaves * kpw);
    const size_t lds = accum_map_lds(S);
    const int epl = (S.E + 63) / 64;
    if (ev_hot0) (void)hipEventRecord(ev_hot0, st);
#define PPM_MAP_LAUNCH(E_, K_)                                                                                   \
    hipLaunchKernelGGL((k_accum_map<E_, K_>), grid, dim3(64 * kMapWaves), lds, st, S, sl, W.rings, W.trace,     \
                       W.mcell, W.mgrp, W.partial32 + (size_t)off * S.P * S.E, W.vis_pairs, W.diag, n)
#define PPM_MAP_KPW(E_)                          \
    do {                                         \
        if (kpw == 1) PPM_MAP_LAUNCH(E_, 1);     \
        else if (kpw == 2) PPM_MAP_LAUNCH(E_, 2); \
        else PPM_MAP_LAUNCH(E_, 4);              \
    } while (0)
    const int step = max_list_per_launch(n_tile, 64 * kMapWaves);
    for (int off = 0; off < n_list; off += step) {
        const int32_t *sl = list + off;
        const int n = n_list - off < step ? n_list - off : step;
        dim3 grid(xcd_grid(n, n_tile));
        if (epl <= 1)
            PPM_MAP_KPW(1);
        else if (epl <= 2)
            PPM_MAP_KPW(2);
        else if (epl <= 4)
            PPM_MAP_KPW(4);
        else
            PPM_MAP_KPW(8);
    }
#undef PPM_MAP_KPW
#undef PPM_MAP_LAUNCH
    if (ev_hot1) (void)hipEventRecord(ev_hot1, st);
    launch_reduce_fold32(S, W, list, B, st, flux_out, counts_out, data, logl);
    return hipGetLastError();
}

}  // namespace ppm
