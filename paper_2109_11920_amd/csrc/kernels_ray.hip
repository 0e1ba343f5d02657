// Ray-driven kernels: one thread per ray, walking its samples along k, with the sampled image staged
// in LDS (whole image, or row bands for large n).
//
//   k_att     attenuation scan, Eq. (1) inner integral: m = W mu, L_k = dx (m_k/2 + sum_{k'>k} m_k'),
//             att = exp(-L), scanned from the detector end with a compensated running sum, stored
//             no smaller than the smallest normal float (the paired kernels take its reciprocal).
//   k_fwd     attenuated projection, Eq. (2): y = dx sum_k att (W f), compensated; epilogues give the
//             MLEM ratio S/y or the Poisson NLL terms of Eq. (5).
//   k_fwd_pair  the same for two candidates per workgroup, sharing each sample's geometry.
//   k_adj_sweep  one reverse MLEM step along every ray: the projection adjoint of the ratio and the
//             attenuation adjoint accumulation, in one sweep.
//   k_tail    sensitivity adjoint, att = exp(-L) and the scan's transpose (a prefix sum).
//
// Layout: att and its adjoint are per-angle slabs in 4 x 8 (sample x bin) blocks (att_row / att_col
// in device_common.h). The threads of a wave take consecutive bins of one angle, so at each k a
// wave's loads cover whole 32-byte block rows, and a ray's offset splits into a per-lane bin part and
// a uniform sample-row part.
#include "launch.h"

namespace boac {

// Map a flat workgroup id to (candidate, chunk) so that all chunks of one candidate run on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs); they share the candidate's image in L2.
__device__ __forceinline__ void ray_block(int bid, int chunks, int C, int &cand, int &chunk) {
    const int total = chunks * C;
    int id = bid;
    if ((total & 7) == 0) id = (id & 7) * (total >> 3) + (id >> 3);
    cand = id / chunks;
    chunk = id - cand * chunks;
}

constexpr int kMaxRpt = 4;
constexpr int kBandChunk = 16;  // samples per load batch in the row-band paths

// ------------------------------------------------------------------ attenuation
template <bool SINGLE>
__device__ __forceinline__ void k_att_body(int bid, float *lds, DevGeom g, const Bands &bands, int rpt, int chunks, int C,
                                             const float *__restrict__ mu, float *__restrict__ att, size_t img_cs,
                                             size_t att_cs, float *__restrict__ E, size_t e_cs) {
    int cand, chunk;
    ray_block(bid, chunks, C, cand, chunk);
    const int nrays = g.nah * g.nb;
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    const float *img = mu + cand * img_cs;
    float *out = att + cand * att_cs;

    for (int bi = 0; bi < bands.count; ++bi) {
        const Band band = bands.band(bi, g.n);
        __syncthreads();
        stage_band<1>(img, g.n, band, lds);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays) continue;
            const int a = ray / g.nb, b = ray - a * g.nb;
            const float2 cs = g.trig[a];
            float Ub, Vb;
            ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
            float *col = out + att_base(g, a, b);
            if constexpr (SINGLE) {
                // single pass from the detector end: running suffix sum T = sum_{k'>k} m_k'; the 4
                // samples of a group (k a multiple of 4) are one 16-byte store, padding rows get 0
                Comp T{0.f, 0.f};
                for (int kg = (g.nt - 1) >> 2; kg >= 0; --kg) {
                    float e[4];
#pragma unroll
                    for (int q = 3; q >= 0; --q) {
                        const int k = 4 * kg + q;
                        e[q] = 0.f;
                        if (k < g.nt) {
                            float U, V;
                            sample_uv(Ub, Vb, tau_of(g, k), cs.x, cs.y, U, V);
                            const Tap t = make_tap<true>(U, V, nf, pitch, band);
                            const float m = lerp2(lds + t.off, pitch, t.fu, t.fv);
                            const float L = g.dx * (fmaf(0.5f, m, T.s) + T.e);
                            e[q] = fmaxf(expf(-L), kMinNormal);
                            comp_add(T, m);
                        }
                    }
                    *reinterpret_cast<float4 *>(col + att_row(g, 4 * kg)) = make_float4(e[0], e[1], e[2], e[3]);
                }
                // opposed-ray pairing: exp(-T) of the whole ray, T = dx sum_k m_k
                if (E) E[cand * e_cs + ray] = expf(-g.dx * comp_value(T));
            } else {
                // pass 1 of 2: store m_k of the samples in this band, a 4-sample group (one 16-byte
                // load and store) at a time from the 4-aligned group holding the first. The ray is this
                // thread's alone and its bands run in order, so a group's samples owned by another band
                // are written back as loaded (values of an earlier band, or not yet written).
                int k0, k1;
                band_k_range(g, band, Vb, cs.x, k0, k1);
                const int kstart = (k0 <= k1) ? (k0 & ~3) : k1 + 1;
                for (int kg = kstart; kg <= k1; kg += 4) {
                    float4 *grp = reinterpret_cast<float4 *>(col + att_row(g, kg));
                    const float4 old = *grp;
                    float ov[4] = {old.x, old.y, old.z, old.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = kg + q;
                        if (k <= k1) {
                            float U, V;
                            sample_uv(Ub, Vb, tau_of(g, k), cs.x, cs.y, U, V);
                            const Tap t = make_tap<false>(U, V, nf, pitch, band);
                            if (t.mine) ov[q] = lerp2(lds + t.off, pitch, t.fu, t.fv);
                        }
                    }
                    *grp = make_float4(ov[0], ov[1], ov[2], ov[3]);
                }
            }
        }
    }
    if constexpr (!SINGLE) {
        // pass 2: scan the stored m_k (written by this same thread) from the detector end
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays) continue;
            const int a = ray / g.nb, b = ray - a * g.nb;
            // 16 samples (4 groups of 4, one 16-byte access each) at a time from the detector end:
            // the chunk's loads precede its stores; padding rows get 0
            constexpr int KG = kBandChunk / 4;
            const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(out, (unsigned)(4 * att_cs));
            const unsigned roff = 4u * (unsigned)att_base(g, a, b);
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            Comp T{0.f, 0.f};
            for (int kg0 = (g.nt - 1) >> 2; kg0 >= 0; kg0 -= KG) {
                float4 mv[KG];
#pragma unroll
                for (int j = 0; j < KG; ++j) {
                    const int kg = kg0 - j;
                    mv[j] = (kg >= 0) ? buffer_ld4(rs, roff + 4u * att_row(g, 4 * kg), 0u) : z4;
                }
#pragma unroll
                for (int j = 0; j < KG; ++j) {
                    const int kg = kg0 - j;
                    if (kg < 0) break;
                    float e[4];
#pragma unroll
                    for (int q = 3; q >= 0; --q) {
                        const int k = 4 * kg + q;
                        e[q] = 0.f;
                        if (k < g.nt) {
                            const float m = f4at(mv[j], q);
                            const float L = g.dx * (fmaf(0.5f, m, T.s) + T.e);
                            e[q] = fmaxf(expf(-L), kMinNormal);
                            comp_add(T, m);
                        }
                    }
                    buffer_st4(rs, roff + 4u * att_row(g, 4 * kg), 0u, make_float4(e[0], e[1], e[2], e[3]));
                }
            }
            if (E) E[cand * e_cs + ray] = expf(-g.dx * comp_value(T));  // opposed-ray pairing
        }
    }
}

#ifndef BOAC_BODIES_ONLY
template <bool SINGLE>
__global__ __launch_bounds__(1024) void k_att(DevGeom g, Bands bands, int rpt, int chunks, int C,
                                             const float *__restrict__ mu, float *__restrict__ att, size_t img_cs,
                                             size_t att_cs, float *__restrict__ E, size_t e_cs) {
    extern __shared__ float lds[];
    k_att_body<SINGLE>(blockIdx.x, lds, g, bands, rpt, chunks, C, mu, att, img_cs, att_cs, E, e_cs);
}
#endif

// Attenuation build with each ray's scan spread over kScanLanes lanes of one wave (single-stage images).
// The ray is walked from the detector end in rounds of kScanLanes 4-sample groups, lane j taking the
// j-th group of the round counted from the detector: each lane samples its 4 values m_k = (W mu)_k from
// the staged image and sums them (compensated); a Kogge-Stone scan over the 8 lanes (3 shuffle steps of
// compensated merges) gives each lane the sum of the groups nearer the detector in this round, to which
// the carry of the earlier rounds is merged; the lane then scans its own 4 samples toward the source,
// L_k = dx (m_k / 2 + sum_{k'>k} m_k'), and stores att = exp(-L) (no smaller than the smallest normal
// float) as one 16-byte store, and the round's total joins the carry. The 8 lanes of a ray and the 8
// rays of a wave (consecutive bins) write whole 128-byte lines of the 4 x 8-block layout. The carry
// ends as the ray total: exp(-T) for opposed-ray pairing. passes: rays per lane group handled in turn,
// so that one image stage serves many rays.
constexpr int kScanLanes = 8;

__device__ __forceinline__ void k_att_scan_body(int bid, float *lds, DevGeom g, Band band, int passes, int chunks, int C,
                                                  const float *__restrict__ mu, float *__restrict__ att,
                                                  size_t img_cs, size_t att_cs, float *__restrict__ E,
                                                  size_t e_cs) {
    int cand, chunk;
    ray_block(bid, chunks, C, cand, chunk);
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    stage_whole(mu + cand * img_cs, g.n, band, lds);
    __syncthreads();
    const int nrays = g.nah * g.nb;
    const int rpp = blockDim.x / kScanLanes;
    const int lane = threadIdx.x & (kScanLanes - 1);
    const int base = (threadIdx.x & (kWave - 1)) & ~(kScanLanes - 1);
    const int ng = (g.nt + 3) >> 2;
    const int rounds = (ng + kScanLanes - 1) / kScanLanes;
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(att + cand * att_cs, (unsigned)(4 * att_cs));
    for (int ps = 0; ps < passes; ++ps) {
        const int ray = (chunk * passes + ps) * rpp + (int)threadIdx.x / kScanLanes;
        const bool live = ray < nrays;
        const int a = live ? ray / g.nb : 0, b = live ? ray - a * g.nb : 0;
        const float2 cs = g.trig[a];
        float Ub, Vb;
        ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
        const unsigned roff = 4u * (unsigned)att_base(g, a, b);
        Comp carry{0.f, 0.f};
        for (int r = 0; r < rounds; ++r) {
            const int grp = ng - 1 - (r * kScanLanes + lane);
            float m[4];
            Comp own{0.f, 0.f};
#pragma unroll
            for (int q = 3; q >= 0; --q) {
                const int k = 4 * grp + q;
                m[q] = 0.f;
                if (live && grp >= 0 && k < g.nt) {
                    float U, V;
                    sample_uv(Ub, Vb, tau_of(g, k), cs.x, cs.y, U, V);
                    m[q] = bilinear_whole(lds, U, V, nf, pitch);
                    comp_add(own, m[q]);
                }
            }
            // inclusive scan over the lanes of the ray (lane 0 nearest the detector)
            Comp inc = own;
#pragma unroll
            for (int off = 1; off < kScanLanes; off <<= 1) {
                const Comp o{__shfl(inc.s, base + ((lane - off) & (kScanLanes - 1)), kWave),
                             __shfl(inc.e, base + ((lane - off) & (kScanLanes - 1)), kWave)};
                if (lane >= off) comp_merge(inc, o);
            }
            const Comp prev{__shfl(inc.s, base + ((lane - 1) & (kScanLanes - 1)), kWave),
                            __shfl(inc.e, base + ((lane - 1) & (kScanLanes - 1)), kWave)};
            const Comp total{__shfl(inc.s, base + kScanLanes - 1, kWave), __shfl(inc.e, base + kScanLanes - 1, kWave)};
            Comp T = carry;
            if (lane > 0) comp_merge(T, prev);
            if (live && grp >= 0) {
                float e[4];
#pragma unroll
                for (int q = 3; q >= 0; --q) {
                    const int k = 4 * grp + q;
                    e[q] = 0.f;
                    if (k < g.nt) {
                        const float L = g.dx * (fmaf(0.5f, m[q], T.s) + T.e);
                        e[q] = fmaxf(expf(-L), kMinNormal);
                        comp_add(T, m[q]);
                    }
                }
                buffer_st4_stream(rs, roff + 4u * att_row(g, 4 * grp), 0u, make_float4(e[0], e[1], e[2], e[3]));
            }
            comp_merge(carry, total);
        }
        if (E && live && lane == 0) E[cand * e_cs + ray] = expf(-g.dx * comp_value(carry));
    }
}

#ifndef BOAC_BODIES_ONLY
__global__ __launch_bounds__(1024) void k_att_scan(DevGeom g, Band band, int passes, int chunks, int C,
                                                  const float *__restrict__ mu, float *__restrict__ att,
                                                  size_t img_cs, size_t att_cs, float *__restrict__ E,
                                                  size_t e_cs) {
    extern __shared__ float lds[];
    k_att_scan_body(blockIdx.x, lds, g, band, passes, chunks, C, mu, att, img_cs, att_cs, E, e_cs);
}
#endif

// ------------------------------------------------------------------ forward projection
// The epilogue of one ray: y, or the MLEM ratio, or (returned) the NLL term; zero_proj is set where
// S > 0 meets y <= 0.
template <int MODE>
__device__ __forceinline__ float fwd_emit(const FwdArgs &A, size_t cand, int ray, float y, bool &zero_proj) {
    const size_t si = cand * A.sino_cs + ray;
    if constexpr (MODE == FWD_PROJ) {
        A.y_out[si] = y;
        return 0.f;
    } else if constexpr (MODE == FWD_RATIO) {
        const float S = A.meas[ray];
        A.r_out[si] = (y > 0.f) ? S / y : 0.f;
        if (A.y_out) A.y_out[si] = y;
        return 0.f;
    } else {  // FWD_NLL
        const float S = A.meas[ray];
        if (A.y_out) A.y_out[si] = y;
        float term;
        if (S > 0.f) {
            if (y > 0.f) {
                // y - S ln y less its measurement-only part S - S ln S (summed with ln Gamma(S + 1) in the
                // likelihood constant): y - S - S ln(y / S), with y - S exact where y is within a factor
                // of 2 of S
                const float d = y - S;
                term = d - S * log1pf(d / S);
            } else if (y <= 0.f) {
                term = __builtin_inff();
                zero_proj = true;
            } else {
                term = y;  // NaN propagates (flagged as non-finite at the end)
            }
        } else {
            term = y;
        }
        return term;
    }
}

// 1 / att for the opposed ray's attenuation exp(-T) / att; att is clamped to the smallest normal
// float (exact for path lengths below ~87 optical depths).
__device__ __forceinline__ float inv_att(float at) { return rcp_clamped(at); }
__device__ __forceinline__ float opposed_att(float e_ray, float at) { return e_ray * inv_att(at); }

// PAIRED (opposed-ray pairing, single stage only): each thread's ray (a, b), a < na/2, also gives the
// projection of ray (a + na/2, nb-1-b) from the same samples and bilinear values.
template <int MODE, bool SINGLE, bool PAIRED>
__device__ __forceinline__ void k_fwd_body(int bid, float *lds, float *red, DevGeom g, const Bands &bands, int rpt, int chunks, int C, FwdArgs A) {
    int cand, chunk;
    ray_block(bid, chunks, C, cand, chunk);
    const int nrays = g.nah * g.nb;
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    const float *att = A.att + cand * A.att_cs;
    const float *img = A.img + cand * A.img_cs;

    Comp acc[kMaxRpt], acc2[PAIRED ? kMaxRpt : 1];
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) acc[j] = Comp{0.f, 0.f};
#pragma unroll
    for (int j = 0; j < (PAIRED ? kMaxRpt : 1); ++j) acc2[j] = Comp{0.f, 0.f};

    for (int bi = 0; bi < bands.count; ++bi) {
        const Band band = bands.band(bi, g.n);
        __syncthreads();
        if (A.img_comps == 1)
            stage_band<1>(img, g.n, band, lds);
        else
            stage_band_strided(img, g.n, A.img_comps, band, lds);  // component 0 of an interleaved pair
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays) continue;
            const int a = ray / g.nb, b = ray - a * g.nb;
            const float2 cs = g.trig[a];
            float Ub, Vb;
            ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
            Comp c = acc[j];
            if constexpr (SINGLE) {
                // att is streamed 16 samples ahead of use: the loads of chunk k0 + 16 are in flight
                // while chunk k0 is computed. The loads go through a buffer resource: a per-lane ray
                // offset plus a uniform offset of the sample row. Each chunk is summed with FMAs and
                // added to the compensated total.
                // Each 16-byte load brings 4 consecutive samples of the ray (one group of the layout).
                constexpr int KC = 16, KG = KC / 4;
                const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
                const unsigned roff = 4u * (unsigned)att_base(g, a, b);
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                const float e_ray = PAIRED ? A.E[cand * A.e_cs + ray] : 0.f;
                Comp c2 = PAIRED ? acc2[j] : Comp{0.f, 0.f};
                float4 cur[KG], nxt[KG];
#pragma unroll
                for (int q = 0; q < KG; ++q) cur[q] = (4 * q < g.nt) ? buffer_ld4_stream(rs, roff, 4u * att_row(g, 4 * q)) : z4;
                float tau = -g.cT;
                for (int k0 = 0; k0 < g.nt; k0 += KC) {
#pragma unroll
                    for (int q = 0; q < KG; ++q) {
                        const int k = k0 + KC + 4 * q;
                        nxt[q] = (k < g.nt) ? buffer_ld4_stream(rs, roff, 4u * att_row(g, k)) : z4;
                    }
                    float part = 0.f, part2 = 0.f;
#pragma unroll
                    for (int q = 0; q < KC; ++q) {
                        if (k0 + q < g.nt) {
                            float U, V;
                            sample_uv(Ub, Vb, tau, cs.x, cs.y, U, V);
                            const float at = f4at(cur[q >> 2], q & 3);
                            const float w = bilinear_whole(lds, U, V, nf, pitch);
                            part = fmaf(at, w, part);
                            if constexpr (PAIRED) part2 = fmaf(opposed_att(e_ray, at), w, part2);
                        }
                        tau += 1.f;
                    }
                    kahan_add(c, part);
                    if constexpr (PAIRED) kahan_add(c2, part2);
#pragma unroll
                    for (int q = 0; q < KG; ++q) cur[q] = nxt[q];
                }
                if constexpr (PAIRED) acc2[j] = c2;
            } else {
                // the ray's samples in this band, 16 at a time from the 4-aligned group holding the
                // first: the chunk's att loads (4 samples per 16-byte load) are issued together, then
                // used; samples before the range are not the band's and fail the ownership test
                int k0 = 0, k1 = g.nt - 1;
                band_k_range(g, band, Vb, cs.x, k0, k1);
                const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
                const unsigned roff = 4u * (unsigned)att_base(g, a, b);
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                const int kstart = (k0 <= k1) ? (k0 & ~3) : k1 + 1;
                const float e_ray = PAIRED ? A.E[cand * A.e_cs + ray] : 0.f;
                Comp c2 = PAIRED ? acc2[j] : Comp{0.f, 0.f};
                for (int kc = kstart; kc <= k1; kc += kBandChunk) {
                    float4 av[kBandChunk / 4];
#pragma unroll
                    for (int q = 0; q < kBandChunk / 4; ++q) {
                        const int k = kc + 4 * q;
                        av[q] = (k <= k1) ? buffer_ld4(rs, roff + 4u * att_row(g, k), 0u) : z4;
                    }
                    float part = 0.f, part2 = 0.f;
#pragma unroll
                    for (int q = 0; q < kBandChunk; ++q) {
                        const int k = kc + q;
                        if (k <= k1) {  // a guard, not a break: the loop stays unrolled and av in registers
                            float U, V;
                            sample_uv(Ub, Vb, tau_of(g, k), cs.x, cs.y, U, V);
                            const Tap t = make_tap<false>(U, V, nf, pitch, band);
                            if (t.mine) {
                                const float at = f4at(av[q >> 2], q & 3);
                                const float w = lerp2(lds + t.off, pitch, t.fu, t.fv);
                                part = fmaf(at, w, part);
                                if constexpr (PAIRED) part2 = fmaf(opposed_att(e_ray, at), w, part2);
                            }
                        }
                    }
                    kahan_add(c, part);
                    if constexpr (PAIRED) kahan_add(c2, part2);
                }
                if constexpr (PAIRED) acc2[j] = c2;
            }
            acc[j] = c;
        }
    }

    // epilogues
    Comp nll{0.f, 0.f};
    bool zero_proj = false;
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) {
        if (j >= rpt) break;
        const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
        if (ray >= nrays) continue;
        const float t0 = fwd_emit<MODE>(A, cand, ray, g.dx * comp_value(acc[j]), zero_proj);
        if constexpr (MODE == FWD_NLL) comp_add(nll, t0);
        if constexpr (PAIRED) {
            const int a = ray / g.nb, b = ray - a * g.nb;
            const float t1 =
                fwd_emit<MODE>(A, cand, (a + g.nah) * g.nb + (g.nb - 1 - b), g.dx * comp_value(acc2[j]), zero_proj);
            if constexpr (MODE == FWD_NLL) comp_add(nll, t1);
        }
    }
    if constexpr (MODE == FWD_NLL) {
        if (zero_proj && A.status) atomicOr(A.status + cand, 1u);
        const Comp r = block_reduce(nll, red);
        if (threadIdx.x == 0) A.partial[(size_t)cand * chunks + chunk] = make_float2(r.s, r.e);
    }
}

#ifndef BOAC_BODIES_ONLY
template <int MODE, bool SINGLE, bool PAIRED>
__global__ __launch_bounds__(1024) void k_fwd(DevGeom g, Bands bands, int rpt, int chunks, int C, FwdArgs A) {
    extern __shared__ float lds[];
    __shared__ float red[32];  // two floats per wave, up to 16 waves
    k_fwd_body<MODE, SINGLE, PAIRED>(blockIdx.x, lds, red, g, bands, rpt, chunks, C, A);
}
#endif

// Forward projection of two candidates per workgroup, both images staged at once (interleaved as
// float2): each sample's position, clamp, tap index and bilinear fractions are computed once and
// serve both candidates (one pair lerp, two FMAs), about half the vector work per candidate-sample of
// k_fwd. Single-stage images only (the pair stage is twice the size). An odd batch's last pair
// repeats its candidate and writes it once. PAIRED: opposed-ray pairing as in k_fwd.
template <int MODE, bool PAIRED>
__device__ __forceinline__ void k_fwd_pair_body(int bid, float *lds, float *red, DevGeom g, const Bands &bands, int rpt, int chunks, int C, FwdArgs A) {
    const int npairs = (C + 1) >> 1;
    int pr, chunk;
    ray_block(bid, chunks, npairs, pr, chunk);
    const int c0 = 2 * pr;
    const bool two = (c0 + 1 < C);
    const int c1 = two ? c0 + 1 : c0;
    const int nrays = g.nah * g.nb;
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    stage_band_pair(A.img + c0 * A.img_cs, A.img + c1 * A.img_cs, g.n, bands.band(0, g.n), lds);
    __syncthreads();
    const float2 *lds2 = reinterpret_cast<const float2 *>(lds);
    const __amdgpu_buffer_rsrc_t r0 = buffer_rsrc(A.att + c0 * A.att_cs, (unsigned)(4 * A.att_cs));
    const __amdgpu_buffer_rsrc_t r1 = buffer_rsrc(A.att + c1 * A.att_cs, (unsigned)(4 * A.att_cs));

    Comp acc0[kMaxRpt], acc1[kMaxRpt], opp0[kMaxRpt], opp1[kMaxRpt];
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) acc0[j] = acc1[j] = opp0[j] = opp1[j] = Comp{0.f, 0.f};
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) {
        if (j >= rpt) break;
        const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
        if (ray >= nrays) continue;
        const int a = ray / g.nb, b = ray - a * g.nb;
        const float2 cs = g.trig[a];
        float Ub, Vb;
        ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
        const unsigned roff = 4u * (unsigned)att_base(g, a, b);
        const float e0 = PAIRED ? A.E[c0 * A.e_cs + ray] : 0.f;
        const float e1 = PAIRED ? A.E[c1 * A.e_cs + ray] : 0.f;
        constexpr int KC = 16, KG = KC / 4;
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 u0[KG], u1[KG], n0[KG], n1[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q) {
            u0[q] = (4 * q < g.nt) ? buffer_ld4_stream(r0, roff, 4u * att_row(g, 4 * q)) : z4;
            u1[q] = (4 * q < g.nt) ? buffer_ld4_stream(r1, roff, 4u * att_row(g, 4 * q)) : z4;
        }
        Comp s0 = acc0[j], s1 = acc1[j], t0 = opp0[j], t1 = opp1[j];
        float tau = -g.cT;
        for (int k0 = 0; k0 < g.nt; k0 += KC) {
#pragma unroll
            for (int q = 0; q < KG; ++q) {
                const int k = k0 + KC + 4 * q;
                n0[q] = (k < g.nt) ? buffer_ld4_stream(r0, roff, 4u * att_row(g, k)) : z4;
                n1[q] = (k < g.nt) ? buffer_ld4_stream(r1, roff, 4u * att_row(g, k)) : z4;
            }
            float p0 = 0.f, p1 = 0.f, o0 = 0.f, o1 = 0.f;
#pragma unroll
            for (int q = 0; q < KC; ++q) {
                if (k0 + q < g.nt) {
                    float U, V;
                    sample_uv(Ub, Vb, tau, cs.x, cs.y, U, V);
                    const float Uc = __builtin_amdgcn_fmed3f(U, -1.f, nf);
                    const float Vc = __builtin_amdgcn_fmed3f(V, -1.f, nf);
                    const int idx = (int)fmaf(floorf(Vc), (float)pitch, floorf(Uc));
                    const float2 w = lerp2x2(lds2 + idx + (pitch + 1), pitch, __builtin_amdgcn_fractf(Uc),
                                             __builtin_amdgcn_fractf(Vc));
                    const float a0 = f4at(u0[q >> 2], q & 3), a1 = f4at(u1[q >> 2], q & 3);
                    p0 = fmaf(a0, w.x, p0);
                    p1 = fmaf(a1, w.y, p1);
                    if constexpr (PAIRED) {
                        o0 = fmaf(opposed_att(e0, a0), w.x, o0);
                        o1 = fmaf(opposed_att(e1, a1), w.y, o1);
                    }
                }
                tau += 1.f;
            }
            kahan_add(s0, p0);
            kahan_add(s1, p1);
            if constexpr (PAIRED) {
                kahan_add(t0, o0);
                kahan_add(t1, o1);
            }
#pragma unroll
            for (int q = 0; q < KG; ++q) {
                u0[q] = n0[q];
                u1[q] = n1[q];
            }
        }
        acc0[j] = s0;
        acc1[j] = s1;
        opp0[j] = t0;
        opp1[j] = t1;
    }

    // epilogues, candidate by candidate
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int cand = h ? c1 : c0;
        const bool live = (h == 0) || two;
        Comp nll{0.f, 0.f};
        bool zero_proj = false;
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays || !live) continue;
            const float t0 = fwd_emit<MODE>(A, cand, ray, g.dx * comp_value(h ? acc1[j] : acc0[j]), zero_proj);
            if constexpr (MODE == FWD_NLL) comp_add(nll, t0);
            if constexpr (PAIRED) {
                const int a = ray / g.nb, b = ray - a * g.nb;
                const float t1 = fwd_emit<MODE>(A, cand, (a + g.nah) * g.nb + (g.nb - 1 - b),
                                                g.dx * comp_value(h ? opp1[j] : opp0[j]), zero_proj);
                if constexpr (MODE == FWD_NLL) comp_add(nll, t1);
            }
        }
        if constexpr (MODE == FWD_NLL) {
            if (zero_proj && A.status) atomicOr(A.status + cand, 1u);
            const Comp r = block_reduce(nll, red);
            if (threadIdx.x == 0 && live) A.partial[(size_t)cand * chunks + chunk] = make_float2(r.s, r.e);
        }
    }
}

#ifndef BOAC_BODIES_ONLY
template <int MODE, bool PAIRED>
__global__ __launch_bounds__(1024) void k_fwd_pair(DevGeom g, Bands bands, int rpt, int chunks, int C, FwdArgs A) {
    extern __shared__ float lds[];
    __shared__ float red[32];  // two floats per wave, up to 16 waves
    k_fwd_pair_body<MODE, PAIRED>(blockIdx.x, lds, red, g, bands, rpt, chunks, C, A);
}
#endif

// ------------------------------------------------------------------ fused reverse sweep
// One reverse MLEM step n, per ray i (pair image = (bbar^n, F^{n+1}) staged in LDS):
//   rbar_i   = dx sum_k att_ik (W bbar^n)_ik                          (adjoint of b^n = A^T r^n)
//   attbar_ik (+)= dx [ r^n_i (W bbar^n)_ik + ybar^{n+1}_i (W F^{n+1})_ik ]
//   ybar^n_i = -rbar_i r^n_i / y^n_i   (0 where y^n_i <= 0)               (adjoint of r = S / y)
// The ybar^{n+1} term is the y^{n+1} = A F^{n+1} adjoint left pending by the previous step (or the
// objective's adjoint for the first step), so each step sweeps the rays once.
// PAIRED (opposed-ray pairing, single stage): the held ray i also carries the opposed ray i', whose
// attenuation at the shared sample is att' = exp(-T) / att; its r_bar and ybar are formed the same
// way, and its attenuation adjoint c' = dx [ r^n_i' W bbar + ybar^{n+1}_i' W F^{n+1} ] reaches the
// held tensors through att' = E / att: att_bar += -att' c' / att, E_bar += c' / att.
template <bool SINGLE, bool PAIRED>
__device__ __forceinline__ void k_adj_sweep_body(int bid, float *lds, DevGeom g, const Bands &bands, int rpt, int chunks, int C, SweepArgs A) {
    int cand, chunk;
    ray_block(bid, chunks, C, cand, chunk);
    const int nrays = g.nah * g.nb;
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    const float *att = A.att + cand * A.att_cs;
    float *ab = A.attbar + cand * A.att_cs;
    const float *img = A.pair + cand * A.img_cs;
    const float2 *lds2 = reinterpret_cast<const float2 *>(lds);

    Comp acc[kMaxRpt], acc2[kMaxRpt], ebj[kMaxRpt];  // PAIRED: r_bar of the opposed ray, its E_bar part
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) acc[j] = acc2[j] = ebj[j] = Comp{0.f, 0.f};

    for (int bi = 0; bi < bands.count; ++bi) {
        const Band band = bands.band(bi, g.n);
        __syncthreads();
        stage_band<2>(img, g.n, band, lds);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays) continue;
            const int a = ray / g.nb, b = ray - a * g.nb;
            const float2 cs = g.trig[a];
            float Ub, Vb;
            ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
            const size_t si = cand * A.sino_cs + ray;
            const float rr = g.dx * A.r[si];
            const float yp = g.dx * A.ybar_in[si];
            const size_t col0 = att_base(g, a, b);
            Comp c = acc[j];
            if constexpr (SINGLE) {
                // as in the forward projection: att and att_bar streamed 16 samples ahead through
                // buffer resources (per-lane ray offset + uniform sample-row offset), chunked
                // compensated sum, tap index formed in float
                // samples move in groups of 4 (one 16-byte load or store); padding rows get 0
                constexpr int KC = 16, KG = KC / 4;
                const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
                const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(ab, (unsigned)(4 * A.att_cs));
                const unsigned roff = 4u * (unsigned)col0;
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                float4 at[KG], an[KG], bt[KG], bn[KG];
#pragma unroll
                for (int q = 0; q < KG; ++q) {
                    const unsigned o = 4u * att_row(g, 4 * q);
                    at[q] = (4 * q < g.nt) ? buffer_ld4_stream(ra, roff, o) : z4;
                    bt[q] = (A.accumulate && 4 * q < g.nt) ? buffer_ld4_stream(rb, roff, o) : z4;
                }
                const size_t si2 = cand * A.sino_cs + (size_t)((a + g.nah) * g.nb + (g.nb - 1 - b));
                const float e_ray = PAIRED ? A.E[cand * A.e_cs + ray] : 0.f;
                const float rr2 = PAIRED ? g.dx * A.r[si2] : 0.f;
                const float yp2 = PAIRED ? g.dx * A.ybar_in[si2] : 0.f;
                Comp c2 = acc2[j], eb = ebj[j];
                float tau = -g.cT;
                for (int k0 = 0; k0 < g.nt; k0 += KC) {
#pragma unroll
                    for (int q = 0; q < KG; ++q) {
                        const int k = k0 + KC + 4 * q;
                        const unsigned o = 4u * att_row(g, k);
                        an[q] = (k < g.nt) ? buffer_ld4_stream(ra, roff, o) : z4;
                        bn[q] = (A.accumulate && k < g.nt) ? buffer_ld4_stream(rb, roff, o) : z4;
                    }
                    float part = 0.f, part2 = 0.f, epart = 0.f;
                    float ov[4];
#pragma unroll
                    for (int q = 0; q < KC; ++q) {
                        const int k = k0 + q;
                        ov[q & 3] = 0.f;
                        if (k < g.nt) {
                            float U, V;
                            sample_uv(Ub, Vb, tau, cs.x, cs.y, U, V);
                            const float Uc = __builtin_amdgcn_fmed3f(U, -1.f, nf);
                            const float Vc = __builtin_amdgcn_fmed3f(V, -1.f, nf);
                            const int idx = (int)fmaf(floorf(Vc), (float)pitch, floorf(Uc));
                            const float2 w = lerp2x2(lds2 + idx + (pitch + 1), pitch, __builtin_amdgcn_fractf(Uc),
                                                     __builtin_amdgcn_fractf(Vc));
                            const float a0 = f4at(at[q >> 2], q & 3);
                            part = fmaf(a0, w.x, part);
                            const float cv = fmaf(rr, w.x, yp * w.y);
                            if constexpr (PAIRED) {
                                const float ri = inv_att(a0);
                                const float ao = e_ray * ri;
                                const float cv2 = fmaf(rr2, w.x, yp2 * w.y);
                                part2 = fmaf(ao, w.x, part2);
                                epart = fmaf(cv2, ri, epart);
                                ov[q & 3] = f4at(bt[q >> 2], q & 3) + fmaf(-ao * ri, cv2, cv);
                            } else {
                                ov[q & 3] = f4at(bt[q >> 2], q & 3) + cv;
                            }
                        }
                        tau += 1.f;
                        if ((q & 3) == 3 && k - 3 < g.nt)
                            buffer_st4_stream(rb, roff, 4u * att_row(g, k - 3), make_float4(ov[0], ov[1], ov[2], ov[3]));
                    }
                    kahan_add(c, part);
                    if constexpr (PAIRED) {
                        kahan_add(c2, part2);
                        kahan_add(eb, epart);
                    }
#pragma unroll
                    for (int q = 0; q < KG; ++q) {
                        at[q] = an[q];
                        bt[q] = bn[q];
                    }
                }
                if constexpr (PAIRED) {
                    acc2[j] = c2;
                    ebj[j] = eb;
                }
            } else {
                // the ray's samples in this band, 16 at a time (loads of att, and of att_bar when
                // accumulating, issued together per chunk)
                // from the 4-aligned group holding the first sample, 16-byte loads and stores; samples
                // before the range fail the ownership test. The ray is this thread's alone and its bands
                // run in order, so a group's samples owned by another band are written back as loaded.
                int k0, k1;
                band_k_range(g, band, Vb, cs.x, k0, k1);
                const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
                const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(ab, (unsigned)(4 * A.att_cs));
                const unsigned roff = 4u * (unsigned)col0;
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                const int kstart = (k0 <= k1) ? (k0 & ~3) : k1 + 1;
                const size_t si2 = cand * A.sino_cs + (size_t)((a + g.nah) * g.nb + (g.nb - 1 - b));
                const float e_ray = PAIRED ? A.E[cand * A.e_cs + ray] : 0.f;
                const float rr2 = PAIRED ? g.dx * A.r[si2] : 0.f;
                const float yp2 = PAIRED ? g.dx * A.ybar_in[si2] : 0.f;
                Comp c2 = acc2[j], eb = ebj[j];
                for (int kc = kstart; kc <= k1; kc += kBandChunk) {
                    float4 av[kBandChunk / 4], bv[kBandChunk / 4];
#pragma unroll
                    for (int q = 0; q < kBandChunk / 4; ++q) {
                        const int k = kc + 4 * q;
                        const unsigned o = roff + 4u * att_row(g, k);
                        av[q] = (k <= k1) ? buffer_ld4(ra, o, 0u) : z4;
                        bv[q] = (k <= k1) ? buffer_ld4(rb, o, 0u) : z4;
                    }
                    float part = 0.f, part2 = 0.f, epart = 0.f;
                    float ov[4];
#pragma unroll
                    for (int q = 0; q < kBandChunk; ++q) {
                        const int k = kc + q;
                        ov[q & 3] = f4at(bv[q >> 2], q & 3);
                        if (k <= k1) {
                            float U, V;
                            sample_uv(Ub, Vb, tau_of(g, k), cs.x, cs.y, U, V);
                            const Tap t = make_tap<false>(U, V, nf, pitch, band);
                            if (t.mine) {
                                const float2 w = lerp2x2(lds2 + t.off, pitch, t.fu, t.fv);
                                const float a0 = f4at(av[q >> 2], q & 3);
                                part = fmaf(a0, w.x, part);
                                const float cv = fmaf(rr, w.x, yp * w.y);
                                const float base = A.accumulate ? ov[q & 3] : 0.f;
                                if constexpr (PAIRED) {
                                    const float ri = inv_att(a0);
                                    const float ao = e_ray * ri;
                                    const float cv2 = fmaf(rr2, w.x, yp2 * w.y);
                                    part2 = fmaf(ao, w.x, part2);
                                    epart = fmaf(cv2, ri, epart);
                                    ov[q & 3] = base + fmaf(-ao * ri, cv2, cv);
                                } else {
                                    ov[q & 3] = base + cv;
                                }
                            }
                        }
                        if ((q & 3) == 3 && k - 3 <= k1)
                            buffer_st4(rb, roff + 4u * att_row(g, k - 3), 0u, make_float4(ov[0], ov[1], ov[2], ov[3]));
                    }
                    kahan_add(c, part);
                    if constexpr (PAIRED) {
                        kahan_add(c2, part2);
                        kahan_add(eb, epart);
                    }
                }
                if constexpr (PAIRED) {
                    acc2[j] = c2;
                    ebj[j] = eb;
                }
            }
            acc[j] = c;
        }
    }
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) {
        if (j >= rpt) break;
        const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
        if (ray >= nrays) continue;
        const size_t si = cand * A.sino_cs + ray;
        const float rbar = g.dx * comp_value(acc[j]);
        const float yn = A.y[si];
        A.ybar_out[si] = (yn > 0.f) ? -(rbar * A.r[si]) / yn : 0.f;
        if constexpr (PAIRED) {
            const int a = ray / g.nb, b = ray - a * g.nb;
            const size_t si2 = cand * A.sino_cs + (size_t)((a + g.nah) * g.nb + (g.nb - 1 - b));
            const float rbar2 = g.dx * comp_value(acc2[j]);
            const float yn2 = A.y[si2];
            A.ybar_out[si2] = (yn2 > 0.f) ? -(rbar2 * A.r[si2]) / yn2 : 0.f;
            float *eo = A.Ebar + cand * A.e_cs + ray;
            *eo = (A.accumulate ? *eo : 0.f) + comp_value(ebj[j]);
        }
    }
}

#ifndef BOAC_BODIES_ONLY
template <bool SINGLE, bool PAIRED>
__global__ __launch_bounds__(1024) void k_adj_sweep(DevGeom g, Bands bands, int rpt, int chunks, int C, SweepArgs A) {
    extern __shared__ float lds[];
    k_adj_sweep_body<SINGLE, PAIRED>(blockIdx.x, lds, g, bands, rpt, chunks, C, A);
}
#endif

// ------------------------------------------------------------------ tail of the attenuation adjoint
// att_bar (+)= dx (W G1 + rho_i W G2) with the pair image (G1, G2) = (s_bar, F^0) and rho = ybar^0
// (the sensitivity adjoint and the last pending projection adjoint); then
// L_bar = -att * att_bar and m_bar_k = dx (L_bar_k / 2 + sum_{k'<k} L_bar_k') (the scan's transpose),
// written in place of att_bar.
// PAIRED (opposed-ray pairing, single stage): the opposed ray's part c' = dx (W G1 + rho_i' W G2)
// reaches att_bar and E_bar as in the sweep; at the ray's end Tbar = -E E_bar (E = exp(-T)), and
// since T = dx sum_k m_k every sample's m_bar gains dx Tbar, written per ray in place of E_bar (the
// field gather adds it).
template <bool SINGLE, bool PAIRED>
__device__ __forceinline__ void k_tail_body(int bid, float *lds, DevGeom g, const Bands &bands, int rpt, int chunks, int C, TailArgs A) {
    int cand, chunk;
    ray_block(bid, chunks, C, cand, chunk);
    const int nrays = g.nah * g.nb;
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    const float *att = A.att + cand * A.att_cs;
    float *ab = A.attbar + cand * A.att_cs;
    const float *img = A.pair + cand * A.img_cs;
    const float2 *lds2 = reinterpret_cast<const float2 *>(lds);
    Comp ebj[kMaxRpt];  // PAIRED, row bands: the opposed ray's E_bar part, summed over the bands
#pragma unroll
    for (int j = 0; j < kMaxRpt; ++j) ebj[j] = Comp{0.f, 0.f};

    for (int bi = 0; bi < bands.count; ++bi) {
        const Band band = bands.band(bi, g.n);
        __syncthreads();
        stage_band<2>(img, g.n, band, lds);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays) continue;
            const int a = ray / g.nb, b = ray - a * g.nb;
            const float2 cs = g.trig[a];
            float Ub, Vb;
            ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
            const float rho = A.rho[cand * A.sino_cs + ray];
            const size_t off = att_base(g, a, b);
            if constexpr (SINGLE) {
                // samples move in groups of 4 (one 16-byte load or store); padding rows get 0
                constexpr int KC = 16, KG = KC / 4;
                const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
                const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(ab, (unsigned)(4 * A.att_cs));
                const unsigned roff = 4u * (unsigned)off;
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                float4 at[KG], an[KG], bt[KG], bn[KG];
#pragma unroll
                for (int q = 0; q < KG; ++q) {
                    const unsigned o = 4u * att_row(g, 4 * q);
                    at[q] = (4 * q < g.nt) ? buffer_ld4_stream(ra, roff, o) : z4;
                    bt[q] = (A.accumulate && 4 * q < g.nt) ? buffer_ld4_stream(rb, roff, o) : z4;
                }
                Comp P{0.f, 0.f};
                const float e_ray = PAIRED ? A.E[cand * A.e_cs + ray] : 0.f;
                const float rho2 =
                    PAIRED ? A.rho[cand * A.sino_cs + (size_t)((a + g.nah) * g.nb + (g.nb - 1 - b))] : 0.f;
                Comp eb{0.f, 0.f};
                float tau = -g.cT;
                for (int k0 = 0; k0 < g.nt; k0 += KC) {
#pragma unroll
                    for (int q = 0; q < KG; ++q) {
                        const int k = k0 + KC + 4 * q;
                        const unsigned o = 4u * att_row(g, k);
                        an[q] = (k < g.nt) ? buffer_ld4_stream(ra, roff, o) : z4;
                        bn[q] = (A.accumulate && k < g.nt) ? buffer_ld4_stream(rb, roff, o) : z4;
                    }
                    float ov[4];
                    float epart = 0.f;
#pragma unroll
                    for (int q = 0; q < KC; ++q) {
                        const int k = k0 + q;
                        ov[q & 3] = 0.f;
                        if (k < g.nt) {
                            float U, V;
                            sample_uv(Ub, Vb, tau, cs.x, cs.y, U, V);
                            const float Uc = __builtin_amdgcn_fmed3f(U, -1.f, nf);
                            const float Vc = __builtin_amdgcn_fmed3f(V, -1.f, nf);
                            const int l0 = __float2int_rd(Uc), i0 = __float2int_rd(Vc);
                            const float2 w = lerp2x2(lds2 + (i0 + 1) * pitch + (l0 + 1), pitch,
                                                     __builtin_amdgcn_fractf(Uc), __builtin_amdgcn_fractf(Vc));
                            const float a0 = f4at(at[q >> 2], q & 3);
                            float abar;
                            if constexpr (PAIRED) {
                                const float ri = inv_att(a0);
                                const float ao = e_ray * ri;
                                const float cv2 = g.dx * fmaf(rho2, w.y, w.x);
                                epart = fmaf(cv2, ri, epart);
                                abar = f4at(bt[q >> 2], q & 3) + fmaf(-ao * ri, cv2, g.dx * fmaf(rho, w.y, w.x));
                            } else {
                                abar = f4at(bt[q >> 2], q & 3) + g.dx * fmaf(rho, w.y, w.x);
                            }
                            const float Lbar = -a0 * abar;
                            ov[q & 3] = g.dx * (fmaf(0.5f, Lbar, P.s) + P.e);
                            comp_add(P, Lbar);
                        }
                        tau += 1.f;
                        if ((q & 3) == 3 && k - 3 < g.nt)
                            buffer_st4_stream(rb, roff, 4u * att_row(g, k - 3), make_float4(ov[0], ov[1], ov[2], ov[3]));
                    }
                    if constexpr (PAIRED) kahan_add(eb, epart);
#pragma unroll
                    for (int q = 0; q < KG; ++q) {
                        at[q] = an[q];
                        bt[q] = bn[q];
                    }
                }
                if constexpr (PAIRED) {
                    float *eo = A.Ebar + cand * A.e_cs + ray;
                    const float etot = (A.accumulate ? *eo : 0.f) + comp_value(eb);
                    *eo = g.dx * (-e_ray * etot);
                }
            } else {
                // pass 1 of 2 (band by band): att_bar (+)= dx (W G1 + rho W G2), 16 samples at a time
                // (from the 4-aligned group holding the first sample, 16-byte loads and stores; samples of
                // another band are written back as loaded, as in the sweep)
                int k0, k1;
                band_k_range(g, band, Vb, cs.x, k0, k1);
                const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
                const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(ab, (unsigned)(4 * A.att_cs));
                const unsigned roff = 4u * (unsigned)att_base(g, a, b);
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                const int kstart = (k0 <= k1) ? (k0 & ~3) : k1 + 1;
                const float e_ray = PAIRED ? A.E[cand * A.e_cs + ray] : 0.f;
                const float rho2 =
                    PAIRED ? A.rho[cand * A.sino_cs + (size_t)((a + g.nah) * g.nb + (g.nb - 1 - b))] : 0.f;
                Comp eb = ebj[j];
                for (int kc = kstart; kc <= k1; kc += kBandChunk) {
                    float4 av[kBandChunk / 4], bv[kBandChunk / 4];
#pragma unroll
                    for (int q = 0; q < kBandChunk / 4; ++q) {
                        const int k = kc + 4 * q;
                        const unsigned o = roff + 4u * att_row(g, k);
                        bv[q] = (k <= k1) ? buffer_ld4(rb, o, 0u) : z4;
                        av[q] = (PAIRED && k <= k1) ? buffer_ld4(ra, o, 0u) : z4;
                    }
                    float ov[4];
                    float epart = 0.f;
#pragma unroll
                    for (int q = 0; q < kBandChunk; ++q) {
                        const int k = kc + q;
                        ov[q & 3] = f4at(bv[q >> 2], q & 3);
                        if (k <= k1) {
                            float U, V;
                            sample_uv(Ub, Vb, tau_of(g, k), cs.x, cs.y, U, V);
                            const Tap t = make_tap<false>(U, V, nf, pitch, band);
                            if (t.mine) {
                                const float2 w = lerp2x2(lds2 + t.off, pitch, t.fu, t.fv);
                                const float base = A.accumulate ? ov[q & 3] : 0.f;
                                const float cv = g.dx * fmaf(rho, w.y, w.x);
                                if constexpr (PAIRED) {
                                    const float ri = inv_att(f4at(av[q >> 2], q & 3));
                                    const float ao = e_ray * ri;
                                    const float cv2 = g.dx * fmaf(rho2, w.y, w.x);
                                    epart = fmaf(cv2, ri, epart);
                                    ov[q & 3] = base + fmaf(-ao * ri, cv2, cv);
                                } else {
                                    ov[q & 3] = base + cv;
                                }
                            }
                        }
                        if ((q & 3) == 3 && k - 3 <= k1)
                            buffer_st4(rb, roff + 4u * att_row(g, k - 3), 0u, make_float4(ov[0], ov[1], ov[2], ov[3]));
                    }
                    if constexpr (PAIRED) kahan_add(eb, epart);
                }
                if constexpr (PAIRED) ebj[j] = eb;
            }
        }
    }
    if constexpr (!SINGLE) {
        // pass 2: every sample of the ray now holds att_bar (written by this thread): scan
#pragma unroll
        for (int j = 0; j < kMaxRpt; ++j) {
            if (j >= rpt) break;
            const int ray = (chunk * rpt + j) * blockDim.x + threadIdx.x;
            if (ray >= nrays) continue;
            const int a = ray / g.nb, b = ray - a * g.nb;
            // 16 samples (4 groups, one 16-byte access each) at a time: the chunk's loads are issued
            // before any of its stores; padding rows get 0
            const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(att, (unsigned)(4 * A.att_cs));
            const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(ab, (unsigned)(4 * A.att_cs));
            const unsigned roff = 4u * (unsigned)att_base(g, a, b);
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            Comp P{0.f, 0.f};
            for (int kc = 0; kc < g.nt; kc += kBandChunk) {
                float4 av[kBandChunk / 4], bv[kBandChunk / 4];
#pragma unroll
                for (int q = 0; q < kBandChunk / 4; ++q) {
                    const int k = kc + 4 * q;
                    const unsigned o = roff + 4u * att_row(g, k);
                    av[q] = (k < g.nt) ? buffer_ld4(ra, o, 0u) : z4;
                    bv[q] = (k < g.nt) ? buffer_ld4(rb, o, 0u) : z4;
                }
                float ov[4];
#pragma unroll
                for (int q = 0; q < kBandChunk; ++q) {
                    const int k = kc + q;
                    ov[q & 3] = 0.f;
                    if (k < g.nt) {
                        const float Lbar = -f4at(av[q >> 2], q & 3) * f4at(bv[q >> 2], q & 3);
                        ov[q & 3] = g.dx * (fmaf(0.5f, Lbar, P.s) + P.e);
                        comp_add(P, Lbar);
                    }
                    if ((q & 3) == 3 && k - 3 < g.nt)
                        buffer_st4(rb, roff + 4u * att_row(g, k - 3), 0u, make_float4(ov[0], ov[1], ov[2], ov[3]));
                }
            }
            if constexpr (PAIRED) {
                float *eo = A.Ebar + cand * A.e_cs + ray;
                const float etot = (A.accumulate ? *eo : 0.f) + comp_value(ebj[j]);
                *eo = g.dx * (-A.E[cand * A.e_cs + ray] * etot);
            }
        }
    }
}

#ifndef BOAC_BODIES_ONLY
template <bool SINGLE, bool PAIRED>
__global__ __launch_bounds__(1024) void k_tail(DevGeom g, Bands bands, int rpt, int chunks, int C, TailArgs A) {
    extern __shared__ float lds[];
    k_tail_body<SINGLE, PAIRED>(blockIdx.x, lds, g, bands, rpt, chunks, C, A);
}
#endif

// Forward projection for few candidates (a grid of one-thread-per-ray workgroups would leave most of the
// GPU idle): each ray is split over kSplitLanes lanes of one wave, lane j taking the 16-sample chunks j,
// j + kSplitLanes, ... of the ray. A chunk is summed exactly as in k_fwd's single-stage path (same
// positions, same bilinear reads, FMAs in sample order), and the chunk sums are then added to the
// compensated total in chunk order after a shuffle, so every ray's result equals k_fwd's and
// k_fwd_pair's bit for bit. Single-stage images, n_samples <= 16 kSplitLanes kSplitCpl; epilogues y and
// the MLEM ratio (the likelihood keeps its per-workgroup partials in k_fwd).
constexpr int kSplitLanes = 8;
constexpr int kSplitCpl = 2;  // chunks per lane

#ifndef BOAC_BODIES_ONLY
template <int MODE, bool PAIRED>
__global__ __launch_bounds__(256) void k_fwd_split(DevGeom g, Band band, int chunks, int C, FwdArgs A) {
    static_assert(MODE != FWD_NLL, "the likelihood epilogue runs in k_fwd");
    extern __shared__ float lds[];
    int cand, chunk;
    ray_block(blockIdx.x, chunks, C, cand, chunk);
    const int nrays = g.nah * g.nb;
    const int pitch = g.n + 3;
    const float nf = (float)g.n;
    const int lane = threadIdx.x & (kSplitLanes - 1);
    const int ray = chunk * (blockDim.x / kSplitLanes) + threadIdx.x / kSplitLanes;
    const bool live = ray < nrays;
    stage_whole(A.img + cand * A.img_cs, g.n, band, lds);
    __syncthreads();

    constexpr int KC = 16, KG = KC / 4;
    const int a = live ? ray / g.nb : 0, b = live ? ray - a * g.nb : 0;
    const float2 cs = g.trig[a];
    float Ub, Vb;
    ray_base(g, sigma_of(g, b), cs.x, cs.y, Ub, Vb);
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(A.att + cand * A.att_cs, (unsigned)(4 * A.att_cs));
    const unsigned roff = 4u * (unsigned)att_base(g, a, b);
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float e_ray = (PAIRED && live) ? A.E[cand * A.e_cs + ray] : 0.f;
    const int nck = (g.nt + KC - 1) / KC;
    float part[kSplitCpl], part2[kSplitCpl];
#pragma unroll
    for (int h = 0; h < kSplitCpl; ++h) {
        part[h] = part2[h] = 0.f;
        const int ck = lane + h * kSplitLanes;
        if (!live || ck >= nck) continue;
        const int k0 = ck * KC;
        float4 v[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q) v[q] = (k0 + 4 * q < g.nt) ? buffer_ld4_stream(rs, roff, 4u * att_row(g, k0 + 4 * q)) : z4;
        float tau = (float)k0 - g.cT;
        float p = 0.f, p2 = 0.f;
#pragma unroll
        for (int q = 0; q < KC; ++q) {
            if (k0 + q < g.nt) {
                float U, V;
                sample_uv(Ub, Vb, tau, cs.x, cs.y, U, V);
                const float at = f4at(v[q >> 2], q & 3);
                const float w = bilinear_whole(lds, U, V, nf, pitch);
                p = fmaf(at, w, p);
                if constexpr (PAIRED) p2 = fmaf(opposed_att(e_ray, at), w, p2);
            }
            tau += 1.f;
        }
        part[h] = p;
        part2[h] = p2;
    }
    // the compensated total over the chunks in order (chunk ck is in lane ck % L, slot ck / L)
    const int base = (threadIdx.x & (kWave - 1)) & ~(kSplitLanes - 1);
    Comp c{0.f, 0.f}, c2{0.f, 0.f};
    for (int ck = 0; ck < nck; ++ck) {
        const int h = ck / kSplitLanes;
        const float mine = (h == 0) ? part[0] : part[kSplitCpl - 1];
        kahan_add(c, __shfl(mine, base + ck % kSplitLanes, kWave));
        if constexpr (PAIRED) {
            const float mine2 = (h == 0) ? part2[0] : part2[kSplitCpl - 1];
            kahan_add(c2, __shfl(mine2, base + ck % kSplitLanes, kWave));
        }
    }
    if (!live || lane != 0) return;
    bool zero_proj = false;
    fwd_emit<MODE>(A, cand, ray, g.dx * comp_value(c), zero_proj);
    if constexpr (PAIRED) fwd_emit<MODE>(A, cand, (a + g.nah) * g.nb + (g.nb - 1 - b), g.dx * comp_value(c2), zero_proj);
}
#endif

#ifndef BOAC_BODIES_ONLY
// ------------------------------------------------------------------ launchers
static dim3 ray_grid(const RayCfg &rc, int C) { return dim3((unsigned)(rc.chunks * C)); }

hipError_t launch_att(const DevGeom &g, const RayCfg &rc, const Bands &bands, const float *mu, float *att,
                      size_t img_cs, size_t att_cs, float *E, size_t e_cs, int C, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        const bool scan = rc.single && rc.scan_passes > 0;
        if ((scan ? rc.scan_block : rc.block) != kPersistThreads)
            return record_unsupported(r, "attenuation build planned with other than 1024 threads");
        t.kind = scan ? T_ATT_SCAN : T_ATT;
        t.variant = rc.single ? 1 : 0;
        t.u.att = {RayTask{g, bands, rc.rpt, scan ? rc.scan_chunks : rc.chunks, C}, mu, att, img_cs, att_cs, E, e_cs,
                   rc.scan_passes};
        t.grid = t.items = (scan ? rc.scan_chunks : rc.chunks) * C;
        t.lds = (unsigned)rc.lds;
        return record_task(r, t);
    }
    if (rc.single && rc.scan_passes > 0) {
        if (rc.scan_block % 64 != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_att_scan, dim3((unsigned)(rc.scan_chunks * C)), dim3(rc.scan_block), rc.lds, st, g,
                           bands.band(0, g.n), rc.scan_passes, rc.scan_chunks, C, mu, att, img_cs, att_cs, E, e_cs);
        return hipGetLastError();
    }
    if (rc.single)
        hipLaunchKernelGGL(k_att<true>, ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt, rc.chunks, C,
                           mu, att, img_cs, att_cs, E, e_cs);
    else
        hipLaunchKernelGGL(k_att<false>, ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt, rc.chunks,
                           C, mu, att, img_cs, att_cs, E, e_cs);
    return hipGetLastError();
}

template <int MODE, bool PAIRED>
static void fwd_mode(const DevGeom &g, const RayCfg &rc, const Bands &bands, const FwdArgs &a, int C,
                     hipStream_t st) {
    if constexpr (MODE != FWD_NLL) {
        if (rc.split_chunks > 0 && rc.single && a.img_comps == 1 && g.nt <= 16 * kSplitLanes * kSplitCpl) {
            hipLaunchKernelGGL((k_fwd_split<MODE, PAIRED>), dim3((unsigned)(rc.split_chunks * C)), dim3(256), rc.lds,
                               st, g, bands.band(0, g.n), rc.split_chunks, C, a);
            return;
        }
    }
    if (rc.pair && rc.single && a.img_comps == 1 && C >= 2)
        hipLaunchKernelGGL((k_fwd_pair<MODE, PAIRED>), dim3((unsigned)(rc.chunks * ((C + 1) / 2))), dim3(rc.block),
                           2 * rc.lds, st, g, bands, rc.rpt, rc.chunks, C, a);
    else if (rc.single)
        hipLaunchKernelGGL((k_fwd<MODE, true, PAIRED>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands,
                           rc.rpt, rc.chunks, C, a);
    else
        hipLaunchKernelGGL((k_fwd<MODE, false, PAIRED>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands,
                           rc.rpt, rc.chunks, C, a);
}

hipError_t launch_fwd(int mode, const DevGeom &g, const RayCfg &rc, const Bands &bands, const FwdArgs &a, int C,
                      hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        if (rc.block != kPersistThreads) return record_unsupported(r, "projection planned with other than 1024 threads");
        if (mode != FWD_NLL && rc.split_chunks > 0) return record_unsupported(r, "ray-split projection");
        TaskRec t{};
        const bool pair = rc.pair && rc.single && a.img_comps == 1 && C >= 2;
        t.kind = pair ? T_FWD_PAIR : T_FWD;
        t.variant = mode | (rc.single ? 4 : 0) | (a.E ? 8 : 0);
        t.u.fwd = {RayTask{g, bands, rc.rpt, rc.chunks, C}, a};
        t.grid = t.items = rc.chunks * (pair ? (C + 1) / 2 : C);
        t.lds = (unsigned)(pair ? 2 * rc.lds : rc.lds);
        return record_task(r, t);
    }
    const bool paired = a.E != nullptr;
    if (paired && g.nah * 2 != g.na) return hipErrorInvalidValue;
    switch (mode) {
        case FWD_PROJ: paired ? fwd_mode<FWD_PROJ, true>(g, rc, bands, a, C, st)
                              : fwd_mode<FWD_PROJ, false>(g, rc, bands, a, C, st); break;
        case FWD_RATIO: paired ? fwd_mode<FWD_RATIO, true>(g, rc, bands, a, C, st)
                               : fwd_mode<FWD_RATIO, false>(g, rc, bands, a, C, st); break;
        case FWD_NLL: paired ? fwd_mode<FWD_NLL, true>(g, rc, bands, a, C, st)
                             : fwd_mode<FWD_NLL, false>(g, rc, bands, a, C, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adj_sweep(const DevGeom &g, const RayCfg &rc, const Bands &bands, const SweepArgs &a, int C,
                            hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        if (rc.block != kPersistThreads) return record_unsupported(r, "reverse sweep planned with other than 1024 threads");
        TaskRec t{};
        t.kind = T_SWEEP;
        t.variant = (rc.single ? 1 : 0) | (a.E ? 2 : 0);
        t.u.sweep = {RayTask{g, bands, rc.rpt, rc.chunks, C}, a};
        t.grid = t.items = rc.chunks * C;
        t.lds = (unsigned)rc.lds;
        return record_task(r, t);
    }
    const bool paired = a.E != nullptr;
    if (paired != (g.nah != g.na) || (paired && (g.nah * 2 != g.na || !a.Ebar))) return hipErrorInvalidValue;
    if (paired && rc.single)
        hipLaunchKernelGGL((k_adj_sweep<true, true>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    else if (paired)
        hipLaunchKernelGGL((k_adj_sweep<false, true>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    else if (rc.single)
        hipLaunchKernelGGL((k_adj_sweep<true, false>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    else
        hipLaunchKernelGGL((k_adj_sweep<false, false>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands,
                           rc.rpt, rc.chunks, C, a);
    return hipGetLastError();
}

hipError_t launch_tail(const DevGeom &g, const RayCfg &rc, const Bands &bands, const TailArgs &a, int C,
                       hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        if (rc.block != kPersistThreads) return record_unsupported(r, "adjoint tail planned with other than 1024 threads");
        TaskRec t{};
        t.kind = T_TAIL;
        t.variant = (rc.single ? 1 : 0) | (a.E ? 2 : 0);
        t.u.tail = {RayTask{g, bands, rc.rpt, rc.chunks, C}, a};
        t.grid = t.items = rc.chunks * C;
        t.lds = (unsigned)rc.lds;
        return record_task(r, t);
    }
    const bool paired = a.E != nullptr;
    if (paired != (g.nah != g.na) || (paired && (g.nah * 2 != g.na || !a.Ebar))) return hipErrorInvalidValue;
    if (paired && rc.single)
        hipLaunchKernelGGL((k_tail<true, true>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    else if (paired)
        hipLaunchKernelGGL((k_tail<false, true>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    else if (rc.single)
        hipLaunchKernelGGL((k_tail<true, false>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    else
        hipLaunchKernelGGL((k_tail<false, false>), ray_grid(rc, C), dim3(rc.block), rc.lds, st, g, bands, rc.rpt,
                           rc.chunks, C, a);
    return hipGetLastError();
}

#endif  // BOAC_BODIES_ONLY

}  // namespace boac
