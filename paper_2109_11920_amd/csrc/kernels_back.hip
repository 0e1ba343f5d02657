// Pixel-driven exact transpose of the attenuated projector (the MLEM backprojection, Eq. (2)
// transposed), fused with the MLEM normalise/update step.
//
// (A^T z)_j = dx sum_a sum_{(b,k)} W_{abk,j} att_abk z_ab. For each angle, pixel j receives from the
// samples whose bilinear footprint covers it; those lie in a (2 hb + 1) x 3 window of (bin, k) around
// the pixel's position in the rotated sample lattice, each with weight hat(U_bk - l) * hat(V_bk - i)
// (hat(x) = max(0, 1 - |x|)), i.e. the forward projector's bilinear weight of that pixel.
//
// A workgroup owns a TW x TH tile of pixels of CG candidates of one slice and loops over every angle:
//   1. stage the tile's footprint in (sample, bin) of att into LDS with the CG candidates
//      interleaved, so that one wide LDS read returns a window sample for every candidate (k_back
//      applies the ray weights z per window column; k_back_slid folds them into the staged values);
//   2. each thread computes the window weights of its pixels once (incrementally from the window
//      centre) and applies them to all CG candidates.
// Angle sums run in blocks of 8 angles, each block added to a compensated total. Because the
// workgroup sees all angles of its pixels, the MLEM update F <- F * b / s is its epilogue: no partial
// images are written.
#include "launch.h"

namespace boac {

template <int CG>
struct Vec;
template <>
struct Vec<1> {
    float v[1];
    __device__ __forceinline__ void load(const float *p) { v[0] = p[0]; }
};
template <>
struct Vec<2> {
    float v[2];
    __device__ __forceinline__ void load(const float *p) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    }
};
template <>
struct Vec<4> {
    float v[4];
    __device__ __forceinline__ void load(const float *p) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
};

template <>
struct Vec<8> {
    float v[8];
    __device__ __forceinline__ void load(const float *p) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        const float4 b = *reinterpret_cast<const float4 *>(p + 4);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
        v[4] = b.x;
        v[5] = b.y;
        v[6] = b.z;
        v[7] = b.w;
    }
};

// hat(x) = max(0, 1 - |x|); since 1 - |x| <= 1 this equals clamp(1 - |x|, 0, 1), which is one VALU
// instruction (subtract with the clamp bit).
__device__ __forceinline__ float hat1(float x) { return __builtin_amdgcn_fmed3f(1.f - fabsf(x), 0.f, 1.f); }
// hat(du) hat(dv) in two instructions: with h = hat(dv) in [0, 1], h - |du| h = h (1 - |du|) lies in
// [0, 1] where |du| <= 1 and is at most 0 elsewhere, so its clamp to [0, 1] (the FMA's clamp bit) is
// the product, rounded once
__device__ __forceinline__ float hat2(float du, float dv) {
    const float h = hat1(dv);
    return __builtin_amdgcn_fmed3f(fmaf(-fabsf(du), h, h), 0.f, 1.f);
}

// Rows of the footprint rectangle a wave stages per angle (waves take rows wave, wave + 4, ...).
template <int TW, int TH>
struct StageRows {
    // rectangle height <= ceil(sqrt((TW-1)^2 + (TH-1)^2)) + 8 (see the host's plan), over 4 waves
    static constexpr int value = (TW == 16 && TH == 16) ? 8 : (TW == 32 && TH == 16) ? 11 : 14;
};

// Prefetch slots per thread: the largest footprint rectangle (wb x wk, bounded by the host's plan)
// over 256 threads.
template <int TW, int TH, int HB>
struct StageSlots {
    static constexpr int value = (HB > 1) ? 8 : (TW == 16 && TH == 16) ? 4 : (TW == 32 && TH == 16) ? 8 : 11;
};

#ifndef BOAC_BODIES_ONLY
template <int CG, int TW, int TH, int HB>
__global__ __launch_bounds__(256) void k_back(DevGeom g, BackCfg T, BackArgs A, int mode) {
    constexpr int PPT = (TW * TH) / 256;
    constexpr int ME = StageSlots<TW, TH, HB>::value;  // prefetch slots per thread
    extern __shared__ float lds[];  // [wkmax][wbmax][CG] footprint, then [wbmax][CG] ray weights
    const int ntiles = T.tiles_x * T.tiles_y;
    const int ngroups = (A.C + CG - 1) / CG;
    const int total = ntiles * ngroups;
    int id = blockIdx.x;
    // the tiles of one candidate group run on one XCD (workgroups are dealt round-robin to the 8
    // XCDs): their footprints overlap in L2. A plan option, chosen by the autotuner.
    if (T.xcd_remap && (total & 7) == 0) id = (id & 7) * (total >> 3) + (id >> 3);
    const int grp = id / ntiles;
    const int tile = id - grp * ntiles;
    const int ty = tile / T.tiles_x, tx = tile - ty * T.tiles_x;
    const int l0 = tx * TW, i0 = ty * TH;
    const int c0 = grp * CG;
    const int ncg = min(CG, A.C - c0);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const float inv_bscale = 1.f / g.bscale;
    const bool weighted = (mode != BACK_SENS && mode != BACK_FIELD);
    const float *src = (mode == BACK_FIELD) ? A.z : A.att;
    float *zl = lds + (size_t)T.wkmax * T.wbmax * CG;
    const int4 *rects = T.rects + (size_t)tile * g.na;

    // per-candidate buffer resources (uniform); candidates past the batch end read as zero
    __amdgpu_buffer_rsrc_t srcq[CG], zq[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        const bool live = q < ncg;
        const int cq = c0 + min(q, ncg - 1);
        srcq[q] = buffer_rsrc(src + (size_t)cq * A.att_cs, live ? (unsigned)(4 * A.att_cs) : 0u);
        zq[q] = buffer_rsrc(weighted ? A.z + (size_t)cq * A.sino_cs : src, (live && weighted) ? (unsigned)(4 * A.sino_cs) : 0u);
    }

    float xj[PPT], yj[PPT], xcj[PPT], ycj[PPT];
    bool pv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * 256;
        const int py = p / TW, px = p % TW;
        pv[j] = (l0 + px < g.n) && (i0 + py < g.n);
        xj[j] = (float)(l0 + px);
        yj[j] = (float)(i0 + py);
        xcj[j] = xj[j] - g.cN;
        ycj[j] = yj[j] - g.cN;
    }
    Comp acc[PPT][CG];
    float blk[PPT][CG];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int q = 0; q < CG; ++q) {
            acc[j][q] = Comp{0.f, 0.f};
            blk[j][q] = 0.f;
        }

    const unsigned a_stride4 = 4u * (unsigned)g.slab;
    // The footprint rectangle is staged with a fixed pitch P = wbmax (height wkmax), so each thread's
    // prefetch slots e = tid + 256 m have fixed rectangle coordinates (kk, bb) for the whole tile.
    const int P = T.wbmax;
    const int PH = T.wbmax * T.wkmax;
    int skk[ME], sbb[ME];
    float fkk[ME], fbb[ME];
#pragma unroll
    for (int m = 0; m < ME; ++m) {
        const int e = threadIdx.x + 256 * m;
        skk[m] = e / P;
        sbb[m] = e - skk[m] * P;
        if (e >= PH) skk[m] = 1 << 20;  // never inside a rectangle
        fkk[m] = (float)skk[m];
        fbb[m] = (float)sbb[m];
    }
    // union of the tile pixels' bilinear supports (open): samples outside it have zero weight for
    // every pixel of the tile, so they are neither loaded nor gathered (their LDS slot holds 0)
    const float sup_l0 = (float)l0 - 1.f - 1e-3f, sup_l1 = (float)min(l0 + TW - 1, g.n - 1) + 1.f + 1e-3f;
    const float sup_i0 = (float)i0 - 1.f - 1e-3f, sup_i1 = (float)min(i0 + TH - 1, g.n - 1) + 1.f + 1e-3f;
    float pre[ME][CG];
    float prez[CG];
    auto prefetch = [&](int a, int4 r) {
        const unsigned abase = (unsigned)a * a_stride4;
        const float2 cs = g.trig[a];
        // image position of the rectangle's corner sample and its steps per bin / per sample
        float Ur, Vr;
        {
            float Ub, Vb;
            ray_base(g, sigma_of(g, r.x), cs.x, cs.y, Ub, Vb);
            sample_uv(Ub, Vb, tau_of(g, r.y), cs.x, cs.y, Ur, Vr);
        }
        const float ubs = cs.x * g.bscale, vbs = cs.y * g.bscale;
#pragma unroll
        for (int m = 0; m < ME; ++m) {
            const int kk = skk[m], bb = sbb[m];
            const int b = r.x + bb, k = r.y + kk;
            const float U = fmaf(fkk[m], -cs.y, fmaf(fbb[m], ubs, Ur));
            const float V = fmaf(fkk[m], cs.x, fmaf(fbb[m], vbs, Vr));
            const bool ok = (U > sup_l0) && (U < sup_l1) && (V > sup_i0) && (V < sup_i1) && (kk < r.w) &&
                            (bb < r.z) && ((unsigned)b < (unsigned)g.nb) && ((unsigned)k < (unsigned)g.nt);
            const unsigned off = abase + 4u * (att_row(g, k) + att_col(b));
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                float v = 0.f;
                if (ok) v = buffer_ld(srcq[q], off);
                pre[m][q] = v;
            }
        }
        // ray weights of the rectangle's bins: one bin per lane (first wave)
        const int b = r.x + lane;
        const bool bin_ok = (lane < r.z) && ((unsigned)b < (unsigned)g.nb);
        const unsigned zoff = 4u * (unsigned)(a * g.nb + b);
#pragma unroll
        for (int q = 0; q < CG; ++q) {
            float z = bin_ok ? 1.f : 0.f;
            if (weighted && bin_ok) z = buffer_ld(zq[q], zoff);
            prez[q] = z;
        }
    };

    int4 cur = rects[0];
    prefetch(0, cur);

    for (int a = 0; a < g.na; ++a) {
        __syncthreads();  // previous gather done with the LDS
        // ---- write the prefetched rectangle (CG candidates interleaved) and the ray weights
        {
#pragma unroll
            for (int m = 0; m < ME; ++m) {
                const int e = threadIdx.x + 256 * m;
                if (e >= PH) break;
                float *dst = lds + e * CG;
                if constexpr (CG == 8) {
                    reinterpret_cast<float4 *>(dst)[0] = make_float4(pre[m][0], pre[m][1], pre[m][2], pre[m][3]);
                    reinterpret_cast<float4 *>(dst)[1] = make_float4(pre[m][4], pre[m][5], pre[m][6], pre[m][7]);
                } else if constexpr (CG == 4) {
                    reinterpret_cast<float4 *>(dst)[0] = make_float4(pre[m][0], pre[m][1], pre[m][2], pre[m][3]);
                } else if constexpr (CG == 2) {
                    reinterpret_cast<float2 *>(dst)[0] = make_float2(pre[m][0], pre[m][1]);
                } else {
                    dst[0] = pre[m][0];
                }
            }
            if (wave == 0 && lane < P) {
#pragma unroll
                for (int q = 0; q < CG; ++q) zl[lane * CG + q] = prez[q];
            }
        }
        __syncthreads();
        const int4 r = cur;
        // ---- issue the next angle's loads; they complete while this angle's gather runs
        if (a + 1 < g.na) {
            cur = rects[a + 1];
            prefetch(a + 1, cur);
        }

        // ---- gather: window weights once per pixel, applied to every candidate
        // U(b,k) = sigma_b c - tau_k s + cN with sigma_b = (b - cB) bscale, tau_k = k - cT:
        // one bin step moves (U, V) by (c, s) bscale, one k step by (-s, c)
        const float2 cs = g.trig[a];
        const float c = cs.x, s = cs.y;
        const float ub = c * g.bscale, vb = s * g.bscale;
        const float fbl = (float)r.x, fkl = (float)r.y, fP = (float)P;
        const float bmin = fbl + (float)HB, bmax = fbl + (float)(r.z - 1 - HB);
        const float kmin = fkl + 1.f, kmax = fkl + (float)(r.w - 2);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!pv[j]) continue;
            const float xc = xcj[j], yc = ycj[j];
            const float Sj = fmaf(xc, c, yc * s) * inv_bscale + g.cB;
            const float Tj = fmaf(yc, c, -xc * s) + g.cT;
            // window centre (nearest sample), kept inside the staged rectangle
            const float bcf = __builtin_amdgcn_fmed3f(floorf(Sj + 0.5f), bmin, bmax);
            const float kcf = __builtin_amdgcn_fmed3f(floorf(Tj + 0.5f), kmin, kmax);
            // offsets of sample (bc, kc) from the pixel, same FMA sequence as the projector
            float Ub, Vb, U0, V0;
            ray_base(g, (bcf - g.cB) * g.bscale, c, s, Ub, Vb);
            sample_uv(Ub, Vb, kcf - g.cT, c, s, U0, V0);
            const float du0 = U0 - xj[j], dv0 = V0 - yj[j];
            const int row = (int)fmaf(kcf - fkl, fP, bcf - fbl);  // exact small integers
            const float *base = lds + row * CG;
            const float *zb = zl + (int)(bcf - fbl) * CG;
            const int rstep = P * CG;
#pragma unroll
            for (int db = -HB; db <= HB; ++db) {
                const float dub = fmaf((float)db, ub, du0);
                const float dvb = fmaf((float)db, vb, dv0);
                float part[CG];
#pragma unroll
                for (int q = 0; q < CG; ++q) part[q] = 0.f;
#pragma unroll
                for (int dk = -1; dk <= 1; ++dk) {
                    const float du = fmaf((float)dk, -s, dub);
                    const float dv = fmaf((float)dk, c, dvb);
                    const float w = hat2(du, dv);
                    Vec<CG> gv;
                    gv.load(base + dk * rstep + db * CG);
#pragma unroll
                    for (int q = 0; q < CG; ++q) part[q] = fmaf(w, gv.v[q], part[q]);
                }
                Vec<CG> zv;
                zv.load(zb + db * CG);
#pragma unroll
                for (int q = 0; q < CG; ++q) blk[j][q] = fmaf(part[q], zv.v[q], blk[j][q]);
            }
        }
        if ((a & 7) == 7 || a == g.na - 1) {
#pragma unroll
            for (int j = 0; j < PPT; ++j)
#pragma unroll
                for (int q = 0; q < CG; ++q) {
                    comp_add(acc[j][q], blk[j][q]);
                    blk[j][q] = 0.f;
                }
        }
    }

    // ---- epilogue
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (!pv[j]) continue;
        const size_t pix = (size_t)yj[j] * g.n + (size_t)xj[j];
#pragma unroll
        for (int q = 0; q < CG; ++q) {
            if (q >= ncg) break;
            const size_t o = (size_t)(c0 + q) * A.img_cs + pix;
            const float v = comp_value(acc[j][q]);
            if (mode == BACK_FIELD) {
                A.out[o] = v;
            } else if (mode == BACK_MLEM) {
                const float b = g.dx * v;
                const float sv = A.s[o];
                const float Q = (sv > 0.f) ? b / sv : 0.f;
                A.out[o] = A.F[o] * Q;
                if (A.q_out) A.q_out[o] = Q;
            } else if (mode == BACK_ADJ) {
                A.out[o] = fmaf(g.dx, v, A.aux[o]);
            } else {
                A.out[o] = g.dx * v;
            }
        }
    }
}
#endif

// ---------------------------------------------------------------------------------------------------
// Slid-block variant (16 x 16 pixel tiles, one-bin half window, at least 32 bins and samples).
//
// The staged footprint is a fixed 32 x 32 block of (sample, bin) whose corner (b0, k0) the host slides
// inside the sinogram so that it contains the tile's footprint rectangle clipped to the sinogram. Every
// staged position is then a real sample: no range tests. Thread t stages bin column b0 + (t & 31) of
// sample rows k0 + (t >> 5) + 8 m, m = 0..3, so its four slots share one per-lane byte offset and
// differ by uniform row steps. The ray weight z_ab is folded in while staging, so LDS holds att * z
// and every window tap is an immediate offset from one LDS address.
//
// A sample outside the union of the tile pixels' open supports is not loaded: it is gathered only
// with weight hat() = 0, so its value need only be finite, and the lane keeps its register's previous
// (finite, initially zero) contents.
//
// Window centres are clamped to [b0 + 1, b0 + 30] x [k0 + 1, k0 + 30]. Inside the sinogram this never
// moves the centre of a pixel whose nearest sample is a real one (the host's rectangle has one sample
// of margin beyond every window); at the sinogram's edges it moves the window only away from bins or
// samples that do not exist, so every tap with a non-zero weight is still gathered.
//
// LDS layout: rows of kSlidPitch slots, each slot 4 candidates wide (one 16-byte read) or narrower;
// 8 candidates use two such planes. A wave's 64 pixels are grouped 4 x 2 per 8 lanes, and the pitch
// of 34 slots spreads the window taps of those 8 pixels over the LDS banks better than a pitch of 32
// (which maps every row of a column to the same banks) or a 16 x 1 row of pixels.
template <int CG>
struct SlidLayout {
    static constexpr int V = CG < 4 ? CG : 4;   // candidates per slot (per plane)
    static constexpr int PLANES = CG / V;
    static constexpr int PLANE = kSlidBlock * kSlidPitch * V;  // floats per plane
};

#ifndef BOAC_BODIES_ONLY
template <int CG, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_back_slid(DevGeom g, BackCfg T, BackArgs A, int mode) {
    constexpr int P = kSlidBlock;
    constexpr int PL = kSlidPitch;
    constexpr int V = SlidLayout<CG>::V;
    constexpr int PLANES = SlidLayout<CG>::PLANES;
    constexpr int PLANE = SlidLayout<CG>::PLANE;
    extern __shared__ float lds[];   // [PLANES][P sample rows][PL slots][V]
    const int ntiles = T.tiles_x * T.tiles_y;
    const int ngroups = (A.C + CG - 1) / CG;
    const int total = ntiles * ngroups;
    int id = blockIdx.x;
    if (T.xcd_remap && (total & 7) == 0) id = (id & 7) * (total >> 3) + (id >> 3);
    const int grp = id / ntiles;
    const int tile = id - grp * ntiles;
    const int ty = tile / T.tiles_x, tx = tile - ty * T.tiles_x;
    const int l0 = tx * 16, i0 = ty * 16;
    const int c0 = grp * CG;
    const int ncg = min(CG, A.C - c0);
    const int tid = threadIdx.x;
    const int lane = tid & 63;

    // this thread's pixel: each 8 lanes of a wave take a 4 x 2 block, a wave a 16 x 4 band
    const int l = l0 + ((lane >> 3) & 3) * 4 + (lane & 3);
    const int i = i0 + (tid >> 6) * 4 + (lane >> 5) * 2 + ((lane >> 2) & 1);
    const bool pv = (l < g.n) && (i < g.n);
    const float xc = (float)l - g.cN, yc = (float)i - g.cN;
    const float cB5 = g.cB + 0.5f, cT5 = g.cT + 0.5f;
    const float inv_bscale = 1.f / g.bscale;

    // open support box of the tile's pixels, as half widths around the box centre (the host stores the
    // staged corner sample's position relative to that centre)
    const int l1 = min(l0 + 15, g.n - 1), i1 = min(i0 + 15, g.n - 1);
    const float hu = 0.5f * (float)(l1 - l0) + 1.f + 1e-3f;
    const float hv = 0.5f * (float)(i1 - i0) + 1.f + 1e-3f;

    // staging slots: bin column bb, sample rows kk0 + 8 m
    constexpr int ME = P * P / 256;
    const int bb = tid & (P - 1), kk0 = tid >> 5;
    const float fbb = (float)bb;
    float fkk[ME];
#pragma unroll
    for (int m = 0; m < ME; ++m) fkk[m] = (float)(kk0 + 8 * m);
    const unsigned row8 = 4u * (unsigned)(g.nb8 << 6);  // bytes of 8 sample rows (2 block rows)
    const unsigned a_stride = 4u * (unsigned)g.slab;
    const unsigned cand_src = 4u * (unsigned)A.att_cs, cand_z = 4u * (unsigned)A.sino_cs;
    const float *src = (mode == BACK_FIELD) ? A.z : A.att;
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(src + (size_t)c0 * A.att_cs, (unsigned)ncg * cand_src);
    const __amdgpu_buffer_rsrc_t rz =
        buffer_rsrc(WEIGHTED ? A.z + (size_t)c0 * A.sino_cs : src, WEIGHTED ? (unsigned)ncg * cand_z : 0u);
    const int4 *rects = T.rects + (size_t)tile * g.na;
    // uniform byte offset of each candidate slot's data; slots past the batch end re-read the last live
    // candidate (in bounds, never written out), so no load needs a branch
    unsigned qs[CG], qz[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        qs[q] = (unsigned)min(q, ncg - 1) * cand_src;
        qz[q] = (unsigned)min(q, ncg - 1) * cand_z;
    }

    Comp acc[CG];
    float blk[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        acc[q] = Comp{0.f, 0.f};
        blk[q] = 0.f;
    }

    float pre[ME][CG], zv[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        zv[q] = 1.f;
#pragma unroll
        for (int m = 0; m < ME; ++m) pre[m][q] = 0.f;
    }
    auto prefetch = [&](int a, int4 r) {
        const float2 cs = g.trig[a];
        const float iu = fmaf(fbb, cs.x * g.bscale, __int_as_float(r.z));
        const float iv = fmaf(fbb, cs.y * g.bscale, __int_as_float(r.w));
        // this thread's samples (r.y + kk0 + 8 m, r.x + bb): a per-lane offset for m = 0, and uniform
        // steps of two block rows for m > 0
        const unsigned sbase = (unsigned)a * a_stride;
        const unsigned slot_off = 4u * (att_row(g, r.y + kk0) + att_col(r.x + bb));
#pragma unroll
        for (int m = 0; m < ME; ++m) {
            const float U = fmaf(fkk[m], -cs.y, iu);
            const float V = fmaf(fkk[m], cs.x, iv);
            if (fabsf(U) < hu && fabsf(V) < hv) {
#pragma unroll
                for (int q = 0; q < CG; ++q) pre[m][q] = buffer_ld(rs, slot_off, sbase + (unsigned)m * row8 + qs[q]);
            }
        }
        if constexpr (WEIGHTED) {
            const unsigned zbase = 4u * (unsigned)(a * g.nb + r.x);
#pragma unroll
            for (int q = 0; q < CG; ++q) zv[q] = buffer_ld(rz, 4u * (unsigned)bb, zbase + qz[q]);
        }
    };

    int4 cur = rects[0];
    prefetch(0, cur);

    for (int a = 0; a < g.na; ++a) {
        __syncthreads();  // previous gather done with the LDS
        {
            float v[ME][CG];
#pragma unroll
            for (int m = 0; m < ME; ++m)
#pragma unroll
                for (int q = 0; q < CG; ++q) v[m][q] = WEIGHTED ? pre[m][q] * zv[q] : pre[m][q];
#pragma unroll
            for (int t = 0; t < ME; ++t) {
                float *d = lds + ((kk0 + 8 * t) * PL + bb) * V;
                if constexpr (CG == 8) {
                    reinterpret_cast<float4 *>(d)[0] = make_float4(v[t][0], v[t][1], v[t][2], v[t][3]);
                    reinterpret_cast<float4 *>(d + PLANE)[0] = make_float4(v[t][4], v[t][5], v[t][6], v[t][7]);
                } else if constexpr (CG == 4) {
                    reinterpret_cast<float4 *>(d)[0] = make_float4(v[t][0], v[t][1], v[t][2], v[t][3]);
                } else if constexpr (CG == 2) {
                    reinterpret_cast<float2 *>(d)[0] = make_float2(v[t][0], v[t][1]);
                } else {
                    d[0] = v[t][0];
                }
            }
        }
        __syncthreads();
        const int4 r = cur;
        if (a + 1 < g.na) {
            cur = rects[a + 1];
            prefetch(a + 1, cur);
        }

        // ---- gather
        const float2 cs = g.trig[a];
        const float c = cs.x, s = cs.y;
        const float ub = c * g.bscale, vb = s * g.bscale;
        const float fb1 = (float)(r.x + 1), fk1 = (float)(r.y + 1);
        if (pv) {
            // nearest sample (bin, sample index) of the pixel, clamped into the staged block
            const float Sj5 = fmaf(xc, c * inv_bscale, fmaf(yc, s * inv_bscale, cB5));
            const float Tj5 = fmaf(yc, c, fmaf(xc, -s, cT5));
            const float bcf = __builtin_amdgcn_fmed3f(floorf(Sj5), fb1, fb1 + (float)(P - 3));
            const float kcf = __builtin_amdgcn_fmed3f(floorf(Tj5), fk1, fk1 + (float)(P - 3));
            // offset of that sample from the pixel: U - x = sigma c - tau s - xc, V - y = sigma s + tau c - yc
            const float sig = (bcf - g.cB) * g.bscale, tau = kcf - g.cT;
            const float du0 = fmaf(sig, c, fmaf(tau, -s, -xc));
            const float dv0 = fmaf(sig, s, fmaf(tau, c, -yc));
            const int corner = (int)(kcf - fk1) * PL + (int)(bcf - fb1);  // window tap (-1, -1)
            const float *base = lds + corner * V;
#pragma unroll
            for (int db = -1; db <= 1; ++db) {
                const float dub = (db == 0) ? du0 : (db < 0 ? du0 - ub : du0 + ub);
                const float dvb = (db == 0) ? dv0 : (db < 0 ? dv0 - vb : dv0 + vb);
#pragma unroll
                for (int dk = -1; dk <= 1; ++dk) {
                    const float du = (dk == 0) ? dub : (dk < 0 ? dub + s : dub - s);
                    const float dv = (dk == 0) ? dvb : (dk < 0 ? dvb - c : dvb + c);
                    const float w = hat2(du, dv);
#pragma unroll
                    for (int h = 0; h < PLANES; ++h) {
                        Vec<V> gv;
                        gv.load(base + h * PLANE + ((dk + 1) * PL + (db + 1)) * V);
#pragma unroll
                        for (int q = 0; q < V; ++q) blk[h * V + q] = fmaf(w, gv.v[q], blk[h * V + q]);
                    }
                }
            }
        }
        if ((a & 7) == 7 || a == g.na - 1) {
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                comp_add(acc[q], blk[q]);
                blk[q] = 0.f;
            }
        }
    }

    if (!pv) return;
    const size_t pix = (size_t)i * g.n + l;
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        if (q >= ncg) break;
        const size_t o = (size_t)(c0 + q) * A.img_cs + pix;
        const float v = comp_value(acc[q]);
        if (mode == BACK_FIELD) {
            A.out[o] = v;
        } else if (mode == BACK_MLEM) {
            const float b = g.dx * v;
            const float sv = A.s[o];
            const float Q = (sv > 0.f) ? b / sv : 0.f;
            A.out[o] = A.F[o] * Q;
            if (A.q_out) A.q_out[o] = Q;
        } else if (mode == BACK_ADJ) {
            A.out[o] = fmaf(g.dx, v, A.aux[o]);
        } else {
            A.out[o] = g.dx * v;
        }
    }
}
#endif

// ---------------------------------------------------------------------------------------------------
// CG consecutive floats from LDS into registers, as wide reads where CG allows (p aligned to CG floats
// for CG <= 4, to 4 floats for CG = 8)
template <int CG>
__device__ __forceinline__ void load_cands(const float *p, float (&v)[CG]) {
    if constexpr (CG % 4 == 0) {
#pragma unroll
        for (int h = 0; h < CG / 4; ++h) {
            const float4 t = reinterpret_cast<const float4 *>(p)[h];
            v[4 * h] = t.x;
            v[4 * h + 1] = t.y;
            v[4 * h + 2] = t.z;
            v[4 * h + 3] = t.w;
        }
    } else if constexpr (CG == 2) {
        const float2 t = reinterpret_cast<const float2 *>(p)[0];
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = p[0];
    }
}

// The gather's epilogue for output element o: v is the compensated sum over the angles.
__device__ __forceinline__ void back_epilogue(const DevGeom &g, const BackArgs &A, int mode, size_t o, float v) {
    if (mode == BACK_FIELD) {
        A.out[o] = v;
    } else if (mode == BACK_MLEM) {
        const float b = g.dx * v;
        const float sv = A.s[o];
        const float Q = (sv > 0.f) ? b / sv : 0.f;
        A.out[o] = A.F[o] * Q;
        if (A.q_out) A.q_out[o] = Q;
    } else if (mode == BACK_ADJ) {
        A.out[o] = fmaf(g.dx, v, A.aux[o]);
    } else {
        A.out[o] = g.dx * v;
    }
}

// Column-group variant of the slid-block gather (n_samples a multiple of 4). The host aligns the
// block's first sample row to a multiple of 4, so the 4 samples k..k+3 (k = first row + 4 j) of a bin
// are one aligned 16-byte load in the attenuation layout (sample fastest inside a 4 x 8 block): thread
// t stages bin t % 32 of rows 4 (t / 32) .. + 3 with one 16-byte load per candidate, a quarter of the
// vector-memory instructions of the slot variant (which is bound by its vector-memory pipeline), and
// 8 lanes on consecutive bins read one whole 128-byte line. All 4 samples share the bin's ray weight,
// folded in while staging as in the slot variant. A group is loaded unless all of it lies outside the
// union of the tile pixels' supports (tested at its centre with half widths grown by 1.5 samples); a
// skipped group keeps finite values, gathered only with weight 0.
// PAIRED (opposed-ray pairing, g.nah = na/2): the slab of angle a < na/2 also stands for angle
// a + na/2, whose sample (nb-1-b, nt-1-k) sits at sample (b, k) of angle a with attenuation
// exp(-T_ab) / att and the same bilinear weights; each staged slot holds both contributions,
// att z_ab + (exp(-T_ab) / att) z_(a+na/2, nb-1-b), so one gather serves the two angles. In the
// field mode (mu_bar = W^T m_bar) the slot holds m_bar + dx Tbar_ab, the per-ray value in A.E.
// The ray weights reach the staging threads through a small LDS table (one load per bin and
// candidate, one angle ahead), and the per-angle trigonometry and block origins through scalar loads
// of host tables (BackCfg::angt, BackCfg::rectf).
// Body of k_back_col4 for workgroup `bid` of the launch's grid, run by 256 threads (thread index tid)
// on the LDS region lds. live = false: a stand-in workgroup beyond the grid (the persistent executor
// runs workgroups four to a 1024-thread group) that takes part in every barrier and loads and writes
// nothing.
template <int CG, bool WEIGHTED, bool PAIRED, bool SPLIT>
__device__ __forceinline__ void k_back_col4_body(int bid, int tid, float *lds, bool live, DevGeom g, BackCfg T,
                                                 BackArgs A, int mode) {
    constexpr int P = kSlidBlock;
    constexpr int PL = kSlidPitch;
    constexpr int V = SlidLayout<CG>::V;
    constexpr int PLANES = SlidLayout<CG>::PLANES;
    constexpr int PLANE = SlidLayout<CG>::PLANE;
    // lds: [PLANES][P rows][PL slots][V], then the ray weights wz, we
    const int ntiles = T.tiles_x * T.tiles_y;
    const int ngroups = (A.C + CG - 1) / CG;
    const int nsplit = SPLIT ? T.asplit : 1;
    const int total = ntiles * ngroups * nsplit;
    int id = bid;
    if (T.xcd_remap && (total & 7) == 0) id = (id & 7) * (total >> 3) + (id >> 3);
    const int grp = id / (ntiles * nsplit);
    const int rem = id - grp * (ntiles * nsplit);
    const int tile = rem / nsplit;
    // angle split: this workgroup gathers the held angles [a_lo, a_hi), whole 8-angle blocks
    const int split = rem - tile * nsplit;
    const int bps = ((g.nah + 7) / 8 + nsplit - 1) / nsplit;
    const int a_lo = min(split * bps * 8, g.nah), a_hi = min((split + 1) * bps * 8, g.nah);
    const int ty = tile / T.tiles_x, tx = tile - ty * T.tiles_x;
    const int l0 = tx * 16, i0 = ty * 16;
    const int c0 = grp * CG;
    const int ncg = live ? min(CG, A.C - c0) : 0;
    const int lane = tid & 63;

    // this thread's pixel: each 8 lanes of a wave take a 4 x 2 block, a wave a 16 x 4 band
    const int l = l0 + ((lane >> 3) & 3) * 4 + (lane & 3);
    const int i = i0 + (tid >> 6) * 4 + (lane >> 5) * 2 + ((lane >> 2) & 1);
    const bool pv = live && (l < g.n) && (i < g.n);
    const float xc = (float)l - g.cN, yc = (float)i - g.cN;
    const float cB5 = g.cB + 0.5f, cT5 = g.cT + 0.5f;

    // open support box of the tile's pixels (half widths around its centre)
    const int l1 = min(l0 + 15, g.n - 1), i1 = min(i0 + 15, g.n - 1);
    const float hu = 0.5f * (float)(l1 - l0) + 1.f + 1e-3f;
    const float hv = 0.5f * (float)(i1 - i0) + 1.f + 1e-3f;

    // staging group: bin bb, rows 4 kb .. 4 kb + 3
    const int bb = tid & (P - 1), kb = tid >> 5;
    const float fbb = (float)bb, fkc = (float)(4 * kb) + 1.5f;  // group centre, in samples
    const unsigned a_stride = 4u * (unsigned)g.slab;
    // byte offset of the group's first sample in the attenuation layout, less the block origin's part:
    // rows 4 kb .. + 3 are one 4-row line group (the block's first row is a multiple of 4) and bin b
    // sits at 4 att_col(b) = 16 b bytes of it
    const unsigned line_bytes = 4u * ((unsigned)g.nb8 << 5);
    const unsigned grp_off = (unsigned)kb * line_bytes + 16u * (unsigned)bb;
    const unsigned cand_src = 4u * (unsigned)A.att_cs, cand_z = 4u * (unsigned)A.sino_cs;
    const float *src = (mode == BACK_FIELD) ? A.z : A.att;
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(src + (size_t)c0 * A.att_cs, (unsigned)ncg * cand_src);
    const __amdgpu_buffer_rsrc_t rz =
        buffer_rsrc(WEIGHTED ? A.z + (size_t)c0 * A.sino_cs : src, WEIGHTED ? (unsigned)ncg * cand_z : 0u);
    const unsigned cand_e = 4u * (unsigned)A.e_cs;
    const __amdgpu_buffer_rsrc_t re =
        buffer_rsrc(PAIRED ? A.E + (size_t)c0 * A.e_cs : src, PAIRED ? (unsigned)ncg * cand_e : 0u);
    // per-angle block origins and trigonometry, read through the constant address space: the tables
    // are not written while the kernel runs, so their uniform loads stay scalar whatever the kernel
    // stores to LDS
    const int4 *rects = T.rects + (size_t)tile * g.nah;
    const float4 *rectf = T.rectf + (size_t)tile * g.nah * 2;  // float forms of the block origins
    unsigned qs[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) qs[q] = (unsigned)min(q, ncg - 1) * cand_src;

    Comp acc[CG];
    float blk[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        acc[q] = Comp{0.f, 0.f};
        blk[q] = 0.f;
    }

    // PAIRED: the initial staging values are 1 (a reciprocal is taken of them; never gathered with a
    // nonzero weight, as in the unpaired case where they are 0)
    float4 pre[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q)
        pre[q] = PAIRED ? make_float4(1.f, 1.f, 1.f, 1.f) : make_float4(0.f, 0.f, 0.f, 0.f);

    // Ray weights of the staged angle, [bin][candidate], shared through LDS: wz = z of the ray, we = its
    // opposed ray's factor exp(-T) z' (PAIRED; exp(-T) alone when unweighted). Thread t < 32 CG loads
    // those of bin t % 32 and candidate t / 32 for the next angle while the current one is gathered,
    // and writes them after the gather (the staging, their only reader, is then done); every thread of
    // a bin reads them back. One load per (bin, candidate) instead of one per staging thread, and no
    // registers held across the gather.
    float *wz = lds + PLANES * PLANE;
    float *we = wz + P * CG;
    const bool wl = (WEIGHTED || PAIRED) && tid < P * CG;
    const int wj = tid & (P - 1), wq = min(tid >> 5, CG - 1);
    const unsigned wcz = (unsigned)min(wq, ncg - 1) * cand_z, wce = (unsigned)min(wq, ncg - 1) * cand_e;
    float lz = 1.f, le = 0.f, lo = 1.f;
    auto wload = [&](int a, int4 r) {
        if (!wl) return;
        if constexpr (WEIGHTED) lz = buffer_ld(rz, 4u * (unsigned)wj + wcz, 4u * (unsigned)(a * g.nb + r.x));
        if constexpr (PAIRED) {
            // exp(-T) of ray (a, bin); the opposed ray (a + na/2, nb-1-bin) takes its weight
            le = buffer_ld(re, 4u * (unsigned)wj + wce, 4u * (unsigned)(a * g.nb + r.x));
            if constexpr (WEIGHTED)
                // bin nb-1-(r.x+wj) of angle a + na/2: the per-lane offset stays non-negative since the
                // block's last bin r.x + 31 is inside the sinogram
                lo = buffer_ld(rz, wcz + 4u * (unsigned)((a + g.nah) * g.nb + (g.nb - 1 - r.x) - wj), 0u);
        }
    };
    auto wstore = [&]() {
        if (!wl) return;
        if constexpr (WEIGHTED) lds[PLANES * PLANE + wj * CG + wq] = lz;
        if constexpr (PAIRED) lds[PLANES * PLANE + P * CG + wj * CG + wq] = WEIGHTED ? le * lo : le;
    };
    auto prefetch = [&](int a, int4 r) {
        const float4 t = const_ld(T.angt, 2 * a);  // c, s, c bscale, s bscale
        const float U = fmaf(fkc, -t.y, fmaf(fbb, t.z, __int_as_float(r.z)));
        const float V = fmaf(fkc, t.x, fmaf(fbb, t.w, __int_as_float(r.w)));
        // a group sample is within 1.5 samples of the group centre; one sample step moves (U, V) by (-s, c)
        if (fabsf(U) < fmaf(1.5f, fabsf(t.y), hu) && fabsf(V) < fmaf(1.5f, fabsf(t.x), hv)) {
            // the block origin's part of the offset is uniform: (r.y / 4) lines and 16 r.x bytes
            const unsigned org = (unsigned)a * a_stride + (unsigned)(r.y >> 2) * line_bytes + 16u * (unsigned)r.x;
#pragma unroll
            for (int q = 0; q < CG; ++q) pre[q] = buffer_ld4(rs, grp_off, org + qs[q]);
        }
    };

    int4 cur = make_int4(0, 0, 0, 0);
    if (a_lo < a_hi) {
        cur = const_ld(rects, a_lo);
        wload(a_lo, cur);
        prefetch(a_lo, cur);
    }
    const bool field = (mode == BACK_FIELD);

    for (int a = a_lo; a < a_hi; ++a) {
        // the gather's per-angle constants, loaded here so the staging hides their latency
        const float4 t0 = const_ld(T.angt, 2 * a), t1 = const_ld(T.angt, 2 * a + 1);
        const float4 f0 = const_ld(rectf, 2 * a), f1 = const_ld(rectf, 2 * a + 1);
        if (a == a_lo) wstore();  // later angles' weights are stored after the previous gather
        __syncthreads();  // previous gather done with the LDS
        // this thread's bin: z and (PAIRED) the opposed ray's factor exp(-T) z'
        float zv[CG], ez[CG];
        if constexpr (WEIGHTED) load_cands<CG>(wz + bb * CG, zv);
        if constexpr (PAIRED) load_cands<CG>(we + bb * CG, ez);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float v[CG];
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                const float x = t == 0 ? pre[q].x : t == 1 ? pre[q].y : t == 2 ? pre[q].z : pre[q].w;
                if constexpr (PAIRED) {
                    // att z + (exp(-T) / att) z'. The attenuation build stores att no smaller than the
                    // smallest normal float (exact for path lengths below ~87 optical depths) and every
                    // staged group lies inside the sinogram, so the reciprocal needs no clamp here. The
                    // field mode (unweighted) stages m_bar plus the ray's dx Tbar instead, picked by a
                    // select rather than a branch per value (its reciprocal is discarded).
                    const float ri = __builtin_amdgcn_rcpf(x);
                    if constexpr (WEIGHTED) {
                        v[q] = fmaf(ri, ez[q], x * zv[q]);
                    } else {
                        v[q] = field ? x + ez[q] : fmaf(ri, ez[q], x);
                    }
                } else {
                    v[q] = WEIGHTED ? x * zv[q] : x;
                }
            }
            float *d = lds + ((4 * kb + t) * PL + bb) * V;
            if constexpr (CG == 8) {
                reinterpret_cast<float4 *>(d)[0] = make_float4(v[0], v[1], v[2], v[3]);
                reinterpret_cast<float4 *>(d + PLANE)[0] = make_float4(v[4], v[5], v[6], v[7]);
            } else if constexpr (CG == 4) {
                reinterpret_cast<float4 *>(d)[0] = make_float4(v[0], v[1], v[2], v[3]);
            } else if constexpr (CG == 2) {
                reinterpret_cast<float2 *>(d)[0] = make_float2(v[0], v[1]);
            } else {
                d[0] = v[0];
            }
        }
        __syncthreads();
        if (a + 1 < a_hi) {
            cur = const_ld(rects, a + 1);
            wload(a + 1, cur);
            prefetch(a + 1, cur);
        }

        // ---- gather (as in the slot variant); t0 = (c, s, c bscale, s bscale), t1 = (c / bscale,
        // s / bscale, ..), f0 = (b0 + 1, k0 + 1, b0 + P - 2, k0 + P - 2), f1.x = (k0 + 1) PL + b0 + 1
        const float c = t0.x, s = t0.y;
        const float ub = t0.z, vb = t0.w;
        if (pv) {
            const float Sj5 = fmaf(xc, t1.x, fmaf(yc, t1.y, cB5));
            const float Tj5 = fmaf(yc, c, fmaf(xc, -s, cT5));
            const float bcf = __builtin_amdgcn_fmed3f(floorf(Sj5), f0.x, f0.z);
            const float kcf = __builtin_amdgcn_fmed3f(floorf(Tj5), f0.y, f0.w);
            const float sig = (bcf - g.cB) * g.bscale, tau = kcf - g.cT;
            const float du0 = fmaf(sig, c, fmaf(tau, -s, -xc));
            const float dv0 = fmaf(sig, s, fmaf(tau, c, -yc));
            // window tap (-1, -1): (kcf - k0 - 1) PL + bcf - b0 - 1, exact in FP32
            const int corner = (int)(fmaf(kcf, (float)PL, bcf) - f1.x);
            const float *base = lds + corner * V;
#pragma unroll
            for (int db = -1; db <= 1; ++db) {
                const float dub = (db == 0) ? du0 : (db < 0 ? du0 - ub : du0 + ub);
                const float dvb = (db == 0) ? dv0 : (db < 0 ? dv0 - vb : dv0 + vb);
#pragma unroll
                for (int dk = -1; dk <= 1; ++dk) {
                    const float du = (dk == 0) ? dub : (dk < 0 ? dub + s : dub - s);
                    const float dv = (dk == 0) ? dvb : (dk < 0 ? dvb - c : dvb + c);
                    const float w = hat2(du, dv);
#pragma unroll
                    for (int h = 0; h < PLANES; ++h) {
                        Vec<V> gv;
                        gv.load(base + h * PLANE + ((dk + 1) * PL + (db + 1)) * V);
#pragma unroll
                        for (int q = 0; q < V; ++q) blk[h * V + q] = fmaf(w, gv.v[q], blk[h * V + q]);
                    }
                }
                // keep the next window row's LDS reads after this row's FMAs: 12 registers of taps in
                // flight instead of 36 (71 VGPRs, one more wave per SIMD)
                if (db < 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (a + 1 < a_hi) wstore();  // the weights of angle a + 1, for its staging
        if ((a & 7) == 7 || a == g.nah - 1) {
            if constexpr (SPLIT) {
                // angle split: the block's sum goes to the partial buffer [block][candidate][pixel];
                // k_back_combine adds the blocks in order, as the loop below would
                if (pv) {
                    const size_t pix = (size_t)i * g.n + l;
#pragma unroll
                    for (int q = 0; q < CG; ++q)
                        if (q < ncg) A.blk_out[((size_t)(a >> 3) * A.C + c0 + q) * A.img_cs + pix] = blk[q];
                }
#pragma unroll
                for (int q = 0; q < CG; ++q) blk[q] = 0.f;
            } else {
#pragma unroll
                for (int q = 0; q < CG; ++q) {
                    comp_add(acc[q], blk[q]);
                    blk[q] = 0.f;
                }
            }
        }
    }

    if (!pv || SPLIT) return;
    const size_t pix = (size_t)i * g.n + l;
    // a guard rather than a break: the loop must unroll, or acc[] would live in scratch memory
#pragma unroll
    for (int q = 0; q < CG; ++q)
        if (q < ncg) back_epilogue(g, A, mode, (size_t)(c0 + q) * A.img_cs + pix, comp_value(acc[q]));
}

#ifndef BOAC_BODIES_ONLY
template <int CG, bool WEIGHTED, bool PAIRED, bool SPLIT>
__global__ __launch_bounds__(256) void k_back_col4(DevGeom g, BackCfg T, BackArgs A, int mode) {
    extern __shared__ float lds[];
    k_back_col4_body<CG, WEIGHTED, PAIRED, SPLIT>(blockIdx.x, threadIdx.x, lds, true, g, T, A, mode);
}
#endif

// Second pass of the angle-split gather: per (candidate, pixel) the 8-angle block sums, added in angle
// order to a compensated total exactly as the unsplit gather adds them, then the same epilogue.
#ifndef BOAC_BODIES_ONLY
__global__ __launch_bounds__(256) void k_back_combine(DevGeom g, BackArgs A, int nblk, int mode) {
    const size_t npix = (size_t)g.n * g.n;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)A.C * npix) return;
    const size_t c = t / npix, pix = t - c * npix;
    const size_t o = c * A.img_cs + pix;
    Comp acc{0.f, 0.f};
    for (int b = 0; b < nblk; ++b) comp_add(acc, A.blk_out[((size_t)b * A.C + c) * A.img_cs + pix]);
    back_epilogue(g, A, mode, o, comp_value(acc));
}
#endif

#ifndef BOAC_BODIES_ONLY
template <int CG, bool SPLIT>
static void back_col4_go(const DevGeom &g, const BackCfg &bc, const BackArgs &a, int mode, hipStream_t st) {
    const int ngroups = (a.C + CG - 1) / CG;
    const dim3 grid((unsigned)(bc.tiles_x * bc.tiles_y * ngroups * (SPLIT ? bc.asplit : 1)));
    const bool weighted = !(mode == BACK_SENS || mode == BACK_FIELD);
    if (a.E) {
        if (weighted)
            hipLaunchKernelGGL((k_back_col4<CG, true, true, SPLIT>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
        else
            hipLaunchKernelGGL((k_back_col4<CG, false, true, SPLIT>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
    } else if (weighted) {
        hipLaunchKernelGGL((k_back_col4<CG, true, false, SPLIT>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
    } else {
        hipLaunchKernelGGL((k_back_col4<CG, false, false, SPLIT>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
    }
}

template <int CG>
static hipError_t back_col4(const DevGeom &g, const BackCfg &bc, const BackArgs &a, int mode, hipStream_t st) {
    if (bc.asplit < 1 || (bc.asplit > 1 && !a.blk_out)) return hipErrorInvalidValue;
    if (a.E && g.nah * 2 != g.na) return hipErrorInvalidValue;
    if (bc.asplit > 1) {
        back_col4_go<CG, true>(g, bc, a, mode, st);
        const size_t n = (size_t)a.C * g.n * g.n;
        hipLaunchKernelGGL(k_back_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, a,
                           (g.nah + 7) / 8, mode);
    } else {
        back_col4_go<CG, false>(g, bc, a, mode, st);
    }
    return hipGetLastError();
}

template <int CG>
static hipError_t back_slid(const DevGeom &g, const BackCfg &bc, const BackArgs &a, int mode, hipStream_t st) {
    const int ngroups = (a.C + CG - 1) / CG;
    const dim3 grid((unsigned)(bc.tiles_x * bc.tiles_y * ngroups));
    if (mode == BACK_SENS || mode == BACK_FIELD)
        hipLaunchKernelGGL((k_back_slid<CG, false>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
    else
        hipLaunchKernelGGL((k_back_slid<CG, true>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
    return hipGetLastError();
}

template <int CG, int TW, int TH, int HB>
static hipError_t back_go(const DevGeom &g, const BackCfg &bc, const BackArgs &a, int mode, hipStream_t st) {
    const int ngroups = (a.C + CG - 1) / CG;
    const dim3 grid((unsigned)(bc.tiles_x * bc.tiles_y * ngroups));
    hipLaunchKernelGGL((k_back<CG, TW, TH, HB>), grid, dim3(256), bc.lds, st, g, bc, a, mode);
    return hipGetLastError();
}

template <int CG, int HB>
static hipError_t back_tile(const DevGeom &g, const BackCfg &bc, const BackArgs &a, int mode, hipStream_t st) {
    if (bc.tw == 16 && bc.th == 16) return back_go<CG, 16, 16, HB>(g, bc, a, mode, st);
    if (bc.tw == 32 && bc.th == 16) return back_go<CG, 32, 16, HB>(g, bc, a, mode, st);
    if (bc.tw == 32 && bc.th == 32) return back_go<CG, 32, 32, HB>(g, bc, a, mode, st);
    return hipErrorInvalidValue;
}

hipError_t launch_back(int mode, const DevGeom &g, const BackCfg &bc, const BackArgs &a, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        if (bc.slid != 2 || bc.asplit != 1 || !(bc.cg == 1 || bc.cg == 2 || bc.cg == 4) || bc.tw != 16 ||
            bc.th != 16 || bc.hb != 1)
            return record_unsupported(r, "backprojection outside the column-group gather (one to four candidates per "
                                         "workgroup, no angle split)");
        if (a.E && g.nah * 2 != g.na) return hipErrorInvalidValue;
        const bool weighted = !(mode == BACK_SENS || mode == BACK_FIELD);
        TaskRec t{};
        t.kind = T_BACK_COL4;
        t.variant = (bc.cg == 1 ? 0 : bc.cg == 2 ? 1 : 2) | (weighted ? 4 : 0) | (a.E ? 8 : 0);
        t.u.back = {g, bc, a, mode};
        t.grid = bc.tiles_x * bc.tiles_y * ((a.C + bc.cg - 1) / bc.cg);
        t.items = (t.grid + 3) / 4;
        t.sub_lds = (unsigned)((bc.lds + 15) / 16 * 16);
        t.lds = 4 * t.sub_lds;
        return record_task(r, t);
    }
    // opposed-ray pairing exists in the column-group gather only
    if ((a.E || g.nah != g.na) && bc.slid != 2) return hipErrorInvalidValue;
    if (bc.slid == 2) {
        if (bc.tw != 16 || bc.th != 16 || bc.hb != 1) return hipErrorInvalidValue;
        switch (bc.cg) {
            case 1: return back_col4<1>(g, bc, a, mode, st);
            case 2: return back_col4<2>(g, bc, a, mode, st);
            case 4: return back_col4<4>(g, bc, a, mode, st);
            case 8: return back_col4<8>(g, bc, a, mode, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (bc.slid) {
        if (bc.tw != 16 || bc.th != 16 || bc.hb != 1) return hipErrorInvalidValue;
        switch (bc.cg) {
            case 1: return back_slid<1>(g, bc, a, mode, st);
            case 2: return back_slid<2>(g, bc, a, mode, st);
            case 4: return back_slid<4>(g, bc, a, mode, st);
            case 8: return back_slid<8>(g, bc, a, mode, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (bc.hb == 1) {
        switch (bc.cg) {
            case 1: return back_tile<1, 1>(g, bc, a, mode, st);
            case 2: return back_tile<2, 1>(g, bc, a, mode, st);
            case 4: return back_tile<4, 1>(g, bc, a, mode, st);
            case 8:
                if (bc.tw == 16 && bc.th == 16) return back_go<8, 16, 16, 1>(g, bc, a, mode, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    // wider bin windows (n_bins > 1.06 n): one configuration
    if (bc.tw != 16 || bc.th != 16 || bc.cg != 1) return hipErrorInvalidValue;
    if (bc.hb == 2) return back_go<1, 16, 16, 2>(g, bc, a, mode, st);
    if (bc.hb == 3) return back_go<1, 16, 16, 3>(g, bc, a, mode, st);
    return hipErrorInvalidValue;
}

#endif  // BOAC_BODIES_ONLY

}  // namespace boac
