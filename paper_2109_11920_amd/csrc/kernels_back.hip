// Pixel-driven exact transpose of the attenuated projector (the MLEM backprojection, Eq. (2)
// transposed), fused with the MLEM normalise/update step.
//
// (A^T z)_j = dx sum_a sum_{(b,k)} W_{abk,j} att_abk z_ab. For each angle, pixel j receives from the
// samples whose bilinear footprint covers it; those lie in a (2 hb + 1) x 3 window of (bin, k) around
// the pixel's position in the rotated sample lattice. Each weight is hat(U_bk - l) * hat(V_bk - i)
// with (U_bk, V_bk) evaluated by the same FMA sequence as the forward projector, so the pair is an
// exact transpose up to FP32 rounding of the weights.
//
// A workgroup owns a tile of pixels of cg candidates of one slice and loops over every angle: it stages
// the tile's footprint rectangle of att * z (bin fastest, coalesced) for its candidates in LDS, then
// each thread gathers for its pixels. The window weights are computed once and applied to all cg
// candidates. Angle sums are compensated. Because the workgroup sees all angles of its pixels, the MLEM
// update F <- F * b / s happens in the epilogue, with no partial images in memory.
#include "launch.h"

namespace boac {

template <int MODE, int CG, int PPT, int HB>
__global__ __launch_bounds__(256) void k_back(DevGeom g, BackCfg T, BackArgs A) {
    extern __shared__ float lds[];
    const int ntiles = T.tiles_x * T.tiles_y;
    const int ngroups = (A.C + CG - 1) / CG;
    const int total = ntiles * ngroups;
    int id = blockIdx.x;
    // keep the tiles of one candidate group on one XCD: their footprints overlap in L2
    if ((total & 7) == 0) id = (id & 7) * (total >> 3) + (id >> 3);
    const int grp = id / ntiles;
    const int tile = id - grp * ntiles;
    const int ty = tile / T.tiles_x, tx = tile - ty * T.tiles_x;
    const int l0 = tx * T.tw, i0 = ty * T.th;
    const int c0 = grp * CG;
    const int ncg = min(CG, A.C - c0);
    const int rect = T.wbmax * T.wkmax;
    const float inv_bscale = 1.f / g.bscale;

    // this thread's pixels
    int pl[PPT], pi[PPT];
    bool pv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * blockDim.x;
        const int py = p / T.tw, px = p - py * T.tw;
        pl[j] = l0 + px;
        pi[j] = i0 + py;
        pv[j] = (py < T.th) && (pl[j] < g.n) && (pi[j] < g.n);
    }
    Comp acc[PPT][CG];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int q = 0; q < CG; ++q) acc[j][q] = Comp{0.f, 0.f};

    // tile corner offsets from the image centre (pixel units)
    const float xl0 = (float)l0 - g.cN, xl1 = (float)min(l0 + T.tw - 1, g.n - 1) - g.cN;
    const float yi0 = (float)i0 - g.cN, yi1 = (float)min(i0 + T.th - 1, g.n - 1) - g.cN;

    for (int a = 0; a < g.na; ++a) {
        const float2 cs = g.trig[a];
        const float c = cs.x, s = cs.y;
        // footprint rectangle: S = (x c + y s)/bscale + cB, T = (-x s + y c) + cT over the tile
        const float sx0 = xl0 * c, sx1 = xl1 * c, sy0 = yi0 * s, sy1 = yi1 * s;
        const float Smin = (fminf(sx0, sx1) + fminf(sy0, sy1)) * inv_bscale + g.cB;
        const float Smax = (fmaxf(sx0, sx1) + fmaxf(sy0, sy1)) * inv_bscale + g.cB;
        const float tx0 = -xl0 * s, tx1 = -xl1 * s, ty0 = yi0 * c, ty1 = yi1 * c;
        const float Tmin = fminf(tx0, tx1) + fminf(ty0, ty1) + g.cT;
        const float Tmax = fmaxf(tx0, tx1) + fmaxf(ty0, ty1) + g.cT;
        const int b_lo = (int)floorf(Smin + 0.5f) - HB - 1;
        const int k_lo = (int)floorf(Tmin + 0.5f) - 2;
        const int wb = min((int)floorf(Smax + 0.5f) + HB + 1 - b_lo + 1, T.wbmax);
        const int wk = min((int)floorf(Tmax + 0.5f) + 2 - k_lo + 1, T.wkmax);

        __syncthreads();
        // stage att * z (or the sample field) for the rectangle, zero outside the sinogram
        const int per = wb * wk;
        for (int idx = threadIdx.x; idx < ncg * per; idx += blockDim.x) {
            const int q = idx / per;
            const int rem = idx - q * per;
            const int kk = rem / wb, bb = rem - kk * wb;
            const int b = b_lo + bb, k = k_lo + kk;
            float v = 0.f;
            if (b >= 0 && b < g.nb && k >= 0 && k < g.nt) {
                const int cand = c0 + q;
                const size_t ai = cand * A.att_cs + ((size_t)a * g.nt + k) * g.nb + b;
                if constexpr (MODE == BACK_FIELD) {
                    v = A.z[ai];
                } else if constexpr (MODE == BACK_SENS) {
                    v = A.att[ai];
                } else {
                    v = A.att[ai] * A.z[cand * A.sino_cs + (size_t)a * g.nb + b];
                }
            }
            lds[q * rect + kk * wb + bb] = v;
        }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!pv[j]) continue;
            const float xj = (float)pl[j] - g.cN, yj = (float)pi[j] - g.cN;
            const float Sj = fmaf(xj, c, yj * s) * inv_bscale + g.cB;
            const float Tj = fmaf(yj, c, -xj * s) + g.cT;
            // window centre, kept inside the staged rectangle
            int bc = (int)floorf(Sj + 0.5f);
            int kc = (int)floorf(Tj + 0.5f);
            bc = min(max(bc, b_lo + HB), b_lo + wb - 1 - HB);
            kc = min(max(kc, k_lo + 1), k_lo + wk - 2);
            const float fl = (float)pl[j], fi = (float)pi[j];
            float part[CG];
#pragma unroll
            for (int q = 0; q < CG; ++q) part[q] = 0.f;
#pragma unroll
            for (int db = -HB; db <= HB; ++db) {
                const int b = bc + db;
                float Ub, Vb;
                ray_base(g, sigma_of(g, b), c, s, Ub, Vb);
#pragma unroll
                for (int dk = -1; dk <= 1; ++dk) {
                    const int k = kc + dk;
                    float U, V;
                    sample_uv(Ub, Vb, tau_of(g, k), c, s, U, V);
                    const float w = hat(U - fl) * hat(V - fi);
                    const int li = (k - k_lo) * wb + (b - b_lo);
#pragma unroll
                    for (int q = 0; q < CG; ++q) part[q] = fmaf(w, lds[q * rect + li], part[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < CG; ++q) comp_add(acc[j][q], part[q]);
        }
    }

    // epilogue
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (!pv[j]) continue;
        const size_t pix = (size_t)pi[j] * g.n + pl[j];
#pragma unroll
        for (int q = 0; q < CG; ++q) {
            if (q >= ncg) break;
            const size_t o = (size_t)(c0 + q) * A.img_cs + pix;
            const float v = comp_value(acc[j][q]);
            if constexpr (MODE == BACK_FIELD) {
                A.out[o] = v;
            } else if constexpr (MODE == BACK_MLEM) {
                const float b = g.dx * v;
                const float sv = A.s[o];
                const float Q = (sv > 0.f) ? b / sv : 0.f;
                A.out[o] = A.F[o] * Q;
                if (A.q_out) A.q_out[o] = Q;
            } else if constexpr (MODE == BACK_ADJ) {
                A.out[o] = fmaf(g.dx, v, A.aux[o]);
            } else {
                A.out[o] = g.dx * v;
            }
        }
    }
}

template <int MODE, int CG, int PPT>
static hipError_t back3(const DevGeom &g, const BackCfg &bc, const BackArgs &a, hipStream_t st) {
    const int ngroups = (a.C + CG - 1) / CG;
    const dim3 grid((unsigned)(bc.tiles_x * bc.tiles_y * ngroups));
    switch (bc.hb) {
        case 1: hipLaunchKernelGGL((k_back<MODE, CG, PPT, 1>), grid, dim3(256), bc.lds, st, g, bc, a); break;
        case 2: hipLaunchKernelGGL((k_back<MODE, CG, PPT, 2>), grid, dim3(256), bc.lds, st, g, bc, a); break;
        case 3: hipLaunchKernelGGL((k_back<MODE, CG, PPT, 3>), grid, dim3(256), bc.lds, st, g, bc, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE, int CG>
static hipError_t back2(const DevGeom &g, const BackCfg &bc, const BackArgs &a, hipStream_t st) {
    switch (bc.ppt) {
        case 1: return back3<MODE, CG, 1>(g, bc, a, st);
        case 2: return back3<MODE, CG, 2>(g, bc, a, st);
        case 4: return back3<MODE, CG, 4>(g, bc, a, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t back1(const DevGeom &g, const BackCfg &bc, const BackArgs &a, hipStream_t st) {
    switch (bc.cg) {
        case 1: return back2<MODE, 1>(g, bc, a, st);
        case 2: return back2<MODE, 2>(g, bc, a, st);
        case 4: return back2<MODE, 4>(g, bc, a, st);
        case 8: return back2<MODE, 8>(g, bc, a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_back(int mode, const DevGeom &g, const BackCfg &bc, const BackArgs &a, hipStream_t st) {
    switch (mode) {
        case BACK_PLAIN: return back1<BACK_PLAIN>(g, bc, a, st);
        case BACK_SENS: return back1<BACK_SENS>(g, bc, a, st);
        case BACK_MLEM: return back1<BACK_MLEM>(g, bc, a, st);
        case BACK_FIELD: return back1<BACK_FIELD>(g, bc, a, st);
        case BACK_ADJ: return back1<BACK_ADJ>(g, bc, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace boac
