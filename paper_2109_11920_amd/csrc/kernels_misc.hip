// Rasteriser (Eqs. 3-4), its adjoint, and the small reduction / elementwise kernels.
//
// Head outline R(theta) = sum_{k=0}^{5} c_k P_k(cos theta) (the Legendre argument read as cos theta),
// brain where r < R, cranium where R < r < R + dR. Each pixel averages a C^1 coverage
// H(d) = S(clamp(d/h + 1/2, 0, 1)), S(x) = 3x^2 - 2x^3, of the signed distances d = R - r and
// d + dR over 4 x 4 sub-samples (h = pixel/4): mu = mu_b fb + mu_c (fo - fb).
#include "launch.h"

namespace boac {

constexpr int kSub = 4;

struct SubGeom {
    float r, ct;  // sub-sample radius and cos(theta)
};

__device__ __forceinline__ SubGeom subsample(const DevGeom &g, int i, int l, int p, int q) {
    const float h = g.dx * 0.25f;
    const float y = ((float)i - g.cN) * g.dx + ((float)p - 1.5f) * h;
    const float x = ((float)l - g.cN) * g.dx + ((float)q - 1.5f) * h;
    SubGeom s;
    s.r = sqrtf(fmaf(x, x, y * y));
    s.ct = (s.r > 1e-12f) ? x / s.r : 1.f;
    return s;
}

__device__ __forceinline__ void legendre6(float x, float P[6]) {
    P[0] = 1.f;
    P[1] = x;
#pragma unroll
    for (int n = 1; n < 5; ++n) P[n + 1] = ((float)(2 * n + 1) * x * P[n] - (float)n * P[n - 1]) / (float)(n + 1);
}

__device__ __forceinline__ float coverage(float d, float inv_h) {
    const float x = fminf(fmaxf(fmaf(d, inv_h, 0.5f), 0.f), 1.f);
    return x * x * (3.f - 2.f * x);
}
__device__ __forceinline__ float coverage_slope(float d, float inv_h) {
    const float x = fminf(fmaxf(fmaf(d, inv_h, 0.5f), 0.f), 1.f);
    return 6.f * x * (1.f - x) * inv_h;
}

// mu of pixel pix of candidate cidx.
__device__ __forceinline__ void raster_at(const DevGeom &g, const float *__restrict__ cand, float delta_r,
                                          float *__restrict__ mu, size_t img_cs, uint32_t *status, int cidx, int pix) {
    if (pix >= g.n * g.n) return;
    const int i = pix / g.n, l = pix - i * g.n;
    const float *th = cand + (size_t)cidx * 8;
    const float inv_h = 4.f / g.dx;
    float fb = 0.f, fo = 0.f;
    bool neg = false;
#pragma unroll
    for (int p = 0; p < kSub; ++p)
#pragma unroll
        for (int q = 0; q < kSub; ++q) {
            const SubGeom s = subsample(g, i, l, p, q);
            float P[6];
            legendre6(s.ct, P);
            float R = 0.f;
#pragma unroll
            for (int k = 0; k < 6; ++k) R = fmaf(th[k], P[k], R);
            neg |= (R < 0.f);
            const float db = R - s.r;
            fb += coverage(db, inv_h);
            fo += coverage(db + delta_r, inv_h);
        }
    fb *= 1.f / 16.f;
    fo *= 1.f / 16.f;
    // fmin/fmax inside the coverage drop NaNs: a non-finite candidate must stay visible
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) finite &= isfinite(th[k]);
    mu[(size_t)cidx * img_cs + pix] = finite ? fmaf(th[6], fb, th[7] * (fo - fb)) : __builtin_nanf("");
    if (status && (neg || !finite)) atomicOr(status + cidx, (neg ? 4u : 0u) | (finite ? 0u : 2u));
}

#ifndef BOAC_BODIES_ONLY
__global__ __launch_bounds__(256) void k_raster(DevGeom g, const float *__restrict__ cand, int C, float delta_r,
                                                float *__restrict__ mu, size_t img_cs, uint32_t *status) {
    raster_at(g, cand, delta_r, mu, img_cs, status, blockIdx.y, blockIdx.x * blockDim.x + threadIdx.x);
}
#endif

// grad_k = sum_j mubar_j dmu_j/dtheta_k for theta = (c_0..c_5, mu_b, mu_c, dR), one workgroup per
// candidate, compensated per component; written as 9 values per candidate.
// One workgroup (any size up to 1024 threads) per candidate cidx; red: 32 floats of shared memory.
__device__ __forceinline__ void k_raster_adj_body(int cidx, float *red, DevGeom g, const float *__restrict__ cand,
                                                  float delta_r, const float *__restrict__ mubar, size_t img_cs,
                                                  float *__restrict__ grad) {
    const float *th = cand + (size_t)cidx * 8;
    const float mub = th[6], muc = th[7];
    const float inv_h = 4.f / g.dx;
    Comp acc[kGradComps];
#pragma unroll
    for (int k = 0; k < kGradComps; ++k) acc[k] = Comp{0.f, 0.f};
    const float *mb = mubar + (size_t)cidx * img_cs;
    for (int pix = threadIdx.x; pix < g.n * g.n; pix += blockDim.x) {
        const float w = mb[pix];
        const int i = pix / g.n, l = pix - i * g.n;
        float gP[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float fb = 0.f, fo = 0.f, so = 0.f;
#pragma unroll
        for (int p = 0; p < kSub; ++p)
#pragma unroll
            for (int q = 0; q < kSub; ++q) {
                const SubGeom s = subsample(g, i, l, p, q);
                float P[6];
                legendre6(s.ct, P);
                float R = 0.f;
#pragma unroll
                for (int k = 0; k < 6; ++k) R = fmaf(th[k], P[k], R);
                const float db = R - s.r;
                fb += coverage(db, inv_h);
                fo += coverage(db + delta_r, inv_h);
                const float slope_o = coverage_slope(db + delta_r, inv_h);
                so += slope_o;
                const float dmu_dR = fmaf(mub - muc, coverage_slope(db, inv_h), muc * slope_o);
#pragma unroll
                for (int k = 0; k < 6; ++k) gP[k] = fmaf(dmu_dR, P[k], gP[k]);
            }
#pragma unroll
        for (int k = 0; k < 6; ++k) comp_add(acc[k], w * gP[k] * (1.f / 16.f));
        comp_add(acc[6], w * fb * (1.f / 16.f));
        comp_add(acc[7], w * (fo - fb) * (1.f / 16.f));
        // dR moves only the outer edge: d mu / d dR = mu_c mean H'(d_b + dR)
        comp_add(acc[8], w * muc * so * (1.f / 16.f));
    }
    for (int k = 0; k < kGradComps; ++k) {
        const Comp r = block_reduce(acc[k], red);
        if (threadIdx.x == 0) grad[(size_t)cidx * kGradComps + k] = comp_value(r);
    }
}

#ifndef BOAC_BODIES_ONLY
__global__ __launch_bounds__(256) void k_raster_adj(DevGeom g, const float *__restrict__ cand, float delta_r,
                                                    const float *__restrict__ mubar, size_t img_cs,
                                                    float *__restrict__ grad) {
    __shared__ float red[32];
    k_raster_adj_body(blockIdx.x, red, g, cand, delta_r, mubar, img_cs, grad);
}
#endif

#ifndef BOAC_BODIES_ONLY
__global__ void k_fill(float *p, size_t count, float v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
#endif
#ifndef BOAC_BODIES_ONLY
__global__ void k_fill_u32(uint32_t *p, size_t count, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
#endif
#ifndef BOAC_BODIES_ONLY
__global__ void k_mul_copy(const float *a, const float *b, float *out, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        out[i] = a[i] * b[i];
}
#endif

#ifndef BOAC_BODIES_ONLY
__global__ void k_copy(const float *src, float *dst, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
#endif

// Adjoint of the objective terms y - S ln y at y = y^K (element t of C x nrays).
__device__ __forceinline__ void ybar_final_at(const float *meas, const float *yK, float *ybar, int nrays,
                                              size_t sino_cs, size_t t) {
    const size_t c = t / nrays, i = t - c * nrays;
    const float y = yK[c * sino_cs + i], S = meas[i];
    // dJ/dy = 1 - S / y, as (y - S) / y: exact difference where y is within a factor of 2 of S
    ybar[c * sino_cs + i] = (y > 0.f) ? (y - S) / y : (S == 0.f ? 1.f : 0.f);
}
#ifndef BOAC_BODIES_ONLY
__global__ void k_ybar_final(const float *meas, const float *yK, float *ybar, int C, int nrays, size_t sino_cs) {
    const size_t total = (size_t)C * nrays;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x)
        ybar_final_at(meas, yK, ybar, nrays, sino_cs, t);
}
#endif

// The part of the likelihood that depends on the measurement alone, summed in double: per bin with
// S > 0, ln Gamma(S + 1) - S ln S + S. The projection's epilogue adds y - S - S ln(y / S) per bin (y for
// S = 0), so that J = sum of both is Eq. (5) rearranged: every term the projection adds is of the size of
// the misfit, not of S ln y, and J keeps its FP32 precision at high counts where the model fits.
// One workgroup's sum over bins first, first + stride, ... in a fixed order (each thread's bins in
// turn, a butterfly in each wave, then the waves in order), returned to thread 0; flag gets bit 8 for
// negative counts. red: scratch of one double per wave (8-byte aligned).
__device__ __forceinline__ double lgamma_block_sum(double *red, const float *meas, int count, int first, int stride,
                                                   uint32_t *flag) {
    double c = 0.0;
    bool neg = false;
    for (int i = first; i < count; i += stride) {
        const float Sf = meas[i];
        neg |= !(Sf >= 0.f);
        if (Sf > 0.f) {
            const double S = (double)Sf;
            c += (lgamma(S + 1.0) - S * log(S)) + S;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if (lane == 0) red[wave] = c;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t += red[w];
    if (neg) atomicOr(flag, 8u);
    return t;
}

__device__ __forceinline__ void put_double(float2 *out, double t) {
    const float hi = (float)t;
    out[0] = make_float2(hi, (float)(t - (double)hi));
}

// The whole constant in one workgroup (the persistent executor's task); out[0] as (value, remainder).
__device__ __forceinline__ void k_lgamma_sum_body(float *red, const float *meas, int count, float2 *out,
                                                  uint32_t *flag) {
    const double t = lgamma_block_sum(reinterpret_cast<double *>(red), meas, count, threadIdx.x, blockDim.x, flag);
    if (threadIdx.x == 0) put_double(out, t);
}

#ifndef BOAC_BODIES_ONLY
__global__ __launch_bounds__(512) void k_lgamma_sum(const float *meas, int count, float2 *out, uint32_t *flag) {
    __shared__ __align__(8) float red[32];
    k_lgamma_sum_body(red, meas, count, out, flag);
}

// The constant over gridDim.x workgroups: workgroup b sums the bins b * blockDim.x + tid + k * gridDim.x *
// blockDim.x into part[b]; k_lgamma_final adds the parts in order.
__global__ __launch_bounds__(512) void k_lgamma_part(const float *meas, int count, double *part, uint32_t *flag) {
    __shared__ double red[16];
    const double t = lgamma_block_sum(red, meas, count, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                                      flag);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_lgamma_final(const double *part, int nparts, float2 *out) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int p = 0; p < nparts; ++p) t += part[p];
    put_double(out, t);
}
#endif

// J[c] = sum of the per-workgroup NLL partials + the ln Gamma constant; status bits.
__device__ __forceinline__ void nll_finish_at(const float2 *partial, int chunks, int C, const float2 *lg,
                                              const uint32_t *meas_flag, float *obj, uint32_t *status, int c) {
    if (c >= C) return;
    Comp acc{lg->x, lg->y};
    for (int j = 0; j < chunks; ++j) {
        const float2 p = partial[(size_t)c * chunks + j];
        comp_merge(acc, Comp{p.x, p.y});
    }
    const float J = comp_value(acc);
    obj[c] = J;
    if (status) {
        uint32_t st = status[c] | (meas_flag ? *meas_flag : 0u);
        if (!isfinite(J)) st |= 2u;
        status[c] = st;
    }
}

#ifndef BOAC_BODIES_ONLY
__global__ void k_nll_finish(const float2 *partial, int chunks, int C, const float2 *lg, const uint32_t *meas_flag,
                             float *obj, uint32_t *status) {
    nll_finish_at(partial, chunks, C, lg, meas_flag, obj, status, blockIdx.x * blockDim.x + threadIdx.x);
}
#endif

// Reverse of F^{n+1} = F^n Q^n (Q^n = b^n / s):
//   bbar = Fbar F^n / s,  sbar -= Fbar F^{n+1} / s,  Fbar_direct = Fbar Q^n      (0 where s <= 0)
__device__ __forceinline__ void adj_elem_at(const AdjElemArgs &A, size_t t) {
    {
        const size_t c = t / A.npix, j = t - c * A.npix;
        const size_t o = c * A.img_cs + j;
        const float fb = A.fbar[o], F = A.F[o], Q = A.Q[o], sv = A.s[o];
        float bbar = 0.f, sb = 0.f;
        if (sv > 0.f) {
            bbar = fb * F / sv;
            sb = fb * (F * Q) / sv;
        }
        A.sbar[o] -= sb;
        A.pair[o] = make_float2(bbar, F * Q);
        A.fbar_direct[o] = fb * Q;
    }
}

#ifndef BOAC_BODIES_ONLY
__global__ void k_adj_elem(AdjElemArgs A) {
    const size_t total = (size_t)A.npix * A.C;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x)
        adj_elem_at(A, t);
}
#endif

// (a, b) pairs; a NULL image stands for its constant
#ifndef BOAC_BODIES_ONLY
__global__ void k_pack_pair(const float *a, float a_const, const float *b, float b_const, float2 *out, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        out[i] = make_float2(a ? a[i] : a_const, b ? b[i] : b_const);
}
#endif

// Copies the first ncomp of the kGradComps raster-adjoint components per candidate; status bit 2 if
// any copied value is not finite.
__device__ __forceinline__ void grad_finish_at(const float *grad, int C, int ncomp, float *d_grad, uint32_t *status,
                                               int c) {
    if (c >= C) return;
    bool bad = false;
    for (int k = 0; k < ncomp; ++k) {
        const float v = grad[(size_t)c * kGradComps + k];
        bad |= !isfinite(v);
        d_grad[(size_t)c * ncomp + k] = v;
    }
    if (bad && status) status[c] |= 2u;
}

#ifndef BOAC_BODIES_ONLY
__global__ void k_grad_finish(const float *grad, int C, int ncomp, float *d_grad, uint32_t *status) {
    grad_finish_at(grad, C, ncomp, d_grad, status, blockIdx.x * blockDim.x + threadIdx.x);
}
#endif

#ifndef BOAC_BODIES_ONLY
// ------------------------------------------------------------------ launchers
static unsigned fill_blocks(size_t count) {
    size_t b = (count + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_raster(const DevGeom &g, const float *cand, int C, float delta_r, float *mu, size_t img_cs,
                         uint32_t *status, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_RASTER;
        t.u.raster = {g, cand, delta_r, mu, img_cs, status, (g.n * g.n + 255) / 256};
        t.grid = t.u.raster.nbx * C;
        t.items = (t.grid + 3) / 4;
        return record_task(r, t);
    }
    for (int c0 = 0; c0 < C; c0 += 65535) {
        const int n = C - c0 < 65535 ? C - c0 : 65535;
        const dim3 grid((unsigned)((g.n * g.n + 255) / 256), (unsigned)n);
        hipLaunchKernelGGL(k_raster, grid, dim3(256), 0, st, g, cand + (size_t)c0 * 8, n, delta_r,
                           mu + (size_t)c0 * img_cs, img_cs, status ? status + c0 : nullptr);
    }
    return hipGetLastError();
}
hipError_t launch_raster_adj(const DevGeom &g, const float *cand, int C, float delta_r, const float *mubar,
                             size_t img_cs, float *grad, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_RASTER_ADJ;
        t.u.raster_adj = {g, cand, delta_r, mubar, img_cs, grad};
        t.grid = t.items = C;
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_raster_adj, dim3((unsigned)C), dim3(256), 0, st, g, cand, delta_r, mubar, img_cs, grad);
    return hipGetLastError();
}
hipError_t launch_fill(float *p, size_t count, float v, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_FILL;
        t.u.elem.out = p;
        t.u.elem.fa = v;
        t.u.elem.count = count;
        t.grid = t.items = (int)((t.u.elem.count + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks(count)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_FILL_U32;
        t.u.elem.out = p;
        t.u.elem.u = v;
        t.u.elem.count = count;
        t.grid = t.items = (int)((t.u.elem.count + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(count)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}
hipError_t launch_mul_copy(const float *a, const float *b, float *out, size_t count, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_MUL_COPY;
        t.u.elem.out = out;
        t.u.elem.a = a;
        t.u.elem.b = b;
        t.u.elem.count = count;
        t.grid = t.items = (int)((t.u.elem.count + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_mul_copy, dim3(fill_blocks(count)), dim3(256), 0, st, a, b, out, count);
    return hipGetLastError();
}
hipError_t launch_copy(const float *src, float *dst, size_t count, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_COPY;
        t.u.elem.out = dst;
        t.u.elem.a = src;
        t.u.elem.count = count;
        t.grid = t.items = (int)((t.u.elem.count + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_copy, dim3(fill_blocks(count)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}
hipError_t launch_ybar_final(const float *meas, const float *yK, float *ybar, int C, int nrays, size_t sino_cs,
                             hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_YBAR;
        t.u.ybar = {meas, yK, ybar, C, nrays, sino_cs};
        t.grid = t.items = (int)(((size_t)C * nrays + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_ybar_final, dim3(fill_blocks((size_t)C * nrays)), dim3(256), 0, st, meas, yK, ybar, C, nrays,
                       sino_cs);
    return hipGetLastError();
}
hipError_t launch_lgamma_sum(const float *meas, int count, float2 *out, uint32_t *flag, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_LGAMMA;
        t.u.lgamma = {meas, count, out, flag};
        t.grid = t.items = 1;
        return record_task(r, t);
    }
    // 512-thread workgroups (double-precision ln Gamma needs more than the 128 registers a 1024-thread
    // workgroup leaves each lane), about 8 bins per thread, at most kLgammaParts of them; the parts in
    // out[2..]
    const int nparts = std::min(kLgammaParts, std::max(1, (count + 4095) / 4096));
    double *part = reinterpret_cast<double *>(out + 2);
    hipLaunchKernelGGL(k_lgamma_part, dim3((unsigned)nparts), dim3(512), 0, st, meas, count, part, flag);
    hipLaunchKernelGGL(k_lgamma_final, dim3(1), dim3(64), 0, st, (const double *)part, nparts, out);
    return hipGetLastError();
}
hipError_t launch_nll_finish(const float2 *partial, int chunks, int C, const float2 *lg, const uint32_t *meas_flag,
                             float *obj, uint32_t *status, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_NLL_FINISH;
        t.u.nll = {partial, chunks, C, lg, meas_flag, obj, status};
        t.grid = t.items = (C + kPersistThreads - 1) / kPersistThreads;
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_nll_finish, dim3((unsigned)((C + 63) / 64)), dim3(64), 0, st, partial, chunks, C, lg,
                       meas_flag, obj, status);
    return hipGetLastError();
}
hipError_t launch_adj_elem(const AdjElemArgs &a, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_ADJ_ELEM;
        t.u.adj = a;
        t.grid = t.items = (int)(((size_t)a.npix * a.C + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_adj_elem, dim3(fill_blocks((size_t)a.npix * a.C)), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_pack_pair(const float *a, float a_const, const float *b, float b_const, float2 *out, size_t count,
                            hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_PACK_PAIR;
        t.u.elem.out = out;
        t.u.elem.a = a;
        t.u.elem.b = b;
        t.u.elem.fa = a_const;
        t.u.elem.fb = b_const;
        t.u.elem.count = count;
        t.grid = t.items = (int)((t.u.elem.count + kPersistElems - 1) / kPersistElems);
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_pack_pair, dim3(fill_blocks(count)), dim3(256), 0, st, a, a_const, b, b_const, out, count);
    return hipGetLastError();
}
hipError_t launch_grad_finish(const float *grad, int C, int ncomp, float *d_grad, uint32_t *status, hipStream_t st) {
    if (TaskRecorder *r = task_recorder()) {
        TaskRec t{};
        t.kind = T_GRAD_FINISH;
        t.u.gfin = {grad, C, ncomp, d_grad, status};
        t.grid = t.items = (C + kPersistThreads - 1) / kPersistThreads;
        return record_task(r, t);
    }
    hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)((C + 63) / 64)), dim3(64), 0, st, grad, C, ncomp, d_grad,
                       status);
    return hipGetLastError();
}

#endif  // BOAC_BODIES_ONLY

}  // namespace boac
