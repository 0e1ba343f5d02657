// Device-side building blocks shared by the BOAC kernels (gfx950, wave64).
//
// Geometry (Eqs. 1-2, discretised as stated in include/boac.h): a sample (a, b, k) sits at pixel-index
// coordinates
//     U = sigma_b cos(phi_a) - tau_k sin(phi_a) + (n-1)/2,   V = sigma_b sin(phi_a) + tau_k cos(phi_a) + (n-1)/2
// with sigma_b = (b - (n_bins-1)/2) n / n_bins and tau_k = k - (n_samples-1)/2. Every kernel evaluates
// U and V with the same FMA sequence (sample_uv) so that the projector, the exact-transpose gather and
// the adjoint sweeps see bit-identical sample positions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace boac {

constexpr int kWave = 64;
// Smallest normal float: an attenuation is clamped to it before its reciprocal is taken (opposed-ray
// pairing), exact for every path length below ~87 optical depths.
constexpr float kMinNormal = 1.17549435e-38f;

// Reciprocal of max(x, kMinNormal). The max is taken on the bit patterns as signed integers, which order
// non-negative floats as the floats do and put every negative float below kMinNormal (same result as
// fmaxf for every non-NaN x); one integer max instead of a float max plus the NaN-quieting
// canonicalisation the compiler adds to a float max of loaded values.
// Element i of a table that no kernel writes while it reads it, loaded through the constant address
// space: with a uniform i these are scalar loads, whatever else the kernel stores.
typedef const __attribute__((address_space(4))) int *const_int_ptr;
typedef const __attribute__((address_space(4))) float *const_float_ptr;
__device__ __forceinline__ int4 const_ld(const int4 *t, int i) {
    const const_int_ptr p = (const_int_ptr)(t + i);
    return make_int4(p[0], p[1], p[2], p[3]);
}
__device__ __forceinline__ float4 const_ld(const float4 *t, int i) {
    const const_float_ptr p = (const_float_ptr)(t + i);
    return make_float4(p[0], p[1], p[2], p[3]);
}
__device__ __forceinline__ float2 const_ld(const float2 *t, int i) {
    const const_float_ptr p = (const_float_ptr)(t + i);
    return make_float2(p[0], p[1]);
}

__device__ __forceinline__ float rcp_clamped(float x) {
    return __builtin_amdgcn_rcpf(__int_as_float(max(__float_as_int(x), __float_as_int(kMinNormal))));
}

struct DevGeom {
    int n, na, nb, nt;
    // angles the attenuation tensor holds: na, or na / 2 with opposed-ray pairing (na even): ray
    // (a, b) and ray (a + na/2, nb-1-b) run along one line in opposite directions, sample k of the
    // first at sample nt-1-k of the second, and with the half-self rule their path lengths add up to
    // the ray total T, so the second ray's attenuation is exp(-T) / att of the first
    int nah;
    float dx;       // pixel size (cm)
    float cN;       // (n-1)/2
    float cB;       // (nb-1)/2
    float cT;       // (nt-1)/2
    float bscale;   // n / nb: bin spacing in pixels
    const float2 *trig;  // [na] (cos phi_a, sin phi_a)
    int nb8;        // attenuation layout: 8-bin blocks per block row, ceil(nb / 8)
    int slab;       // attenuation layout: elements per angle, 4 ceil(nt / 4) x 8 nb8
};

// Attenuation-tensor layout. Per candidate, na slabs (one per angle) of the samples (k, b); a slab is
// tiled in 4 x 8 blocks (4 consecutive samples of 8 consecutive bins, one 128-byte line), blocks
// running bin-block fastest, and within a block sample fastest: the 4 samples of one bin are 16
// contiguous bytes. Element (a, k, b) is at a slab + att_row(k) + att_col(b). A ray's samples keep a
// fixed bin part (att_col) and a row part (att_row) that depends on k only; a pixel tile's footprint
// in the slab covers about half as many partly used lines as in a row-major slab, and 4 samples of a
// bin (k a multiple of 4) are one aligned 16-byte load.
__device__ __forceinline__ unsigned att_col(int b) { return (unsigned)(((b >> 3) << 5) + ((b & 7) << 2)); }
__device__ __forceinline__ unsigned att_row(const DevGeom &g, int k) {
    return (unsigned)((k >> 2) * (g.nb8 << 5) + (k & 3));
}
__device__ __forceinline__ size_t att_base(const DevGeom &g, int a, int b) {
    return (size_t)a * (size_t)g.slab + att_col(b);
}

// Row band of an image staged in LDS: samples whose clamped row floor lies in [alo, ahi) use it;
// rows alo..ahi (inclusive) are staged, columns -1..n+1, zero outside the image.
struct Band {
    int alo, ahi;
    bool first, last;
};

__device__ __forceinline__ float sigma_of(const DevGeom &g, int b) {
    return ((float)b - g.cB) * g.bscale;
}
__device__ __forceinline__ float tau_of(const DevGeom &g, int k) { return (float)k - g.cT; }

// Per-ray constants: Ub = sigma c + cN, Vb = sigma s + cN.
__device__ __forceinline__ void ray_base(const DevGeom &g, float sigma, float c, float s, float &Ub, float &Vb) {
    Ub = fmaf(sigma, c, g.cN);
    Vb = fmaf(sigma, s, g.cN);
}
__device__ __forceinline__ void sample_uv(float Ub, float Vb, float tau, float c, float s, float &U, float &V) {
    U = fmaf(tau, -s, Ub);
    V = fmaf(tau, c, Vb);
}

// ---------------------------------------------------------------- compensated arithmetic
// Error-free transformation (Knuth TwoSum): a + b = s + e exactly. The translation units are built
// with -ffp-contract=off so the compiler cannot fuse or reassociate these steps.
struct Comp {
    float s, e;
};
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    float bp = s - a;
    float ap = s - bp;
    e = (a - ap) + (b - bp);
}
__device__ __forceinline__ void comp_add(Comp &c, float x) {
    float s, e;
    two_sum(c.s, x, s, e);
    c.s = s;
    c.e += e;
}
__device__ __forceinline__ void comp_merge(Comp &c, const Comp &o) {
    float s, e;
    two_sum(c.s, o.s, s, e);
    c.s = s;
    c.e += e + o.e;
}
__device__ __forceinline__ float comp_value(const Comp &c) { return c.s + c.e; }
// Kahan's compensated step (4 operations): e carries the running rounding residual.
__device__ __forceinline__ void kahan_add(Comp &c, float x) {
    const float y = x + c.e;
    const float t = c.s + y;
    c.e = y - (t - c.s);
    c.s = t;
}

// Wave64 reduction of a compensated pair (cross-lane TwoSum tree).
__device__ __forceinline__ Comp wave_reduce(Comp c) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Comp o;
        o.s = __shfl_xor(c.s, off, kWave);
        o.e = __shfl_xor(c.e, off, kWave);
        comp_merge(c, o);
    }
    return c;
}

// Block reduction of a compensated pair; every thread must call it. Result valid in thread 0.
// scratch: >= 2 * (blockDim/64) floats of shared memory.
__device__ __forceinline__ Comp block_reduce(Comp c, float *scratch) {
    c = wave_reduce(c);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if (lane == 0) {
        scratch[2 * wave] = c.s;
        scratch[2 * wave + 1] = c.e;
    }
    __syncthreads();
    Comp r{0.f, 0.f};
    if (threadIdx.x == 0) {
        for (int w = 0; w < nw; ++w) comp_merge(r, Comp{scratch[2 * w], scratch[2 * w + 1]});
    }
    return r;
}

// ---------------------------------------------------------------- LDS image staging
// Stage rows band.alo..band.ahi and columns -1..n+1 of an n x n image (NC = 1 scalar image, NC = 2
// interleaved pair) into lds with row pitch n+3, zero outside the image. Eight loads per thread are
// issued before their stores so the copy is not one memory round trip per element; the row index
// uses an exact float reciprocal (idx < 2^20, pitch <= 1027).
template <int NC>
__device__ __forceinline__ void stage_band(const float *__restrict__ img, int n, const Band &band, float *lds) {
    constexpr int U = 8;
    const int pitch = n + 3;
    const int rows = band.ahi - band.alo + 1;
    const int total = rows * pitch;
    const float inv_pitch = 1.f / (float)pitch;
    for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
        float v[U][NC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            const int rr = (int)(((float)idx + 0.5f) * inv_pitch);
            const int i = band.alo + rr;
            const int l = idx - rr * pitch - 1;
            const bool in = (idx < total) && (i >= 0) && (i < n) && (l >= 0) && (l < n);
            if constexpr (NC == 1) {
                v[u][0] = in ? img[(size_t)i * n + l] : 0.f;
            } else {
                const float2 t = in ? reinterpret_cast<const float2 *>(img)[(size_t)i * n + l] : make_float2(0.f, 0.f);
                v[u][0] = t.x;
                v[u][1] = t.y;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) {
                if constexpr (NC == 1)
                    lds[idx] = v[u][0];
                else
                    reinterpret_cast<float2 *>(lds)[idx] = make_float2(v[u][0], v[u][1]);
            }
        }
    }
}

// The whole n x n image (n a multiple of 4) into lds with the layout of stage_band's single band (rows
// and columns -1..n+1, pitch n+3, zero border): 16-byte loads, U of them in flight per thread, so a
// small workgroup stages an image in a few memory round trips. Falls back to stage_band otherwise.
template <int U = 8>
__device__ __forceinline__ void stage_whole(const float *__restrict__ img, int n, const Band &band, float *lds) {
    if ((n & 3) != 0 || band.alo != -1 || band.ahi != n + 1) {
        stage_band<1>(img, n, band, lds);
        return;
    }
    const int pitch = n + 3;
    // zero border: rows -1, n, n+1 and columns -1, n, n+1 of every staged row
    for (int t = threadIdx.x; t < 3 * pitch; t += blockDim.x) {
        const int r = t / pitch, c = t - r * pitch;
        lds[(r == 0 ? 0 : n + r) * pitch + c] = 0.f;
    }
    for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) {
        const int r = t / 3, c = t - 3 * r;
        lds[(r + 1) * pitch + (c == 0 ? 0 : n + c)] = 0.f;
    }
    const int q = n >> 2;  // 16-byte groups per row
    const int total = n * q;
    const float4 *src = reinterpret_cast<const float4 *>(img);
    for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            v[u] = (idx < total) ? src[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) {
                const int r = idx / q, c = 4 * (idx - r * q);
                float *d = lds + (r + 1) * pitch + c + 1;
                d[0] = v[u].x;
                d[1] = v[u].y;
                d[2] = v[u].z;
                d[3] = v[u].w;
            }
        }
    }
}

// Two images staged interleaved (float2: first image, second image) with the same zero border.
__device__ __forceinline__ void stage_band_pair(const float *__restrict__ img0, const float *__restrict__ img1, int n,
                                                const Band &band, float *lds) {
    constexpr int U = 8;
    const int pitch = n + 3;
    const int rows = band.ahi - band.alo + 1;
    const int total = rows * pitch;
    const float inv_pitch = 1.f / (float)pitch;
    for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            const int rr = (int)(((float)idx + 0.5f) * inv_pitch);
            const int i = band.alo + rr;
            const int l = idx - rr * pitch - 1;
            const bool in = (idx < total) && (i >= 0) && (i < n) && (l >= 0) && (l < n);
            v[u] = in ? make_float2(img0[(size_t)i * n + l], img1[(size_t)i * n + l]) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) reinterpret_cast<float2 *>(lds)[idx] = v[u];
        }
    }
}

// Component `comp` of an image with `stride` floats per pixel (one plane of an interleaved image).
__device__ __forceinline__ void stage_band_strided(const float *__restrict__ img, int n, int stride, const Band &band,
                                                   float *lds) {
    constexpr int U = 8;
    const int pitch = n + 3;
    const int rows = band.ahi - band.alo + 1;
    const int total = rows * pitch;
    const float inv_pitch = 1.f / (float)pitch;
    for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            const int rr = (int)(((float)idx + 0.5f) * inv_pitch);
            const int i = band.alo + rr;
            const int l = idx - rr * pitch - 1;
            const bool in = (idx < total) && (i >= 0) && (i < n) && (l >= 0) && (l < n);
            v[u] = in ? img[((size_t)i * n + l) * stride] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) lds[idx] = v[u];
        }
    }
}

// Bilinear read at (U, V) from a staged band (NC = 1 scalar image, NC = 2 interleaved pair).
// Returns false if the sample belongs to another band (only when !SINGLE).
struct Tap {
    int off;     // LDS element offset of the (i0, l0) tap
    float fu, fv;
    bool mine;
};
// The tap row floor(Vc) lies in [alo, ahi) exactly when Vc does (integer limits), so ownership is two
// float compares; the offset (floor(Vc) - alo) pitch + floor(Uc) + 1 is formed exactly in float
// (|value| < 2^24); fract(x) = x - floor(x) exactly.
template <bool SINGLE>
__device__ __forceinline__ Tap make_tap(float U, float V, float nf, int pitch, const Band &band) {
    const float Uc = __builtin_amdgcn_fmed3f(U, -1.f, nf);
    const float Vc = __builtin_amdgcn_fmed3f(V, -1.f, nf);
    const float falo = (float)band.alo;
    Tap t;
    t.fu = __builtin_amdgcn_fractf(Uc);
    t.fv = __builtin_amdgcn_fractf(Vc);
    t.off = (int)fmaf(floorf(Vc) - falo, (float)pitch, floorf(Uc) + 1.f);
    t.mine = SINGLE ? true : (Vc >= falo && Vc < (float)band.ahi);
    return t;
}
__device__ __forceinline__ float lerp2(const float *p, int pitch, float fu, float fv) {
    const float v00 = p[0], v01 = p[1], v10 = p[pitch], v11 = p[pitch + 1];
    const float top = fmaf(fu, v01 - v00, v00);
    const float bot = fmaf(fu, v11 - v10, v10);
    return fmaf(fv, bot - top, top);
}
__device__ __forceinline__ float2 lerp2x2(const float2 *p, int pitch, float fu, float fv) {
    const float2 v00 = p[0], v01 = p[1], v10 = p[pitch], v11 = p[pitch + 1];
    float2 r;
    float top = fmaf(fu, v01.x - v00.x, v00.x);
    float bot = fmaf(fu, v11.x - v10.x, v10.x);
    r.x = fmaf(fv, bot - top, top);
    top = fmaf(fu, v01.y - v00.y, v00.y);
    bot = fmaf(fu, v11.y - v10.y, v10.y);
    r.y = fmaf(fv, bot - top, top);
    return r;
}

// k-range of a ray that may fall into `band` (conservative; membership is re-checked per sample).
__device__ __forceinline__ void band_k_range(const DevGeom &g, const Band &band, float Vb, float c, int &k0, int &k1) {
    if (band.first && band.last) {
        k0 = 0;
        k1 = g.nt - 1;
        return;
    }
    const float vlo = band.first ? -1e30f : (float)band.alo;
    const float vhi = band.last ? 1e30f : (float)band.ahi;
    if (fabsf(c) < 1e-7f) {
        // V is constant along the ray (up to the tiny slope): take the whole ray if it can touch
        const float vmin = Vb - fabsf(c) * (g.cT + 1.f) - 1.f, vmax = Vb + fabsf(c) * (g.cT + 1.f) + 1.f;
        if (vmax < vlo - 1.f || vmin > vhi + 1.f) {
            k0 = 1;
            k1 = 0;
        } else {
            k0 = 0;
            k1 = g.nt - 1;
        }
        return;
    }
    // V(k) = Vb + (k - cT) c  =>  k = (V - Vb)/c + cT
    float ka = (fmaxf(vlo, -4.f * (float)g.nt - 8.f) - Vb) / c + g.cT;
    float kb = (fminf(vhi, 4.f * (float)g.nt + 8.f) - Vb) / c + g.cT;
    float lo = fminf(ka, kb), hi = fmaxf(ka, kb);
    lo = fmaxf(lo - 2.f, 0.f);
    hi = fminf(hi + 2.f, (float)(g.nt - 1));
    k0 = (int)floorf(lo);
    k1 = (int)ceilf(hi);
}

// Bilinear read at (U, V) from a whole-image stage (rows -1..n+1, columns -1..n+1, pitch n+3):
// the clamp to [-1, n] keeps every tap inside the zero border. The tap's index floor(V) pitch +
// floor(U) is formed in float (exact: small integers) and converted once, which is cheaper than an
// integer multiply.
__device__ __forceinline__ float bilinear_whole(const float *lds, float U, float V, float nf, int pitch) {
    const float Uc = __builtin_amdgcn_fmed3f(U, -1.f, nf);
    const float Vc = __builtin_amdgcn_fmed3f(V, -1.f, nf);
    const float fu = __builtin_amdgcn_fractf(Uc);
    const float fv = __builtin_amdgcn_fractf(Vc);
    const int idx = (int)fmaf(floorf(Vc), (float)pitch, floorf(Uc));
    return lerp2(lds + idx + (pitch + 1), pitch, fu, fv);
}

// Raw buffer resource over `bytes` bytes at p (gfx9 descriptor word 3): loads take a 32-bit byte offset
// from the uniform base. Every load below is predicated to in-range offsets; elements that must read
// as zero are zeroed in registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const float *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buffer_ld(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    // the b32 load yields the raw 32-bit word: reinterpret it, do not convert it
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
// Same with a uniform (scalar) byte offset added to the per-lane one.
__device__ __forceinline__ float buffer_ld(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned uniform_off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, uniform_off, 0));
}
// 16-byte load (4 consecutive floats) at a per-lane plus a uniform byte offset.
__device__ __forceinline__ float4 buffer_ld4(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned uniform_off) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, uniform_off, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}
// The same load with the non-temporal hint, for data a launch streams once (the ray kernels' walks over
// the attenuation tensors): the lines are not kept for reuse. Measured on the paired projection of the
// 256-candidate batch: 197 against 223 us per launch. The gather, whose tiles reuse each other's
// samples through L2, keeps the plain load (4% slower with the hint).
__device__ __forceinline__ float4 buffer_ld4_stream(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned uniform_off) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, uniform_off, 2);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}
// Vector store of one float at a per-lane plus a uniform byte offset.
__device__ __forceinline__ void buffer_st(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned uniform_off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, uniform_off, 0);
}
// Vector store of 4 consecutive floats at a per-lane plus a uniform byte offset.
__device__ __forceinline__ void buffer_st4(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned uniform_off, float4 v) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 w = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, byte_off, uniform_off, 0);
}
// The same store with the non-temporal hint, for the single-stage ray kernels' streams written once per
// launch (the attenuation build's tensor, the reverse sweep's and tail's adjoint): measured 1-2% faster
// on those kernels.
__device__ __forceinline__ void buffer_st4_stream(__amdgpu_buffer_rsrc_t r, unsigned byte_off, unsigned uniform_off,
                                                  float4 v) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 w = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, byte_off, uniform_off, 2);
}
// Component q (0..3, a compile-time constant after unrolling) of v.
__device__ __forceinline__ float f4at(const float4 &v, int q) { return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w; }

// hat(x) = max(0, 1 - |x|)
__device__ __forceinline__ float hat(float x) { return fmaxf(1.f - fabsf(x), 0.f); }

}  // namespace boac
