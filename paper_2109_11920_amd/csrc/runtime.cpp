// libboac host runtime: argument validation, device scratch, launch plans (defaults + autotuner
// cache), kernel-time instrumentation, HIP-graph capture of batched evaluations, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/boac.h"
#include "gp_host.h"
#include "launch.h"

using namespace boac;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static boac_status fail(boac_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail(BOAC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));        \
    } while (0)

#define BOAC_TRY(expr)                    \
    do {                                  \
        boac_status _s = (expr);          \
        if (_s != BOAC_OK) return _s;     \
    } while (0)

// ------------------------------------------------------------------ no-allocation scratch
// File-scope device array behind boac_objective_noalloc: each device the library runs on holds its own
// copy until the process ends. In host code `scratch` names a host-side stand-in, never the device
// memory: its device address is taken once per device with hipGetSymbolAddress (noalloc_base) and only
// that address is passed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[BOAC_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static std::map<int, void *> g_noalloc_base;  // device -> device address of `scratch`

// Device address of this device's `scratch` (the device must be current); looked up once per device.
static boac_status noalloc_base(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_base.find(device);
    if (it != g_noalloc_base.end()) {
        *out = it->second;
        return BOAC_OK;
    }
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(BOAC_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
    }
    g_noalloc_base[device] = ptr;
    *out = ptr;
    return BOAC_OK;
}

// ------------------------------------------------------------------ validation (no HIP calls)
static constexpr size_t kLdsBudget = 160 * 1024 - 256;  // gfx950: 160 KiB of LDS per workgroup

// Elements per angle of an attenuation tensor stored in 4 x 8 (sample x bin) blocks.
static size_t att_slab(const boac_geom &g) {
    return (size_t)((g.n_samples + 3) / 4 * 4) * (size_t)((g.n_bins + 7) / 8 * 8);
}

// Half width, in bins, of the window of bins around a pixel's nearest bin that can hold samples of its
// bilinear support: ceil(sqrt(2) rho - 1/2), rho = n_bins / n. Below rho ~ 0.35 that is 0 (bins wider
// than ~2.8 pixels: only the nearest bin can reach the pixel); the kernels' narrowest window, one bin
// either side, then also covers it (the extra taps carry weight 0).
static int bin_half_window(const boac_geom &g) {
    const double rho = (double)g.n_bins / (double)g.n;
    return std::max(1, (int)std::ceil(std::sqrt(2.0) * rho - 0.5));
}

static boac_status check_geom(const boac_geom *g) {
    if (!g) return fail(BOAC_EINVAL, "geometry pointer is NULL");
    if (g->n < 2 || g->n > 1024) return fail(BOAC_ESHAPE, "n = %d outside [2, 1024]", g->n);
    if (g->n_angles < 2 || g->n_angles > 8192) return fail(BOAC_ESHAPE, "n_angles = %d outside [2, 8192]", g->n_angles);
    if (g->n_bins < 2 || g->n_bins > 4096) return fail(BOAC_ESHAPE, "n_bins = %d outside [2, 4096]", g->n_bins);
    if (g->n_bins > 2 * g->n) return fail(BOAC_ESHAPE, "n_bins = %d above 2 n = %d", g->n_bins, 2 * g->n);
    if (g->n_samples < 2 || g->n_samples > 1024)
        return fail(BOAC_ESHAPE, "n_samples = %d outside [2, 1024]", g->n_samples);
    if (!(g->pixel_cm > 0.f) || !std::isfinite(g->pixel_cm))
        return fail(BOAC_ESHAPE, "pixel_cm = %g must be positive and finite", (double)g->pixel_cm);
    if ((double)g->n_angles * att_slab(*g) * 4.0 >= 4294967296.0)
        return fail(BOAC_ESHAPE, "n_angles * n_bins * n_samples = %.0f samples: above 2^30 per candidate",
                    (double)g->n_angles * g->n_bins * g->n_samples);
    const int hb = bin_half_window(*g);
    if (hb > 3)
        return fail(BOAC_ESHAPE, "n_bins / n = %g gives a bin window of %d; supported 1..3", (double)g->n_bins / g->n, hb);
    if ((size_t)(g->n + 3) * 4 * 2 * 2 > kLdsBudget)
        return fail(BOAC_ESHAPE, "n = %d too large for LDS row staging", g->n);
    return BOAC_OK;
}

static boac_status check_ptr(const void *p, const char *name, bool nullable = false) {
    if (!p) return nullable ? BOAC_OK : fail(BOAC_EINVAL, "%s is NULL", name);
    if (((uintptr_t)p & 15u) != 0) return fail(BOAC_EINVAL, "%s is not 16-byte aligned", name);
    return BOAC_OK;
}

static boac_status check_count(int32_t C) {
    if (C < 1 || C > (1 << 20)) return fail(BOAC_EINVAL, "candidate count C = %d outside [1, 2^20]", C);
    return BOAC_OK;
}

// ------------------------------------------------------------------ context
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct PendingTiming {
    int kind;
    hipEvent_t e0, e1;
    double bytes;
};

struct Plan {
    RayCfg ray1, ray2;  // ray kernels staging one image / an interleaved pair
    Bands bands1, bands2;
    BackCfg back;
};

// Bump allocation from a fixed device region (the no-allocation entry point): named buffers of one call
// are carved in request order, and a name requested again gets its earlier range when that is large
// enough. No HIP call is made.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    std::map<std::string, std::pair<size_t, size_t>> named;  // name -> (offset, bytes)
};

struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t scratch_gen = 0;  // scratch generation the graph's kernels were captured against
    void *aux = nullptr;       // persistent batches: the executor's state (error word at index 1)
};

struct boac_ctx {
    int device = 0;
    int n_cu = 256;
    std::map<std::string, DevBuf> bufs;
    std::map<std::vector<int>, float2 *> trig;
    std::map<std::vector<int>, int4 *> rects;
    std::map<std::string, std::vector<int>> tune;
    bool profiling = false;
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> free_events;
    int64_t stat_count[BOAC_K_COUNT] = {};
    double stat_ms[BOAC_K_COUNT] = {};
    double stat_bytes[BOAC_K_COUNT] = {};
    std::vector<GraphEntry> graphs;
    bool capturing = false;
    // bumped whenever a scratch buffer is freed and reallocated: a graph captured under an older
    // generation may hold pointers to freed memory and is never replayed
    uint64_t scratch_gen = 0;
    int64_t graph_captures = 0, graph_replays = 0;
    std::string ns;                    // scratch namespace of the work being emitted (batch lane)
    void *noalloc = nullptr;           // device address of this device's no-allocation scratch
    Arena *arena = nullptr;            // set during a no-allocation call: scratch and tables come from it
    hipStream_t arena_stream = nullptr;
    std::map<std::vector<int>, std::vector<int4>> host_rects;   // host copies uploaded into an arena
    std::map<int, std::vector<float2>> host_trig;
    // batch execution: 0 = concurrent stream lanes captured in a graph, 1 = one persistent launch
    int batch_mode = 0;
    long long spin_limit = 0;
    bool persist_plans = false;        // plans for the persistent executor (1024-thread ray workgroups)
    bool recording = false;            // launches are being recorded as tasks
    std::vector<hipStream_t> lanes;    // concurrent streams of the batch scheduler
    std::vector<hipEvent_t> lane_done;
    hipEvent_t fork = nullptr;
};

static boac_status arena_take(Arena &a, const std::string &name, size_t bytes, void **out) {
    auto it = a.named.find(name);
    if (it != a.named.end() && it->second.second >= bytes) {
        *out = a.base + it->second.first;
        return BOAC_OK;
    }
    const size_t off = (a.used + 255) & ~(size_t)255;
    if (off + bytes > a.cap)
        return fail(BOAC_ENOMEM, "scratch '%s' (%zu bytes at offset %zu) exceeds the %zu-byte no-allocation scratch",
                    name.c_str(), bytes, off, a.cap);
    a.used = off + bytes;
    a.named[name] = {off, bytes};
    *out = a.base + off;
    return BOAC_OK;
}

static boac_status ensure(boac_ctx *ctx, const char *name, size_t bytes, void **out) {
    if (ctx->arena) return arena_take(*ctx->arena, ctx->ns + name, bytes, out);
    DevBuf &b = ctx->bufs[ctx->ns + name];
    if (b.bytes < bytes) {
        if (ctx->capturing) return fail(BOAC_EDEVICE, "scratch '%s' must grow during graph capture", name);
        if (b.p) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(b.p));
            b.p = nullptr;
            b.bytes = 0;
        }
        size_t want = bytes + bytes / 8;
        want = (want + (2u << 20) - 1) & ~(size_t)((2u << 20) - 1);
        hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            b.p = nullptr;
            (void)hipGetLastError();
            return fail(BOAC_ENOMEM, "scratch '%s': hipMalloc(%zu) failed: %s", name, want, hipGetErrorString(e));
        }
        b.bytes = want;
        ++ctx->scratch_gen;
    }
    *out = b.p;
    return BOAC_OK;
}

template <typename T>
static boac_status ensure_t(boac_ctx *ctx, const char *name, size_t count, T **out) {
    void *p = nullptr;
    BOAC_TRY(ensure(ctx, name, count * sizeof(T), &p));
    *out = (T *)p;
    return BOAC_OK;
}

static boac_status host_trig(int na, std::vector<float2> &h);

// cos/sin of 2 pi a / na in double, exact at multiples of 90 degrees, rounded to float
static boac_status trig_table(boac_ctx *ctx, int na, const float2 **out) {
    if (ctx->arena) {
        // host copy kept in the context (the source of an asynchronous upload must outlive it)
        std::vector<float2> &h = ctx->host_trig[na];
        if (h.empty()) BOAC_TRY(host_trig(na, h));
        void *d = nullptr;
        BOAC_TRY(arena_take(*ctx->arena, "#trig", sizeof(float2) * na, &d));
        HIP_TRY(hipMemcpyAsync(d, h.data(), sizeof(float2) * na, hipMemcpyHostToDevice, ctx->arena_stream));
        *out = (const float2 *)d;
        return BOAC_OK;
    }
    std::vector<int> key{na};
    auto it = ctx->trig.find(key);
    if (it != ctx->trig.end()) {
        *out = it->second;
        return BOAC_OK;
    }
    if (ctx->capturing) return fail(BOAC_EDEVICE, "trig table upload during graph capture");
    std::vector<float2> h;
    BOAC_TRY(host_trig(na, h));
    float2 *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(float2) * na));
    HIP_TRY(hipMemcpy(d, h.data(), sizeof(float2) * na, hipMemcpyHostToDevice));
    ctx->trig[key] = d;
    *out = d;
    return BOAC_OK;
}

static boac_status host_trig(int na, std::vector<float2> &h) {
    h.resize(na);
    for (int a = 0; a < na; ++a) {
        // reduce to the first quadrant on integers so that 0/90/180/270 deg are exact
        const long num = 4L * a;  // angle = 2 pi a / na = (pi/2) * (4a / na)
        const long quad = num / na;
        const long rem = num - quad * na;
        const double frac = (double)rem / (double)na * (M_PI / 2.0);
        double c = std::cos(frac), s = std::sin(frac);
        if (rem == 0) {
            c = 1.0;
            s = 0.0;
        }
        double cc, ss;
        switch (quad & 3) {
            case 0: cc = c; ss = s; break;
            case 1: cc = -s; ss = c; break;
            case 2: cc = -c; ss = -s; break;
            default: cc = s; ss = -c; break;
        }
        h[a] = make_float2((float)cc, (float)ss);
    }
    return BOAC_OK;
}

// Footprint rectangles of every (pixel tile, angle) of the backprojection: bins and samples whose
// window can reach a pixel of the tile, with one sample of margin on every side (the kernel's window
// centres, computed in FP32, stay inside). Computed in double from the same FP32 angle table.
// nah: angles held (the first nah of the n_angles, the table's stride per tile).
static boac_status rect_table(boac_ctx *ctx, const boac_geom &g, BackCfg *bc, int nah) {
    std::vector<int> key{g.n, g.n_angles, g.n_bins, g.n_samples, bc->tw, bc->th, bc->hb, bc->slid, nah};
    const size_t nent = (size_t)bc->tiles_x * bc->tiles_y * nah;
    // one allocation: the int4 rectangles, then (slid blocks) their float forms and the angle table
    auto point = [&](int4 *d) {
        bc->rects = d;
        bc->rectf = bc->slid ? reinterpret_cast<const float4 *>(d + nent) : nullptr;
        bc->angt = bc->slid ? bc->rectf + 2 * nent : nullptr;
    };
    auto it = ctx->rects.find(key);
    if (!ctx->arena && it != ctx->rects.end()) {
        point(it->second);
        return BOAC_OK;
    }
    if (ctx->arena) {
        auto hit = ctx->host_rects.find(key);
        if (hit != ctx->host_rects.end()) {
            void *d = nullptr;
            BOAC_TRY(arena_take(*ctx->arena, "#rects", sizeof(int4) * hit->second.size(), &d));
            HIP_TRY(hipMemcpyAsync(d, hit->second.data(), sizeof(int4) * hit->second.size(), hipMemcpyHostToDevice,
                                   ctx->arena_stream));
            point((int4 *)d);
            return BOAC_OK;
        }
    }
    if (ctx->capturing) return fail(BOAC_EDEVICE, "rectangle table upload during graph capture");
    std::vector<float2> trig;
    BOAC_TRY(host_trig(g.n_angles, trig));
    const double cN = 0.5 * (g.n - 1), cB = 0.5 * (g.n_bins - 1), cT = 0.5 * (g.n_samples - 1);
    const double inv_bscale = (double)g.n_bins / (double)g.n;
    const int ntiles = bc->tiles_x * bc->tiles_y;
    const int wb_cap = std::min(bc->wbmax, 64);
    const int wk_cap = bc->wkmax;
    std::vector<int4> h((size_t)ntiles * nah);
    for (int t = 0; t < ntiles; ++t) {
        const int ty = t / bc->tiles_x, tx = t % bc->tiles_x;
        const int l0 = tx * bc->tw, i0 = ty * bc->th;
        const double xl[2] = {l0 - cN, std::min(l0 + bc->tw - 1, g.n - 1) - cN};
        const double yi[2] = {i0 - cN, std::min(i0 + bc->th - 1, g.n - 1) - cN};
        for (int a = 0; a < nah; ++a) {
            const double c = trig[a].x, s = trig[a].y;
            double Smin = 1e300, Smax = -1e300, Tmin = 1e300, Tmax = -1e300;
            for (double x : xl)
                for (double y : yi) {
                    const double S = (x * c + y * s) * inv_bscale + cB;
                    const double T = (-x * s + y * c) + cT;
                    Smin = std::min(Smin, S);
                    Smax = std::max(Smax, S);
                    Tmin = std::min(Tmin, T);
                    Tmax = std::max(Tmax, T);
                }
            const int b_lo = (int)std::floor(Smin + 0.5) - bc->hb - 1;
            const int b_hi = (int)std::floor(Smax + 0.5) + bc->hb + 1;
            const int k_lo = (int)std::floor(Tmin + 0.5) - 2;
            const int k_hi = (int)std::floor(Tmax + 0.5) + 2;
            const int wb = b_hi - b_lo + 1, wk = k_hi - k_lo + 1;
            if (bc->slid) {
                // slide the fixed block inside the sinogram; it still holds the clipped rectangle
                if (wb > kSlidBlock || wk > kSlidBlock)
                    return fail(BOAC_EDEVICE, "internal: footprint %dx%d exceeds the %d-block", wb, wk, kSlidBlock);
                const int b0 = std::min(std::max(b_lo, 0), g.n_bins - kSlidBlock);
                int k0 = std::min(std::max(k_lo, 0), g.n_samples - kSlidBlock);
                if (bc->slid == 2) {
                    // column-group variant: the first sample row a multiple of 4 (n_samples is one, so
                    // the block still ends inside the sinogram); it must still reach the clipped
                    // footprint's last row
                    k0 &= ~3;
                    if (std::min(k_hi, g.n_samples - 1) >= k0 + kSlidBlock)
                        return fail(BOAC_EDEVICE, "internal: aligned footprint exceeds the %d-block", kSlidBlock);
                }
                // image position of sample (b0, k0), relative to the centre of the tile's support box
                const double sig = ((double)b0 - cB) * ((double)g.n / (double)g.n_bins), tau = (double)k0 - cT;
                const double u = sig * c - tau * s - 0.5 * (xl[0] + xl[1]);
                const double v = sig * s + tau * c - 0.5 * (yi[0] + yi[1]);
                float uf = (float)u, vf = (float)v;
                int ub, vb;
                std::memcpy(&ub, &uf, 4);
                std::memcpy(&vb, &vf, 4);
                h[(size_t)t * nah + a] = make_int4(b0, k0, ub, vb);
                continue;
            }
            const int slots = (bc->hb > 1) ? 8 : (bc->tw == 16 && bc->th == 16) ? 4 : (bc->tw == 32 && bc->th == 16) ? 8 : 11;
            if (wb > wb_cap || wk > wk_cap || wb * wk > 256 * slots)
                return fail(BOAC_EDEVICE, "internal: footprint %dx%d exceeds the staged bound %dx%d", wb, wk, wb_cap,
                            wk_cap);
            h[(size_t)t * nah + a] = make_int4(b_lo, k_lo, wb, wk);
        }
    }
    if (bc->slid) {
        // float forms of the block origins and per-angle trigonometry for the slid-block gathers, each
        // value the FP32 operation the kernel would otherwise repeat per angle (same rounding)
        const float bscale = (float)g.n / (float)g.n_bins;
        const float inv_bscale = 1.f / bscale;
        for (size_t e = 0; e < nent; ++e) {
            const float fb1 = (float)(h[e].x + 1), fk1 = (float)(h[e].y + 1);
            const float f[8] = {fb1, fk1, fb1 + (float)(kSlidBlock - 3), fk1 + (float)(kSlidBlock - 3),
                                fk1 * (float)kSlidPitch + fb1, 0.f, 0.f, 0.f};
            int4 w[2];
            std::memcpy(w, f, sizeof(f));
            h.push_back(w[0]);
            h.push_back(w[1]);
        }
        for (int a = 0; a < nah; ++a) {
            const float c = trig[a].x, s = trig[a].y;
            const float f[8] = {c, s, c * bscale, s * bscale, c * inv_bscale, s * inv_bscale, 0.f, 0.f};
            int4 w[2];
            std::memcpy(w, f, sizeof(f));
            h.push_back(w[0]);
            h.push_back(w[1]);
        }
    }
    if (ctx->arena) {
        // host copy kept in the context (the source of an asynchronous upload must outlive it)
        std::vector<int4> &keep = ctx->host_rects[key];
        keep = std::move(h);
        void *d = nullptr;
        BOAC_TRY(arena_take(*ctx->arena, "#rects", sizeof(int4) * keep.size(), &d));
        HIP_TRY(hipMemcpyAsync(d, keep.data(), sizeof(int4) * keep.size(), hipMemcpyHostToDevice, ctx->arena_stream));
        point((int4 *)d);
        return BOAC_OK;
    }
    int4 *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(int4) * h.size()));
    HIP_TRY(hipMemcpy(d, h.data(), sizeof(int4) * h.size(), hipMemcpyHostToDevice));
    ctx->rects[key] = d;
    point(d);
    return BOAC_OK;
}

static boac_status dev_geom(boac_ctx *ctx, const boac_geom &g, DevGeom *dg) {
    dg->n = g.n;
    dg->na = g.n_angles;
    dg->nah = g.n_angles;
    dg->nb = g.n_bins;
    dg->nt = g.n_samples;
    dg->dx = g.pixel_cm;
    dg->cN = 0.5f * (float)(g.n - 1);
    dg->cB = 0.5f * (float)(g.n_bins - 1);
    dg->cT = 0.5f * (float)(g.n_samples - 1);
    dg->bscale = (float)g.n / (float)g.n_bins;
    dg->nb8 = (g.n_bins + 7) / 8;
    dg->slab = (int)att_slab(g);
    return trig_table(ctx, g.n_angles, &dg->trig);
}

// ------------------------------------------------------------------ plans
// Row bands needed to stage an n x n image of `comps` float components (columns -1..n+1) within
// the LDS budget: 1 when the whole image fits.
static constexpr int band_count(int n, int comps) {
    const size_t pitch_bytes = (size_t)(n + 3) * 4 * comps;
    if (pitch_bytes * (n + 3) <= kLdsBudget) return 1;
    const int rows = (int)(kLdsBudget / pitch_bytes) - 1;  // assigned rows per band (staged = rows + 1)
    return (n + 2 + rows - 1) / rows;                     // assigned range [-1, n+1)
}
static void make_bands(int n, int comps, RayCfg *rc, Bands *bands) {
    const size_t pitch_bytes = (size_t)(n + 3) * 4 * comps;
    const int count = band_count(n, comps);
    const int span = n + 2;  // assigned range [-1, n+1)
    // the same number of bands with rows spread evenly: the last band is not empty and no band
    // stages more rows than band_count allowed for
    bands->count = count;
    bands->rows = (span + count - 1) / count;
    rc->single = count == 1;
    rc->lds = pitch_bytes * (size_t)(bands->rows + 1);
}

static std::string shape_key(const char *kind, const boac_geom &g, int C, int extra) {
    char buf[160];
    snprintf(buf, sizeof buf, "%s:%dx%dx%dx%d:%d:%d", kind, g.n, g.n_angles, g.n_bins, g.n_samples, C, extra);
    return buf;
}

// Candidate counts up to this one get the few-candidate plans (ray-split projection, angle-split
// gather): the unbatched evaluation and small calls, where a plan for many candidates leaves CUs idle.
constexpr int kFewCand = 8;

// nah: angles whose rays the kernels walk (n_angles, or half of them with opposed-ray pairing).
static void ray_plan(boac_ctx *ctx, const boac_geom &g, int C, int comps, RayCfg *rc, Bands *bands, int nah) {
    make_bands(g.n, comps, rc, bands);
    const int nrays = nah * g.n_bins;
    // the paired forward projection where both images fit one stage (default on)
    const bool pair_fits = comps == 1 && rc->single && 2 * rc->lds <= kLdsBudget && C >= 2;
    rc->pair = pair_fits;
    // default: 1024-thread workgroups (the image stage is shared by more waves, and a stage that fills
    // the LDS still gives 16 waves per CU), one resident per CU; the rays per thread that minimise
    // (rounds of workgroups over the CUs) x (rays per thread + a fixed cost per workgroup: the image
    // stage, the first loads and the epilogue, about 0.6 of a ray pass as measured on the paired
    // projection at 96-192 candidates). A paired projection has one workgroup per chunk and candidate
    // pair. Where even one ray per thread leaves CUs without a workgroup, smaller workgroups.
    const long groups = pair_fits ? (C + 1) / 2 : C;
    rc->block = 1024;
    rc->rpt = 1;
    double best = 0.0;
    for (int rpt : {4, 2, 1}) {
        const long wgs = (long)((nrays + 1024 * rpt - 1) / (1024 * rpt)) * groups;
        const double cost = (double)((wgs + ctx->n_cu - 1) / ctx->n_cu) * (rpt + 0.6);
        if (rpt == 4 || cost < best) {
            best = cost;
            rc->rpt = rpt;
        }
    }
    if ((long)((nrays + 1023) / 1024) * groups < ctx->n_cu) {
        rc->rpt = 1;
        rc->block = ((long)((nrays + 511) / 512) * groups >= ctx->n_cu) ? 512 : 256;
    }
    // plan cache entry: [threads per workgroup, rays per thread, paired forward projection]
    auto it = ctx->tune.find(shape_key("ray", g, C, comps));
    if (it != ctx->tune.end() && it->second.size() >= 2) {
        const int blk = it->second[0], rpt = it->second[1];
        if (blk >= 64 && blk <= 1024 && blk % 64 == 0 && rpt >= 1 && rpt <= 4) {
            rc->block = blk;
            rc->rpt = rpt;
        }
        if (it->second.size() >= 3) rc->pair = pair_fits && it->second[2] != 0;
    }
    rc->chunks = (nrays + rc->block * rc->rpt - 1) / (rc->block * rc->rpt);
    // few candidates (at most kFewCand): the projection splits each ray over 8 lanes when one thread per
    // ray would not give every CU a workgroup (single-stage images, up to 256 samples; each 32-ray
    // workgroup stages the whole image, which pays only while the GPU would otherwise idle;
    // BOAC_FWD_SPLIT=0 turns it off)
    rc->split_chunks = 0;
    const char *es = std::getenv("BOAC_FWD_SPLIT");
    const bool split_on = !(es && es[0] == '0');
    if (split_on && C <= kFewCand && comps == 1 && rc->single && g.n_samples <= 256 &&
        (long)rc->chunks * C < ctx->n_cu)
        rc->split_chunks = (nrays + 31) / 32;
    // attenuation build: the scan of each ray spread over 8 lanes (single stage, up to 256 samples;
    // BOAC_ATT_SCAN=0: one thread per ray); 1024-thread workgroups when there are rays enough, and as
    // many rays per lane group as still give every CU two workgroups (at most 32)
    rc->scan_block = rc->scan_passes = rc->scan_chunks = 0;
    const char *ea = std::getenv("BOAC_ATT_SCAN");
    if (!(ea && ea[0] == '0') && comps == 1 && rc->single && g.n_samples <= 256) {
        rc->scan_block = ((long)nrays * C >= 64L * ctx->n_cu * 128) ? 1024 : 256;
        const int rpp = rc->scan_block / 8;
        const long total = (nrays + rpp - 1) / rpp;
        rc->scan_passes = (int)std::min<long>(32, std::max<long>(1, total * C / (2L * ctx->n_cu)));
        rc->scan_chunks = (int)((total + rc->scan_passes - 1) / rc->scan_passes);
    }
    if (ctx->persist_plans) {
        // the persistent executor runs ray kernels as 1024-thread items: the most rays per thread that
        // still give every CU an item, no ray split
        rc->block = 1024;
        rc->rpt = 1;
        for (int rpt : {4, 2, 1})
            if ((long)((nrays + 1024 * rpt - 1) / (1024 * rpt)) * C >= ctx->n_cu || rpt == 1) {
                rc->rpt = rpt;
                break;
            }
        rc->chunks = (nrays + 1024 * rc->rpt - 1) / (1024 * rc->rpt);
        rc->split_chunks = 0;
        if (rc->scan_passes > 0) {
            const long total = (nrays + 127) / 128;
            rc->scan_block = 1024;
            rc->scan_passes = (int)std::min<long>(32, std::max<long>(1, total * C / (long)ctx->n_cu));
            rc->scan_chunks = (int)((total + rc->scan_passes - 1) / rc->scan_passes);
        }
    }
}

static void back_fill(const boac_geom &g, BackCfg *bc) {
    bc->ppt = bc->tw * bc->th / 256;
    bc->hb = bin_half_window(g);
    const double diag = std::sqrt((double)(bc->tw - 1) * (bc->tw - 1) + (double)(bc->th - 1) * (bc->th - 1));
    const double rho = (double)g.n_bins / g.n;
    bc->wbmax = (int)std::ceil(diag * rho) + 2 * bc->hb + 6;
    bc->wkmax = (int)std::ceil(diag) + 8;
    bc->tiles_x = (g.n + bc->tw - 1) / bc->tw;
    bc->tiles_y = (g.n + bc->th - 1) / bc->th;
    // slid blocks: the staged block, then two [bin][candidate] ray-weight tables
    bc->lds = bc->slid ? (size_t)bc->cg * (kSlidBlock * kSlidPitch + 2 * kSlidBlock) * sizeof(float)
                       : (size_t)bc->cg * (bc->wbmax * bc->wkmax + bc->wbmax) * sizeof(float);
}

// rows of the footprint rectangle the back kernel can stage per angle (4 waves x rows per wave)
static int back_stage_rows(const BackCfg &b) {
    if (b.tw == 16 && b.th == 16) return 4 * 8;
    if (b.tw == 32 && b.th == 16) return 4 * 11;
    return 4 * 14;
}

static bool back_cfg_ok(const BackCfg &b) {
    if (b.slid) return false;  // checked by slid_ok, which needs the geometry
    const bool tile = (b.tw == 16 && b.th == 16) || (b.tw == 32 && b.th == 16) || (b.tw == 32 && b.th == 32);
    const bool cg = b.cg == 1 || b.cg == 2 || b.cg == 4 || (b.cg == 8 && b.tw == 16 && b.th == 16);
    if (!tile || !cg || b.lds > kLdsBudget) return false;
    if (b.wbmax > 64 || b.wkmax > back_stage_rows(b)) return false;
    // the kernel's per-thread prefetch slots cover the fixed-pitch rectangle
    const int slots = (b.hb > 1) ? 8 : (b.tw == 16 && b.th == 16) ? 4 : (b.tw == 32 && b.th == 16) ? 8 : 11;
    if (b.wbmax * b.wkmax > 256 * slots) return false;
    if (b.hb > 1) return b.tw == 16 && b.th == 16 && b.cg == 1;
    return b.hb == 1;
}

// The slid-block kernel: 16 x 16 tiles, one-bin half window, a footprint within the 32 x 32 block, a
// sinogram at least one block wide and tall, and 32-bit buffer offsets that cannot wrap (the kernel's
// largest offset is below 2 cg bytes-per-candidate).
static bool slid_ok(const boac_geom &g, const BackCfg &b) {
    if (!(b.slid == 1 || b.slid == 2) || b.tw != 16 || b.th != 16 || b.hb != 1) return false;
    if (b.slid == 2 && g.n_samples % 4 != 0) return false;
    if (!(b.cg == 1 || b.cg == 2 || b.cg == 4 || b.cg == 8) || b.lds > kLdsBudget) return false;
    if (b.wbmax > kSlidBlock || b.wkmax > kSlidBlock) return false;
    if (g.n_bins < kSlidBlock || g.n_samples < kSlidBlock) return false;
    const double att_bytes = 4.0 * g.n_angles * (double)att_slab(g);
    return 2.0 * b.cg * att_bytes < 4294967296.0;
}

static bool plan_ok(const boac_geom &g, const BackCfg &b) { return b.slid ? slid_ok(g, b) : back_cfg_ok(b); }

// nah: angles the gather walks (n_angles, or half of them with opposed-ray pairing)
static void back_plan(boac_ctx *ctx, const boac_geom &g, int C, BackCfg *bc, int nah) {
    // preference order: the slid-block kernel where it applies, then the general one; big candidate
    // groups amortise the footprint staging and the window weights, and the choice falls back while
    // the grid would not fill the GPU twice over
    static const int prefs[][4] = {{16, 16, 4, 2}, {16, 16, 2, 2}, {16, 16, 1, 2},
                                   {16, 16, 4, 1}, {16, 16, 2, 1}, {16, 16, 1, 1},
                                   {16, 16, 4, 0}, {16, 16, 2, 0}, {16, 16, 1, 0}};
    const long target = 2L * ctx->n_cu;
    bool set = false;
    int slid_seen = -1;
    for (const auto &pf : prefs) {
        if (set && pf[3] != slid_seen) break;  // stay within the first kernel family that applies
        BackCfg t{};
        t.tw = pf[0];
        t.th = pf[1];
        t.cg = pf[2];
        t.slid = pf[3];
        t.xcd_remap = 1;
        back_fill(g, &t);
        if (!plan_ok(g, t)) continue;
        *bc = t;
        set = true;
        slid_seen = t.slid;
        if (C >= t.cg && (long)t.tiles_x * t.tiles_y * ((C + t.cg - 1) / t.cg) >= target) break;
    }
    if (!set || bin_half_window(g) > 1) {
        BackCfg t{};
        t.tw = 16;
        t.th = 16;
        t.cg = 1;
        t.xcd_remap = 1;
        back_fill(g, &t);
        *bc = t;
    }
    // plan cache entry: [tile width, tile height, candidates per workgroup, XCD remap, slid block
    // (0: general kernel, 1: slot staging, 2: column-group staging)]
    auto it = ctx->tune.find(shape_key("back", g, C, 0));
    if (it != ctx->tune.end() && it->second.size() >= 3) {
        BackCfg t{};
        t.tw = it->second[0];
        t.th = it->second[1];
        t.cg = it->second[2];
        t.xcd_remap = it->second.size() >= 4 ? (it->second[3] != 0) : 1;
        t.slid = it->second.size() >= 5 ? it->second[4] : 0;
        back_fill(g, &t);
        if (plan_ok(g, t)) *bc = t;
    }
    // few candidates (at most kFewCand): the column-group gather splits the angles in whole 8-angle
    // blocks over more workgroups (a second pass adds the blocks in order) while the grid would not fill
    // the GPU twice over (BOAC_GATHER_SPLIT=0 turns it off)
    bc->asplit = 1;
    if (ctx->persist_plans && bc->slid == 2 && bc->cg > 4) {
        bc->cg = 4;  // the persistent executor runs one to four candidates per gather workgroup
        back_fill(g, bc);
    }
    const char *eg = std::getenv("BOAC_GATHER_SPLIT");
    if (bc->slid == 2 && C <= kFewCand && !ctx->persist_plans && !(eg && eg[0] == '0')) {
        const long wgs = (long)bc->tiles_x * bc->tiles_y * ((C + bc->cg - 1) / bc->cg);
        const int nblk = (nah + 7) / 8;
        if (wgs < 2L * ctx->n_cu)
            bc->asplit = (int)std::min<long>(nblk, (2L * ctx->n_cu + wgs - 1) / wgs);
    }
}

static boac_status make_plan(boac_ctx *ctx, const boac_geom &g, int C, Plan *p, int nah = -1) {
    if (nah < 0) nah = g.n_angles;
    ray_plan(ctx, g, C, 1, &p->ray1, &p->bands1, nah);
    ray_plan(ctx, g, C, 2, &p->ray2, &p->bands2, nah);
    back_plan(ctx, g, C, &p->back, nah);
    return rect_table(ctx, g, &p->back, nah);
}

// ------------------------------------------------------------------ instrumentation
static hipEvent_t take_event(boac_ctx *ctx) {
    if (!ctx->free_events.empty()) {
        hipEvent_t e = ctx->free_events.back();
        ctx->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename F>
static boac_status timed(boac_ctx *ctx, int kind, double bytes, hipStream_t st, F &&launch) {
    const bool t = ctx->profiling && !ctx->capturing && !ctx->arena && !ctx->recording;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (t) {
        e0 = take_event(ctx);
        e1 = take_event(ctx);
        if (e0 && e1) HIP_TRY(hipEventRecord(e0, st));
    }
    hipError_t e = launch();
    if (e != hipSuccess) return fail(BOAC_EDEVICE, "kernel launch (kind %d) failed: %s", kind, hipGetErrorString(e));
    if (t && e0 && e1) {
        HIP_TRY(hipEventRecord(e1, st));
        ctx->pending.push_back(PendingTiming{kind, e0, e1, bytes});
    }
    return BOAC_OK;
}

static boac_status drain_timings(boac_ctx *ctx) {
    for (auto &p : ctx->pending) {
        HIP_TRY(hipEventSynchronize(p.e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.e0, p.e1));
        ctx->stat_count[p.kind] += 1;
        ctx->stat_ms[p.kind] += ms;
        ctx->stat_bytes[p.kind] += p.bytes;
        ctx->free_events.push_back(p.e0);
        ctx->free_events.push_back(p.e1);
    }
    ctx->pending.clear();
    return BOAC_OK;
}

// ------------------------------------------------------------------ evaluation pipeline
struct Sizes {
    size_t I, Y, V;  // elements per candidate: image, sinogram, attenuation tensor (algorithmic)
    size_t VS;       // attenuation tensor stride per candidate (4 x 8-block slabs, padded)
    size_t E;        // opposed-ray pairing: exp(-T) per held ray (0 without pairing)
};
// nah: angles the attenuation tensor holds (n_angles, or n_angles / 2 with opposed-ray pairing)
static Sizes sizes_of(const boac_geom &g, int nah = -1) {
    if (nah < 0) nah = g.n_angles;
    return Sizes{(size_t)g.n * g.n, (size_t)g.n_angles * g.n_bins, (size_t)nah * g.n_bins * g.n_samples,
                 (size_t)nah * att_slab(g), nah < g.n_angles ? (size_t)nah * g.n_bins : 0};
}

// Opposed-ray pairing (the attenuation tensor for half the angles plus exp(-T) per ray, both rays of a
// line from one pass) applies to an even angle count with the column-group gather;
// BOAC_OPPOSED_RAYS=0 turns it off.
static bool pairing_enabled() {
    const char *e = std::getenv("BOAC_OPPOSED_RAYS");
    return !(e && e[0] == '0');
}

// The plan switches read from the environment (each on unless set to 0), one bit each: part of a
// captured batch graph's key, so that a graph is not replayed under other switches.
static uint64_t plan_switch_bits() {
    uint64_t bits = 0;
    int i = 0;
    for (const char *name : {"BOAC_OPPOSED_RAYS", "BOAC_FWD_SPLIT", "BOAC_ATT_SCAN", "BOAC_GATHER_SPLIT"}) {
        const char *e = std::getenv(name);
        if (e && e[0] == '0') bits |= 1ull << i;
        ++i;
    }
    return bits;
}

// Launch geometry, plan and sizes of one slice for the attenuation-weighted paths (projection,
// backprojection, MLEM, objective); with allow_pairing, opposed-ray pairing where it applies.
static boac_status plan_slice(boac_ctx *ctx, const boac_geom &g, int C, bool allow_pairing, DevGeom *dg, Plan *p,
                              Sizes *z) {
    BOAC_TRY(dev_geom(ctx, g, dg));
    *z = sizes_of(g);
    BOAC_TRY(make_plan(ctx, g, C, p));
    if (allow_pairing && pairing_enabled() && g.n_angles % 2 == 0 && p->back.slid == 2) {
        const int nah = g.n_angles / 2;
        dg->nah = nah;
        *z = sizes_of(g, nah);
        BOAC_TRY(make_plan(ctx, g, C, p, nah));
        if (p->back.slid != 2) return fail(BOAC_EDEVICE, "internal: paired plan changed family");
    }
    return BOAC_OK;
}

// Bytes models (algorithmic HBM traffic per launch) used by the instrumentation.
static double bytes_att(const Sizes &z, int C) { return 4.0 * C * (double)(z.I + z.V + z.E); }
static double bytes_fwd(const Sizes &z, int C) { return 4.0 * C * (double)(z.V + z.E + z.I + 2 * z.Y); }
static double bytes_back(const Sizes &z, int C, int mode) {
    double per = (double)z.V + z.E + z.I;  // att (and exp(-T)) read + image written
    if (mode == BACK_PLAIN || mode == BACK_MLEM || mode == BACK_ADJ) per += z.Y;
    if (mode == BACK_MLEM) per += 2.0 * z.I;
    if (mode == BACK_ADJ) per += z.I;
    if (mode == BACK_FIELD) per += 0.0;
    return 4.0 * C * per;
}

// E: exp(-T) per held ray with opposed-ray pairing (z.E > 0), else null
static boac_status run_att(boac_ctx *ctx, const DevGeom &dg, const Plan &p, const Sizes &z, const float *mu,
                           float *att, int C, hipStream_t st, float *E = nullptr) {
    return timed(ctx, BOAC_K_ATT, bytes_att(z, C), st,
                 [&] { return launch_att(dg, p.ray1, p.bands1, mu, att, z.I, z.VS, E, z.E, C, st); });
}

static boac_status run_fwd(boac_ctx *ctx, int mode, const DevGeom &dg, const Plan &p, const Sizes &z,
                           const FwdArgs &a, int C, hipStream_t st) {
    return timed(ctx, BOAC_K_FWD, bytes_fwd(z, C), st,
                 [&] { return launch_fwd(mode, dg, p.ray1, p.bands1, a, C, st); });
}

static boac_status run_back(boac_ctx *ctx, int mode, const DevGeom &dg, const Plan &p, const Sizes &z,
                            const BackArgs &a, hipStream_t st) {
    BackArgs b = a;
    double bytes = bytes_back(z, a.C, mode);
    if (p.back.asplit > 1) {
        // angle split: one partial image per 8-angle block, written by the gather, read by the combine pass
        const size_t nblk = (size_t)(dg.nah + 7) / 8;
        BOAC_TRY(ensure_t(ctx, "blk", nblk * a.C * z.I, &b.blk_out));
        bytes += 8.0 * nblk * a.C * z.I;
    }
    return timed(ctx, BOAC_K_BACK, bytes, st, [&] { return launch_back(mode, dg, p.back, b, st); });
}

static FwdArgs fwd_args(const Sizes &z, const float *att, const float *img, const float *meas,
                        const float *E = nullptr) {
    FwdArgs a{};
    a.att = att;
    a.E = E;
    a.e_cs = z.E;
    a.img = img;
    a.meas = meas;
    a.att_cs = z.VS;
    a.img_cs = z.I;
    a.sino_cs = z.Y;
    a.img_comps = 1;
    return a;
}
static BackArgs back_args(const Sizes &z, const float *att, const float *zz, float *out, int C,
                          const float *E = nullptr) {
    BackArgs a{};
    a.att = att;
    a.E = E;
    a.e_cs = z.E;
    a.z = zz;
    a.out = out;
    a.att_cs = z.VS;
    a.sino_cs = z.Y;
    a.img_cs = z.I;
    a.C = C;
    return a;
}

// Maximum candidates whose attenuation tensors are resident at once (device scratch bound).
static int cand_chunk(const Sizes &z, int C, int tensors) {
    const double budget = 48.0 * (1ull << 30);  // of 288 GB HBM
    const double per = 4.0 * (double)z.VS * tensors + 64.0 * (double)z.I;
    int m = (int)std::max(1.0, std::floor(budget / per));
    return std::min(m, C);
}

// Candidates per chunk of a forward evaluation that fit the no-allocation scratch: an upper bound of
// the per-candidate buffers (mu, att, exp(-T), s, two images, the ratio sinogram, one partial per ray
// chunk of the smallest plan) against what the fixed buffers (tables, status, reductions) leave.
// 0 when not even one candidate fits.
static int arena_chunk(const boac_geom &g, int C, size_t cap) {
    const Sizes z = sizes_of(g);
    const double nrays = (double)g.n_angles * g.n_bins;
    const double per = 4.0 * (4.0 * z.I + (double)z.VS + (double)z.Y + (double)z.Y) + 8.0 * std::ceil(nrays / 64.0) +
                       8 * 256.0;
    const double tiles = std::ceil(g.n / 16.0) * std::ceil(g.n / 16.0);
    const double fixed = 8.0 * g.n_angles + 48.0 * tiles * g.n_angles + 32.0 * g.n_angles + 4.0 * C + 64.0 +
                         16 * 256.0 + 8.0 * kLgammaOut;
    if ((double)cap < fixed + per) return 0;
    return (int)std::min<double>(C, std::floor(((double)cap - fixed) / per));
}

// Forward evaluation of C candidates of one slice. With env_grad set, also the envelope gradient:
// dJ/dtheta with the reconstruction F^K held fixed (one projection adjoint after the objective),
// ncomp components per candidate (8, or 9 with dR).
static boac_status eval_forward(boac_ctx *ctx, const boac_geom &g, const float *meas, const float *cand, int C,
                                float delta_r, int K, float *obj, float *img_out, uint32_t *status, hipStream_t st,
                                float *env_grad = nullptr, int ncomp = 8) {
    const int Cc = ctx->arena ? arena_chunk(g, C, ctx->arena->cap) : cand_chunk(sizes_of(g), C, env_grad ? 2 : 1);
    if (Cc < 1) return fail(BOAC_ENOMEM, "one candidate of this geometry needs more than the %zu-byte no-allocation "
                            "scratch", ctx->arena ? ctx->arena->cap : (size_t)0);
    DevGeom dg;
    Plan p;
    Sizes z;
    BOAC_TRY(plan_slice(ctx, g, Cc, true, &dg, &p, &z));
    float *E = nullptr, *Ebar = nullptr;
    if (z.E) BOAC_TRY(ensure_t(ctx, "attE", (size_t)Cc * z.E, &E));
    if (z.E && env_grad) BOAC_TRY(ensure_t(ctx, "attEbar", (size_t)Cc * z.E, &Ebar));
    float *mu, *att, *s, *F0, *F1, *r;
    float2 *partial, *lg;
    uint32_t *flag, *st_int;
    BOAC_TRY(ensure_t(ctx, "mu", (size_t)Cc * z.I, &mu));
    BOAC_TRY(ensure_t(ctx, "att", (size_t)Cc * z.VS, &att));
    BOAC_TRY(ensure_t(ctx, "s", (size_t)Cc * z.I, &s));
    BOAC_TRY(ensure_t(ctx, "F0", (size_t)Cc * z.I, &F0));
    BOAC_TRY(ensure_t(ctx, "F1", (size_t)Cc * z.I, &F1));
    BOAC_TRY(ensure_t(ctx, "r", (size_t)Cc * z.Y, &r));
    BOAC_TRY(ensure_t(ctx, "partial", (size_t)Cc * p.ray1.chunks, &partial));
    BOAC_TRY(ensure_t(ctx, "lg", kLgammaOut, &lg));
    BOAC_TRY(ensure_t(ctx, "flag", 4, &flag));
    BOAC_TRY(ensure_t(ctx, "status_int", (size_t)C, &st_int));
    float *attbar = nullptr, *yK = nullptr, *ybar = nullptr, *mubar = nullptr, *gtmp = nullptr;
    float2 *pair = nullptr;
    if (env_grad) {
        BOAC_TRY(ensure_t(ctx, "attbar", (size_t)Cc * z.VS, &attbar));
        BOAC_TRY(ensure_t(ctx, "yK", (size_t)Cc * z.Y, &yK));
        BOAC_TRY(ensure_t(ctx, "ybar", (size_t)Cc * z.Y, &ybar));
        BOAC_TRY(ensure_t(ctx, "mubar", (size_t)Cc * z.I, &mubar));
        BOAC_TRY(ensure_t(ctx, "gtmp", (size_t)Cc * kGradComps, &gtmp));
        BOAC_TRY(ensure_t(ctx, "pair", (size_t)Cc * z.I, &pair));
    }
    uint32_t *stat = status ? status : st_int;

    HIP_TRY(launch_fill_u32(flag, 4, 0u, st));
    HIP_TRY(launch_fill_u32(stat, (size_t)C, 0u, st));
    BOAC_TRY(timed(ctx, BOAC_K_REDUCE, 4.0 * z.Y, st,
                   [&] { return launch_lgamma_sum(meas, (int)z.Y, lg, flag, st); }));

    for (int c0 = 0; c0 < C; c0 += Cc) {
        const int n = std::min(Cc, C - c0);
        const float *cd = cand + (size_t)c0 * 8;
        BOAC_TRY(timed(ctx, BOAC_K_RASTER, 4.0 * n * (8 + z.I), st,
                       [&] { return launch_raster(dg, cd, n, delta_r, mu, z.I, stat + c0, st); }));
        BOAC_TRY(run_att(ctx, dg, p, z, mu, att, n, st, E));
        {
            BackArgs b = back_args(z, att, nullptr, s, n, E);
            BOAC_TRY(run_back(ctx, BACK_SENS, dg, p, z, b, st));
        }
        HIP_TRY(launch_fill(F0, (size_t)n * z.I, 1.f, st));
        float *Fc = F0, *Fn = F1;
        for (int it = 0; it < K; ++it) {
            FwdArgs a = fwd_args(z, att, Fc, meas, E);
            a.r_out = r;
            BOAC_TRY(run_fwd(ctx, FWD_RATIO, dg, p, z, a, n, st));
            BackArgs b = back_args(z, att, r, Fn, n, E);
            b.F = Fc;
            b.s = s;
            BOAC_TRY(run_back(ctx, BACK_MLEM, dg, p, z, b, st));
            std::swap(Fc, Fn);
        }
        FwdArgs a = fwd_args(z, att, Fc, meas, E);
        a.partial = partial;
        a.status = stat + c0;
        a.y_out = yK;
        BOAC_TRY(run_fwd(ctx, FWD_NLL, dg, p, z, a, n, st));
        BOAC_TRY(timed(ctx, BOAC_K_REDUCE, 8.0 * n * p.ray1.chunks, st, [&] {
            return launch_nll_finish(partial, p.ray1.chunks, n, lg, flag, obj + c0, stat + c0, st);
        }));
        if (img_out) HIP_TRY(launch_copy(Fc, img_out + (size_t)c0 * z.I, (size_t)n * z.I, st));
        if (env_grad) {
            // y = A F^K with F^K constant: att_bar = dx ybar (W F^K), then the scan and exp transposes
            // (the tail with a zero first image and rho = ybar), mu_bar = W^T m_bar, raster adjoint
            const size_t nI = (size_t)n * z.I, nY = (size_t)n * z.Y;
            BOAC_TRY(timed(ctx, BOAC_K_OTHER, 12.0 * nY, st,
                           [&] { return launch_ybar_final(meas, yK, ybar, n, (int)z.Y, z.Y, st); }));
            HIP_TRY(launch_pack_pair(nullptr, 0.f, Fc, 0.f, pair, nI, st));
            TailArgs ta{};
            ta.att = att;
            ta.attbar = attbar;
            ta.pair = (const float *)pair;
            ta.rho = ybar;
            ta.att_cs = z.VS;
            ta.img_cs = 2 * z.I;
            ta.sino_cs = z.Y;
            ta.accumulate = 0;
            ta.E = E;
            ta.Ebar = Ebar;
            ta.e_cs = z.E;
            BOAC_TRY(timed(ctx, BOAC_K_ADJ_RAY, 4.0 * n * (2.0 * z.V + 2 * z.E + 2 * z.I + z.Y), st,
                           [&] { return launch_tail(dg, p.ray2, p.bands2, ta, n, st); }));
            BackArgs b = back_args(z, att, attbar, mubar, n, Ebar);
            BOAC_TRY(run_back(ctx, BACK_FIELD, dg, p, z, b, st));
            BOAC_TRY(timed(ctx, BOAC_K_ADJ_PIX, 4.0 * n * z.I, st,
                           [&] { return launch_raster_adj(dg, cd, n, delta_r, mubar, z.I, gtmp, st); }));
            BOAC_TRY(timed(ctx, BOAC_K_OTHER, 4.0 * n * (kGradComps + ncomp), st, [&] {
                return launch_grad_finish(gtmp, n, ncomp, env_grad + (size_t)c0 * ncomp, stat + c0, st);
            }));
        }
    }
    return BOAC_OK;
}

// Objective and gradient of C candidates of one slice.
// ncomp gradient components per candidate: 8, or 9 with dR.
static boac_status eval_grad(boac_ctx *ctx, const boac_geom &g, const float *meas, const float *cand, int C,
                             float delta_r, int K, int ck, float *obj, float *grad, uint32_t *status, hipStream_t st,
                             int ncomp = 8) {
    if (ck < 1) ck = 1;
    if (ck > std::max(K, 1)) ck = std::max(K, 1);
    const int nck = (K + ck - 1) / ck;  // stored records 0, ck, 2ck, ... < K
    const int Cc = cand_chunk(sizes_of(g), C, 2);
    DevGeom dg;
    Plan p;
    Sizes z;
    BOAC_TRY(plan_slice(ctx, g, Cc, true, &dg, &p, &z));
    float *E = nullptr, *Ebar = nullptr;
    if (z.E) {
        BOAC_TRY(ensure_t(ctx, "attE", (size_t)Cc * z.E, &E));
        BOAC_TRY(ensure_t(ctx, "attEbar", (size_t)Cc * z.E, &Ebar));
    }
    const size_t I = z.I, Y = z.Y;
    float *mu, *att, *attbar, *s, *sbar, *fbar, *fdir, *mubar, *gtmp, *yK, *ybar, *ybar2, *Ftmp, *Fwork;
    float2 *pair, *partial, *lg;
    uint32_t *flag, *st_int;
    // records: F, y, r, Q per record; ckpt slots nck, segment slots ck
    float *recF, *recY, *recR, *recQ, *segF, *segY, *segR, *segQ;
    BOAC_TRY(ensure_t(ctx, "mu", (size_t)Cc * I, &mu));
    BOAC_TRY(ensure_t(ctx, "att", (size_t)Cc * z.VS, &att));
    BOAC_TRY(ensure_t(ctx, "attbar", (size_t)Cc * z.VS, &attbar));
    BOAC_TRY(ensure_t(ctx, "s", (size_t)Cc * I, &s));
    BOAC_TRY(ensure_t(ctx, "sbar", (size_t)Cc * I, &sbar));
    BOAC_TRY(ensure_t(ctx, "fbar", (size_t)Cc * I, &fbar));
    BOAC_TRY(ensure_t(ctx, "fdir", (size_t)Cc * I, &fdir));
    BOAC_TRY(ensure_t(ctx, "mubar", (size_t)Cc * I, &mubar));
    BOAC_TRY(ensure_t(ctx, "gtmp", (size_t)Cc * kGradComps, &gtmp));
    BOAC_TRY(ensure_t(ctx, "yK", (size_t)Cc * Y, &yK));
    BOAC_TRY(ensure_t(ctx, "ybar", (size_t)Cc * Y, &ybar));
    BOAC_TRY(ensure_t(ctx, "ybar2", (size_t)Cc * Y, &ybar2));
    BOAC_TRY(ensure_t(ctx, "Ftmp", (size_t)Cc * I, &Ftmp));
    BOAC_TRY(ensure_t(ctx, "Fwork", (size_t)2 * Cc * I, &Fwork));
    BOAC_TRY(ensure_t(ctx, "pair", (size_t)Cc * I, &pair));
    BOAC_TRY(ensure_t(ctx, "partial", (size_t)Cc * p.ray1.chunks, &partial));
    BOAC_TRY(ensure_t(ctx, "lg", kLgammaOut, &lg));
    BOAC_TRY(ensure_t(ctx, "flag", 4, &flag));
    BOAC_TRY(ensure_t(ctx, "status_int", (size_t)C, &st_int));
    BOAC_TRY(ensure_t(ctx, "recF", (size_t)std::max(nck, 1) * Cc * I, &recF));
    BOAC_TRY(ensure_t(ctx, "recY", (size_t)std::max(nck, 1) * Cc * Y, &recY));
    BOAC_TRY(ensure_t(ctx, "recR", (size_t)std::max(nck, 1) * Cc * Y, &recR));
    BOAC_TRY(ensure_t(ctx, "recQ", (size_t)std::max(nck, 1) * Cc * I, &recQ));
    BOAC_TRY(ensure_t(ctx, "segF", (size_t)ck * Cc * I, &segF));
    BOAC_TRY(ensure_t(ctx, "segY", (size_t)ck * Cc * Y, &segY));
    BOAC_TRY(ensure_t(ctx, "segR", (size_t)ck * Cc * Y, &segR));
    BOAC_TRY(ensure_t(ctx, "segQ", (size_t)ck * Cc * I, &segQ));
    uint32_t *stat = status ? status : st_int;

    HIP_TRY(launch_fill_u32(flag, 4, 0u, st));
    HIP_TRY(launch_fill_u32(stat, (size_t)C, 0u, st));
    BOAC_TRY(timed(ctx, BOAC_K_REDUCE, 4.0 * Y, st, [&] { return launch_lgamma_sum(meas, (int)Y, lg, flag, st); }));

    for (int c0 = 0; c0 < C; c0 += Cc) {
        const int n = std::min(Cc, C - c0);
        const float *cd = cand + (size_t)c0 * 8;
        const size_t nI = (size_t)n * I, nY = (size_t)n * Y;
        auto rec = [&](float *base, int slot, size_t per) { return base + (size_t)slot * Cc * per; };

        BOAC_TRY(timed(ctx, BOAC_K_RASTER, 4.0 * n * (8 + I), st,
                       [&] { return launch_raster(dg, cd, n, delta_r, mu, I, stat + c0, st); }));
        BOAC_TRY(run_att(ctx, dg, p, z, mu, att, n, st, E));
        {
            BackArgs b = back_args(z, att, nullptr, s, n, E);
            BOAC_TRY(run_back(ctx, BACK_SENS, dg, p, z, b, st));
        }
        // one MLEM iteration from record (F, y, r, Q) slots: fills y, r, Q and writes F^{n+1} to Fnext
        auto iterate = [&](const float *F, float *y, float *r, float *Q, float *Fnext) -> boac_status {
            FwdArgs a = fwd_args(z, att, F, meas, E);
            a.r_out = r;
            a.y_out = y;
            BOAC_TRY(run_fwd(ctx, FWD_RATIO, dg, p, z, a, n, st));
            BackArgs b = back_args(z, att, r, Fnext, n, E);
            b.F = F;
            b.s = s;
            b.q_out = Q;
            return run_back(ctx, BACK_MLEM, dg, p, z, b, st);
        };

        // ---- forward sweep, storing records at checkpoints
        float *Fcur = rec(recF, 0, I);
        HIP_TRY(launch_fill(Fcur, nI, 1.f, st));
        float *work[2] = {Fwork, Fwork + (size_t)Cc * I};
        int wsel = 0;
        for (int it = 0; it < K; ++it) {
            const bool is_ck = (it % ck) == 0;
            float *y = is_ck ? rec(recY, it / ck, Y) : segY;
            float *r = is_ck ? rec(recR, it / ck, Y) : segR;
            float *Q = is_ck ? rec(recQ, it / ck, I) : segQ;
            float *Fnext;
            if ((it + 1) < K && ((it + 1) % ck) == 0) {
                Fnext = rec(recF, (it + 1) / ck, I);
            } else {
                Fnext = work[wsel];
                wsel ^= 1;
            }
            BOAC_TRY(iterate(Fcur, y, r, Q, Fnext));
            Fcur = Fnext;
        }
        // ---- objective at F^K (y^K kept for the reverse sweep)
        {
            FwdArgs a = fwd_args(z, att, Fcur, meas, E);
            a.partial = partial;
            a.status = stat + c0;
            a.y_out = yK;
            BOAC_TRY(run_fwd(ctx, FWD_NLL, dg, p, z, a, n, st));
            BOAC_TRY(timed(ctx, BOAC_K_REDUCE, 8.0 * n * p.ray1.chunks, st, [&] {
                return launch_nll_finish(partial, p.ray1.chunks, n, lg, flag, obj + c0, stat + c0, st);
            }));
        }
        // ---- reverse sweep
        // d/dy (y - S ln y) at y^K: ybar^K = 1 - S / y^K where y^K > 0 (1 where S = 0). It stays
        // pending (its att_bar term is added by the first reverse step's sweep, or by the tail).
        float *ypend = ybar, *ynext = ybar2;
        HIP_TRY(launch_fill(sbar, nI, 0.f, st));
        BOAC_TRY(timed(ctx, BOAC_K_OTHER, 12.0 * nY, st,
                       [&] { return launch_ybar_final(meas, yK, ypend, n, (int)Y, Y, st); }));
        if (K > 0) {
            BackArgs b = back_args(z, att, ypend, fbar, n, E);
            BOAC_TRY(run_back(ctx, BACK_PLAIN, dg, p, z, b, st));
        }
        bool first = true;
        for (int sg = nck - 1; sg >= 0; --sg) {
            const int n0 = sg * ck, n1 = std::min(n0 + ck, K);
            // segment slot j holds record n0 + j
            std::vector<float *> sF(ck), sY(ck), sR(ck), sQ(ck);
            sF[0] = rec(recF, sg, I);
            sY[0] = rec(recY, sg, Y);
            sR[0] = rec(recR, sg, Y);
            sQ[0] = rec(recQ, sg, I);
            for (int j = 1; j < n1 - n0; ++j) {
                sF[j] = rec(segF, j, I);
                sY[j] = rec(segY, j, Y);
                sR[j] = rec(segR, j, Y);
                sQ[j] = rec(segQ, j, I);
                // F^{n0+j} = F^{n0+j-1} * Q^{n0+j-1}, bit-identical to the forward sweep's update
                HIP_TRY(launch_mul_copy(sF[j - 1], sQ[j - 1], sF[j], nI, st));
                BOAC_TRY(iterate(sF[j], sY[j], sR[j], sQ[j], Ftmp));
            }
            for (int j = n1 - n0 - 1; j >= 0; --j) {
                const int it = n0 + j;
                // F^{n+1} = F^n Q^n:  bbar^n, s_bar, direct part of F_bar^n; pair (bbar^n, F^{n+1})
                AdjElemArgs e{};
                e.fbar = fbar;
                e.F = sF[j];
                e.Q = sQ[j];
                e.s = s;
                e.sbar = sbar;
                e.pair = pair;
                e.fbar_direct = fdir;
                e.img_cs = I;
                e.npix = (int)I;
                e.C = n;
                BOAC_TRY(timed(ctx, BOAC_K_OTHER, 4.0 * n * 8.0 * I, st, [&] { return launch_adj_elem(e, st); }));
                // one sweep: ybar^n and att_bar += dx (r^n W bbar^n + ybar^{n+1} W F^{n+1})
                SweepArgs sa{};
                sa.att = att;
                sa.attbar = attbar;
                sa.pair = (const float *)pair;
                sa.r = sR[j];
                sa.y = sY[j];
                sa.ybar_in = ypend;
                sa.ybar_out = ynext;
                sa.att_cs = z.VS;
                sa.img_cs = 2 * I;
                sa.sino_cs = Y;
                sa.accumulate = first ? 0 : 1;
                sa.E = E;
                sa.Ebar = Ebar;
                sa.e_cs = z.E;
                BOAC_TRY(timed(ctx, BOAC_K_ADJ_RAY, 4.0 * n * ((first ? 2.0 : 3.0) * z.V + 2 * I + 4 * Y), st,
                               [&] { return launch_adj_sweep(dg, p.ray2, p.bands2, sa, n, st); }));
                first = false;
                std::swap(ypend, ynext);
                if (it > 0) {
                    BackArgs b = back_args(z, att, ypend, fbar, n, E);
                    b.aux = fdir;
                    BOAC_TRY(run_back(ctx, BACK_ADJ, dg, p, z, b, st));
                }
            }
        }
        // ---- tail: sensitivity adjoint and the pending projection adjoint (with F^0 = 1), exp and
        // scan transposes, mu_bar, raster adjoint
        {
            HIP_TRY(launch_pack_pair(sbar, 0.f, nullptr, 1.f, pair, nI, st));
            TailArgs ta{};
            ta.att = att;
            ta.attbar = attbar;
            ta.pair = (const float *)pair;
            ta.rho = ypend;
            ta.att_cs = z.VS;
            ta.img_cs = 2 * I;
            ta.sino_cs = Y;
            ta.accumulate = first ? 0 : 1;
            ta.E = E;
            ta.Ebar = Ebar;
            ta.e_cs = z.E;
            BOAC_TRY(timed(ctx, BOAC_K_ADJ_RAY, 4.0 * n * (3.0 * z.V + 2 * I + Y), st,
                           [&] { return launch_tail(dg, p.ray2, p.bands2, ta, n, st); }));
            BackArgs b = back_args(z, att, attbar, mubar, n, Ebar);
            BOAC_TRY(run_back(ctx, BACK_FIELD, dg, p, z, b, st));
            BOAC_TRY(timed(ctx, BOAC_K_ADJ_PIX, 4.0 * n * I, st,
                           [&] { return launch_raster_adj(dg, cd, n, delta_r, mubar, I, gtmp, st); }));
            BOAC_TRY(timed(ctx, BOAC_K_OTHER, 4.0 * n * (kGradComps + ncomp), st, [&] {
                return launch_grad_finish(gtmp, n, ncomp, grad + (size_t)c0 * ncomp, stat + c0, st);
            }));
        }
    }
    return BOAC_OK;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

int32_t boac_version(void) { return (1 << 16) | 0; }

const char *boac_last_error(void) { return g_last_error.c_str(); }

static void load_tune(boac_ctx *ctx, const char *path) {
    if (!path || !*path) path = std::getenv("BOAC_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "rb");
    if (!f) return;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    std::fclose(f);
    // flat JSON object {"key": [ints], ...}
    size_t i = 0;
    while (true) {
        size_t q0 = s.find('"', i);
        if (q0 == std::string::npos) break;
        size_t q1 = s.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        size_t b0 = s.find('[', q1);
        size_t b1 = s.find(']', b0 == std::string::npos ? q1 : b0);
        if (b0 == std::string::npos || b1 == std::string::npos) break;
        std::vector<int> vals;
        const char *p = s.c_str() + b0 + 1;
        const char *end = s.c_str() + b1;
        while (p < end) {
            char *e = nullptr;
            long v = std::strtol(p, &e, 10);
            if (e == p) {
                ++p;
                continue;
            }
            vals.push_back((int)v);
            p = e;
        }
        ctx->tune[key] = vals;
        i = b1 + 1;
    }
}

boac_status boac_ctx_create(int32_t device, const char *tune_cache_path, boac_ctx **out) {
    if (!out) return fail(BOAC_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(BOAC_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    }
    if (device < 0 || device >= count) return fail(BOAC_EINVAL, "device %d outside [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BOAC_ENOTSUP, "device %d is %s; libboac is built for gfx950", device, prop.gcnArchName);
    auto ctx = std::make_unique<boac_ctx>();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    BOAC_TRY(noalloc_base(device, &ctx->noalloc));
    load_tune(ctx.get(), tune_cache_path);
    *out = ctx.release();
    return BOAC_OK;
}

void boac_ctx_destroy(boac_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &g : ctx->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (auto &kv : ctx->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    for (auto &kv : ctx->trig) (void)hipFree(kv.second);
    for (auto &kv : ctx->rects) (void)hipFree(kv.second);
    for (auto &p : ctx->pending) {
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    for (auto st : ctx->lanes) (void)hipStreamDestroy(st);
    for (auto e : ctx->lane_done) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    delete ctx;
}

#define CTX_CHECK()                                                      \
    do {                                                                 \
        if (!ctx) return fail(BOAC_EINVAL, "context is NULL");           \
        HIP_TRY(hipSetDevice(ctx->device));                              \
    } while (0)

boac_status boac_rasterize_mu(boac_ctx *ctx, const boac_geom *geom, const boac_cand *d_cand, int32_t C,
                              float delta_r_cm, float *d_mu, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_cand, "d_cand"));
    BOAC_TRY(check_ptr(d_mu, "d_mu"));
    if (!(delta_r_cm > 0.f) || !std::isfinite(delta_r_cm)) return fail(BOAC_EINVAL, "delta_r_cm must be > 0");
    CTX_CHECK();
    DevGeom dg;
    BOAC_TRY(dev_geom(ctx, *geom, &dg));
    hipStream_t st = (hipStream_t)stream;
    const Sizes z = sizes_of(*geom);
    return timed(ctx, BOAC_K_RASTER, 4.0 * C * (8 + z.I), st, [&] {
        return launch_raster(dg, (const float *)d_cand, C, delta_r_cm, d_mu, z.I, nullptr, st);
    });
}

// att for a chunk of candidates from caller mu maps
// The attenuation tensors of n candidates (and exp(-T) per held ray with opposed-ray pairing).
static boac_status build_att(boac_ctx *ctx, const Sizes &z, const DevGeom &dg, const Plan &p, const float *mu,
                             int n, float **att_out, float **E_out, hipStream_t st) {
    float *att, *E = nullptr;
    BOAC_TRY(ensure_t(ctx, "att", (size_t)n * z.VS, &att));
    if (z.E) BOAC_TRY(ensure_t(ctx, "attE", (size_t)n * z.E, &E));
    BOAC_TRY(run_att(ctx, dg, p, z, mu, att, n, st, E));
    *att_out = att;
    *E_out = E;
    return BOAC_OK;
}

boac_status boac_project(boac_ctx *ctx, const boac_geom *geom, const float *d_mu, const float *d_img, int32_t C,
                         float *d_sino, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_mu, "d_mu"));
    BOAC_TRY(check_ptr(d_img, "d_img"));
    BOAC_TRY(check_ptr(d_sino, "d_sino"));
    CTX_CHECK();
    hipStream_t st = (hipStream_t)stream;
    const int Cc = cand_chunk(sizes_of(*geom), C, 1);
    DevGeom dg;
    Plan p;
    Sizes z;
    BOAC_TRY(plan_slice(ctx, *geom, Cc, true, &dg, &p, &z));
    for (int c0 = 0; c0 < C; c0 += Cc) {
        const int n = std::min(Cc, C - c0);
        float *att, *E;
        BOAC_TRY(build_att(ctx, z, dg, p, d_mu + (size_t)c0 * z.I, n, &att, &E, st));
        FwdArgs a = fwd_args(z, att, d_img + (size_t)c0 * z.I, nullptr, E);
        a.y_out = d_sino + (size_t)c0 * z.Y;
        BOAC_TRY(run_fwd(ctx, FWD_PROJ, dg, p, z, a, n, st));
    }
    return BOAC_OK;
}

boac_status boac_backproject(boac_ctx *ctx, const boac_geom *geom, const float *d_mu, const float *d_sino, int32_t C,
                             float *d_img, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_mu, "d_mu"));
    BOAC_TRY(check_ptr(d_sino, "d_sino"));
    BOAC_TRY(check_ptr(d_img, "d_img"));
    CTX_CHECK();
    hipStream_t st = (hipStream_t)stream;
    const int Cc = cand_chunk(sizes_of(*geom), C, 1);
    DevGeom dg;
    Plan p;
    Sizes z;
    BOAC_TRY(plan_slice(ctx, *geom, Cc, true, &dg, &p, &z));
    for (int c0 = 0; c0 < C; c0 += Cc) {
        const int n = std::min(Cc, C - c0);
        float *att, *E;
        BOAC_TRY(build_att(ctx, z, dg, p, d_mu + (size_t)c0 * z.I, n, &att, &E, st));
        BackArgs b = back_args(z, att, d_sino + (size_t)c0 * z.Y, d_img + (size_t)c0 * z.I, n, E);
        BOAC_TRY(run_back(ctx, BACK_PLAIN, dg, p, z, b, st));
    }
    return BOAC_OK;
}

boac_status boac_mlem(boac_ctx *ctx, const boac_geom *geom, const float *d_mu, const float *d_meas, int32_t C,
                      int32_t n_iter, float *d_img_inout, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_mu, "d_mu"));
    BOAC_TRY(check_ptr(d_meas, "d_meas"));
    BOAC_TRY(check_ptr(d_img_inout, "d_img_inout"));
    if (n_iter < 0 || n_iter > 100000) return fail(BOAC_EINVAL, "n_iter = %d outside [0, 100000]", n_iter);
    CTX_CHECK();
    hipStream_t st = (hipStream_t)stream;
    const int Cc = cand_chunk(sizes_of(*geom), C, 1);
    DevGeom dg;
    Plan p;
    Sizes z;
    BOAC_TRY(plan_slice(ctx, *geom, Cc, true, &dg, &p, &z));
    float *s, *Fs, *r;
    BOAC_TRY(ensure_t(ctx, "s", (size_t)Cc * z.I, &s));
    BOAC_TRY(ensure_t(ctx, "F1", (size_t)Cc * z.I, &Fs));
    BOAC_TRY(ensure_t(ctx, "r", (size_t)Cc * z.Y, &r));
    for (int c0 = 0; c0 < C; c0 += Cc) {
        const int n = std::min(Cc, C - c0);
        float *att, *E;
        BOAC_TRY(build_att(ctx, z, dg, p, d_mu + (size_t)c0 * z.I, n, &att, &E, st));
        BackArgs sb = back_args(z, att, nullptr, s, n, E);
        BOAC_TRY(run_back(ctx, BACK_SENS, dg, p, z, sb, st));
        float *Fio = d_img_inout + (size_t)c0 * z.I;
        float *Fc = Fio, *Fn = Fs;
        for (int it = 0; it < n_iter; ++it) {
            FwdArgs a = fwd_args(z, att, Fc, d_meas, E);
            a.r_out = r;
            BOAC_TRY(run_fwd(ctx, FWD_RATIO, dg, p, z, a, n, st));
            BackArgs b = back_args(z, att, r, Fn, n, E);
            b.F = Fc;
            b.s = s;
            BOAC_TRY(run_back(ctx, BACK_MLEM, dg, p, z, b, st));
            std::swap(Fc, Fn);
        }
        if (Fc != Fio) HIP_TRY(launch_copy(Fc, Fio, (size_t)n * z.I, st));
    }
    return BOAC_OK;
}

boac_status boac_objective(boac_ctx *ctx, const boac_geom *geom, const float *d_meas, const boac_cand *d_cand,
                           int32_t C, float delta_r_cm, int32_t n_iter, float *d_obj, float *d_img_out,
                           uint32_t *d_status, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_meas, "d_meas"));
    BOAC_TRY(check_ptr(d_cand, "d_cand"));
    BOAC_TRY(check_ptr(d_obj, "d_obj"));
    BOAC_TRY(check_ptr(d_img_out, "d_img_out", true));
    BOAC_TRY(check_ptr(d_status, "d_status", true));
    if (n_iter < 0 || n_iter > 100000) return fail(BOAC_EINVAL, "n_iter = %d outside [0, 100000]", n_iter);
    if (!(delta_r_cm > 0.f) || !std::isfinite(delta_r_cm)) return fail(BOAC_EINVAL, "delta_r_cm must be > 0");
    CTX_CHECK();
    return eval_forward(ctx, *geom, d_meas, (const float *)d_cand, C, delta_r_cm, n_iter, d_obj, d_img_out, d_status,
                        (hipStream_t)stream);
}

boac_status boac_objective_noalloc(boac_ctx *ctx, const boac_geom *geom, const float *d_meas,
                                   const boac_cand *d_cand, int32_t C, float delta_r_cm, int32_t n_iter,
                                   float *d_obj, float *d_img_out, uint32_t *d_status, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_meas, "d_meas"));
    BOAC_TRY(check_ptr(d_cand, "d_cand"));
    BOAC_TRY(check_ptr(d_obj, "d_obj"));
    BOAC_TRY(check_ptr(d_img_out, "d_img_out", true));
    BOAC_TRY(check_ptr(d_status, "d_status", true));
    if (n_iter < 0 || n_iter > 100000) return fail(BOAC_EINVAL, "n_iter = %d outside [0, 100000]", n_iter);
    if (!(delta_r_cm > 0.f) || !std::isfinite(delta_r_cm)) return fail(BOAC_EINVAL, "delta_r_cm must be > 0");
    if (arena_chunk(*geom, C, BOAC_NOALLOC_SCRATCH_BYTES) < 1)
        return fail(BOAC_ENOMEM, "boac_objective_noalloc: %d candidates of a %dx%d image, %d angles x %d bins x %d "
                    "samples need more than the %u-byte no-allocation scratch",
                    C, geom->n, geom->n, geom->n_angles, geom->n_bins, geom->n_samples,
                    (unsigned)BOAC_NOALLOC_SCRATCH_BYTES);
    CTX_CHECK();
    if (!ctx->noalloc) return fail(BOAC_EDEVICE, "no-allocation scratch address unknown");
    Arena arena;
    arena.base = (char *)ctx->noalloc;
    arena.cap = BOAC_NOALLOC_SCRATCH_BYTES;
    ctx->arena = &arena;
    ctx->arena_stream = (hipStream_t)stream;
    ctx->ns.clear();
    const boac_status r = eval_forward(ctx, *geom, d_meas, (const float *)d_cand, C, delta_r_cm, n_iter, d_obj,
                                       d_img_out, d_status, (hipStream_t)stream);
    ctx->arena = nullptr;
    ctx->arena_stream = nullptr;
    return r;
}

boac_status boac_objective_grad(boac_ctx *ctx, const boac_geom *geom, const float *d_meas, const boac_cand *d_cand,
                                int32_t C, float delta_r_cm, int32_t n_iter, int32_t ckpt_every, float *d_obj,
                                float *d_grad, uint32_t *d_status, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_meas, "d_meas"));
    BOAC_TRY(check_ptr(d_cand, "d_cand"));
    BOAC_TRY(check_ptr(d_obj, "d_obj"));
    BOAC_TRY(check_ptr(d_grad, "d_grad"));
    BOAC_TRY(check_ptr(d_status, "d_status", true));
    if (n_iter < 0 || n_iter > 100000) return fail(BOAC_EINVAL, "n_iter = %d outside [0, 100000]", n_iter);
    if (ckpt_every < 1) return fail(BOAC_EINVAL, "ckpt_every = %d must be >= 1", ckpt_every);
    if (!(delta_r_cm > 0.f) || !std::isfinite(delta_r_cm)) return fail(BOAC_EINVAL, "delta_r_cm must be > 0");
    CTX_CHECK();
    return eval_grad(ctx, *geom, d_meas, (const float *)d_cand, C, delta_r_cm, n_iter, ckpt_every, d_obj, d_grad,
                     d_status, (hipStream_t)stream);
}

boac_status boac_objective_grad_ex(boac_ctx *ctx, const boac_geom *geom, const float *d_meas,
                                   const boac_cand *d_cand, int32_t C, float delta_r_cm, int32_t n_iter,
                                   int32_t ckpt_every, int32_t grad_mode, float *d_obj, float *d_grad,
                                   uint32_t *d_status, void *stream) {
    BOAC_TRY(check_geom(geom));
    BOAC_TRY(check_count(C));
    BOAC_TRY(check_ptr(d_meas, "d_meas"));
    BOAC_TRY(check_ptr(d_cand, "d_cand"));
    BOAC_TRY(check_ptr(d_obj, "d_obj"));
    BOAC_TRY(check_ptr(d_grad, "d_grad"));
    BOAC_TRY(check_ptr(d_status, "d_status", true));
    if (n_iter < 0 || n_iter > 100000) return fail(BOAC_EINVAL, "n_iter = %d outside [0, 100000]", n_iter);
    if (ckpt_every < 1) return fail(BOAC_EINVAL, "ckpt_every = %d must be >= 1", ckpt_every);
    if (!(delta_r_cm > 0.f) || !std::isfinite(delta_r_cm)) return fail(BOAC_EINVAL, "delta_r_cm must be > 0");
    if (grad_mode != BOAC_GRAD_UNROLLED && grad_mode != BOAC_GRAD_ENVELOPE)
        return fail(BOAC_EINVAL, "grad_mode = %d is neither BOAC_GRAD_UNROLLED nor BOAC_GRAD_ENVELOPE", grad_mode);
    CTX_CHECK();
    if (grad_mode == BOAC_GRAD_ENVELOPE)
        return eval_forward(ctx, *geom, d_meas, (const float *)d_cand, C, delta_r_cm, n_iter, d_obj, nullptr,
                            d_status, (hipStream_t)stream, d_grad, 9);
    return eval_grad(ctx, *geom, d_meas, (const float *)d_cand, C, delta_r_cm, n_iter, ckpt_every, d_obj, d_grad,
                     d_status, (hipStream_t)stream, 9);
}

// ------------------------------------------------------------------ surrogate (Eqs. 7-10)
boac_status boac_gp_fit(const double *h_u, const double *h_y, int32_t n, int32_t d, const double *h_lengths,
                        int32_t n_lengths, int32_t n_select, double noise, double *h_linv, double *h_alpha,
                        boac_gp_info *info) {
    if (n < 1 || n > 8192) return fail(BOAC_EINVAL, "n = %d outside [1, 8192]", n);
    if (d < 1 || d > 64) return fail(BOAC_EINVAL, "d = %d outside [1, 64]", d);
    if (n_lengths < 1) return fail(BOAC_EINVAL, "n_lengths = %d must be >= 1", n_lengths);
    if (!h_u || !h_y || !h_lengths || !h_linv || !h_alpha || !info)
        return fail(BOAC_EINVAL, "a pointer argument of boac_gp_fit is NULL");
    if (!(noise >= 0.0) || !std::isfinite(noise)) return fail(BOAC_EINVAL, "noise must be finite and >= 0");
    for (int i = 0; i < n_lengths; ++i)
        if (!(h_lengths[i] > 0.0) || !std::isfinite(h_lengths[i]))
            return fail(BOAC_EINVAL, "length %d is not a positive finite value", i);
    for (size_t i = 0; i < (size_t)n * d; ++i)
        if (!std::isfinite(h_u[i])) return fail(BOAC_EINVAL, "h_u[%zu] is not finite", i);
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(h_y[i])) return fail(BOAC_EINVAL, "h_y[%d] is not finite", i);
    // model selection on the n_select smallest objectives (stable: ties by index)
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    int ns = n;
    if (n_select > 0 && n_select < n) {
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return h_y[a] < h_y[b]; });
        ns = n_select;
    }
    std::vector<double> us((size_t)ns * d), ys(ns), L((size_t)n * n), al(n);
    for (int r = 0; r < ns; ++r) {
        ys[r] = h_y[idx[r]];
        for (int c = 0; c < d; ++c) us[(size_t)r * d + c] = h_u[(size_t)idx[r] * d + c];
    }
    // the grid's fits are independent: up to 16 host threads take them in turn, each with its own
    // factor; the choice below runs over the results in grid order (first on ties), as a serial loop
    std::vector<double> lmls(n_lengths, 0.0);
    std::vector<char> ok(n_lengths, 0);
    const int nthreads = std::max(1, std::min({n_lengths, 16, (int)std::thread::hardware_concurrency()}));
    std::atomic<int> next{0};
    auto worker = [&] {
        std::vector<double> Lw((size_t)ns * ns), aw(ns);
        double mw, sw, lw;
        for (int g = next++; g < n_lengths; g = next++) {
            ok[g] = gp_fit_fixed(us.data(), ys.data(), ns, d, h_lengths[g], 1.0, noise, Lw.data(), aw.data(), &mw, &sw,
                                 &lw);
            lmls[g] = lw;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
    int best = -1;
    double best_lml = 0.0, m0, s, lml;
    for (int g = 0; g < n_lengths; ++g) {
        if (!ok[g]) continue;
        if (best < 0 || lmls[g] > best_lml) {
            best = g;
            best_lml = lmls[g];
        }
    }
    if (best < 0) return fail(BOAC_EINVAL, "no length-scale gives a positive definite covariance; raise noise");
    if (!gp_fit_fixed(h_u, h_y, n, d, h_lengths[best], 1.0, noise, L.data(), h_alpha, &m0, &s, &lml))
        return fail(BOAC_EINVAL, "covariance of all %d observations is not positive definite; raise noise", n);
    gp_tri_inverse(L.data(), h_linv, n);
    info->n = n;
    info->d = d;
    info->length = h_lengths[best];
    info->amp = 1.0;
    info->noise = noise;
    info->m0 = m0;
    info->s = s;
    info->lml = lml;
    return BOAC_OK;
}

// The EI launch arguments of a fitted surrogate for M queries, validated (no device call; the scratch
// pointers are set by gp_ei_scratch).
static boac_status gp_ei_args(const boac_gp_info *info, const double *d_u, const double *d_linv,
                              const double *d_alpha, int32_t M, double best, double xi, GpEiArgs *out) {
    if (!info) return fail(BOAC_EINVAL, "info is NULL");
    if (info->n < 1 || info->n > 8192 || info->d < 1 || info->d > 64)
        return fail(BOAC_EINVAL, "info holds n = %d, d = %d outside the supported range", info->n, info->d);
    if (!(info->length > 0.0) || !std::isfinite(info->length) || !(info->s > 0.0) || !std::isfinite(info->s) ||
        !std::isfinite(info->m0) || !(info->amp > 0.0) || !std::isfinite(info->amp))
        return fail(BOAC_EINVAL, "info holds a non-positive or non-finite model parameter");
    if (M < 1 || M > (1 << 20)) return fail(BOAC_EINVAL, "M = %d outside [1, 2^20]", M);
    if (!std::isfinite(best) || !(xi >= 0.0) || !std::isfinite(xi))
        return fail(BOAC_EINVAL, "best must be finite and xi finite and >= 0");
    BOAC_TRY(check_ptr(d_u, "d_u"));
    BOAC_TRY(check_ptr(d_linv, "d_linv"));
    BOAC_TRY(check_ptr(d_alpha, "d_alpha"));
    GpEiArgs a{};
    a.u = d_u;
    a.linv = d_linv;
    a.alpha = d_alpha;
    a.n = info->n;
    a.d = info->d;
    a.M = M;
    a.npad = (info->n + 63) / 64 * 64;
    a.nti = (info->n + 63) / 64;
    a.inv2l2 = 1.0 / (2.0 * info->length * info->length);
    a.amp = info->amp;
    a.m0 = info->m0;
    a.s = info->s;
    a.best = best;
    a.xi = xi;
    *out = a;
    return BOAC_OK;
}

static boac_status gp_ei_scratch(boac_ctx *ctx, GpEiArgs *a) {
    BOAC_TRY(ensure_t(ctx, "gp_ks", (size_t)a->M * a->npad, &a->ks));
    return ensure_t(ctx, "gp_part", (size_t)a->M * a->nti, &a->part);
}

boac_status boac_gp_ei(boac_ctx *ctx, const boac_gp_info *info, const double *d_u, const double *d_linv,
                       const double *d_alpha, const double *d_q, int32_t M, double best, double xi, double *d_mu,
                       double *d_sigma, double *d_ei, void *stream) {
    GpEiArgs a{};
    BOAC_TRY(gp_ei_args(info, d_u, d_linv, d_alpha, M, best, xi, &a));
    BOAC_TRY(check_ptr(d_q, "d_q"));
    BOAC_TRY(check_ptr(d_ei, "d_ei"));
    BOAC_TRY(check_ptr(d_mu, "d_mu", true));
    BOAC_TRY(check_ptr(d_sigma, "d_sigma", true));
    CTX_CHECK();
    BOAC_TRY(gp_ei_scratch(ctx, &a));
    a.q = d_q;
    a.mu = d_mu;
    a.sd = d_sigma;
    a.ei = d_ei;
    const hipStream_t st = (hipStream_t)stream;
    return timed(ctx, BOAC_K_GP, 0.0, st, [&] { return launch_gp_ei(a, st); });
}

// The local rounds of the acquisition search: n_local rounds of points, EI, centre moves and chain steps
// (the chains split evenly over nc centres, per = P / nc each), writing each round's points and values.
static boac_status chaos_local_rounds(boac_ctx *ctx, GpEiArgs a, double *d_z, int P, double *d_centres,
                                      double *d_centre_ei, int nc, double radius0, double shrink, int n_local,
                                      double *d_pts, double *d_vals, hipStream_t st) {
    const int per = P / nc, M = per * nc, d = a.d;
    double r = radius0;
    for (int t = 0; t < n_local; ++t) {
        double *U = d_pts + (size_t)t * M * d;
        double *e = d_vals + (size_t)t * M;
        HIP_TRY(launch_chaos_points(d_z, d_centres, r, per, nc, d, U, st));
        a.q = U;
        a.ei = e;
        a.mu = a.sd = nullptr;
        BOAC_TRY(timed(ctx, BOAC_K_GP, 0.0, st, [&] { return launch_gp_ei(a, st); }));
        HIP_TRY(launch_chaos_centres(U, e, per, nc, d, d_centres, d_centre_ei, st));
        HIP_TRY(launch_chaos_step(d_z, P * d, st));
        r *= shrink;
    }
    return BOAC_OK;
}

boac_status boac_gp_chaos_local(boac_ctx *ctx, const boac_gp_info *info, const double *d_u, const double *d_linv,
                                const double *d_alpha, double best, double xi, double *d_z, int32_t P,
                                double *d_centres, double *d_centre_ei, int32_t n_centres, double radius0,
                                double shrink, int32_t n_local, double *d_pts, double *d_vals, void *stream) {
    if (P < 1 || n_centres < 1 || n_centres > P)
        return fail(BOAC_EINVAL, "need 1 <= n_centres <= P (P = %d, n_centres = %d)", P, n_centres);
    if (n_local < 0 || n_local > 4096) return fail(BOAC_EINVAL, "n_local = %d outside [0, 4096]", n_local);
    if (!std::isfinite(radius0) || !(radius0 >= 0.0) || !std::isfinite(shrink) || !(shrink >= 0.0))
        return fail(BOAC_EINVAL, "radius0 and shrink must be finite and >= 0");
    BOAC_TRY(check_ptr(d_z, "d_z"));
    BOAC_TRY(check_ptr(d_centres, "d_centres"));
    BOAC_TRY(check_ptr(d_centre_ei, "d_centre_ei"));
    BOAC_TRY(check_ptr(d_pts, "d_pts", n_local == 0));
    BOAC_TRY(check_ptr(d_vals, "d_vals", n_local == 0));
    const int per = P / n_centres;
    const int M = per * n_centres;
    GpEiArgs a{};
    BOAC_TRY(gp_ei_args(info, d_u, d_linv, d_alpha, M, best, xi, &a));
    const int d = a.d;
    if ((long long)P * d >= (1LL << 31) || (long long)n_local * M * d >= (1LL << 40))
        return fail(BOAC_EINVAL, "P x d or n_local x M x d too large");
    CTX_CHECK();
    BOAC_TRY(gp_ei_scratch(ctx, &a));
    return chaos_local_rounds(ctx, a, d_z, P, d_centres, d_centre_ei, n_centres, radius0, shrink, n_local, d_pts,
                              d_vals, (hipStream_t)stream);
}

boac_status boac_gp_chaos_search(boac_ctx *ctx, const boac_gp_info *info, const double *d_u, const double *d_linv,
                                 const double *d_alpha, double best, double xi, const double *d_z0, int32_t P,
                                 int32_t n_global, int32_t n_local, int32_t centres, int32_t q, double radius0,
                                 double shrink, double exclusion, int32_t per_step, const double *d_taken,
                                 int32_t T, double *d_props, int32_t *h_count, double *h_max, int64_t *h_queries,
                                 void *stream) {
    if (P < 1 || P > kPoolMax) return fail(BOAC_EINVAL, "P = %d chains outside [1, %d]", P, kPoolMax);
    if (n_global < 1 || n_global > 4096 || n_local < 0 || n_local > 4096)
        return fail(BOAC_EINVAL, "n_global = %d or n_local = %d outside [1, 4096] / [0, 4096]", n_global, n_local);
    if (centres < 1 || q < 1 || per_step < 1 || T < 0)
        return fail(BOAC_EINVAL, "centres, q and per_step must be >= 1 and T >= 0");
    if (!std::isfinite(radius0) || !(radius0 >= 0.0) || !std::isfinite(shrink) || !(shrink >= 0.0) ||
        !std::isfinite(exclusion) || !(exclusion >= 0.0))
        return fail(BOAC_EINVAL, "radius0, shrink and exclusion must be finite and >= 0");
    const long kept = std::min(P, per_step);
    const long npool = kept * ((long)n_global + n_local);
    if (npool > kGreedyMax)
        return fail(BOAC_EINVAL, "pool of %ld entries above %d: fewer rounds or a smaller per_step", npool, kGreedyMax);
    if ((long)n_global * P > (1L << 20)) return fail(BOAC_EINVAL, "n_global x P above 2^20 queries");
    BOAC_TRY(check_ptr(d_z0, "d_z0"));
    BOAC_TRY(check_ptr(d_taken, "d_taken", T == 0));
    BOAC_TRY(check_ptr(d_props, "d_props"));
    if (!h_count || !h_max || !h_queries) return fail(BOAC_EINVAL, "h_count, h_max and h_queries must be given");
    GpEiArgs ag{};
    BOAC_TRY(gp_ei_args(info, d_u, d_linv, d_alpha, n_global * P, best, xi, &ag));
    const int d = ag.d;
    const int nc_max = std::min(std::max(centres, q), P);
    CTX_CHECK();
    const hipStream_t st = (hipStream_t)stream;
    double *z = nullptr, *gpts = nullptr, *gvals = nullptr, *lpts = nullptr, *lvals = nullptr, *pool = nullptr,
           *poolv = nullptr, *C = nullptr, *Ce = nullptr, *vmax = nullptr;
    int *idx = nullptr, *cnt = nullptr;
    BOAC_TRY(ensure_t(ctx, "gs_z", (size_t)P * d, &z));
    BOAC_TRY(ensure_t(ctx, "gs_gpts", (size_t)n_global * P * d, &gpts));
    BOAC_TRY(ensure_t(ctx, "gs_gvals", (size_t)n_global * P, &gvals));
    BOAC_TRY(ensure_t(ctx, "gs_lpts", (size_t)std::max(n_local, 1) * P * d, &lpts));
    BOAC_TRY(ensure_t(ctx, "gs_lvals", (size_t)std::max(n_local, 1) * P, &lvals));
    BOAC_TRY(ensure_t(ctx, "gs_pool", (size_t)npool * d, &pool));
    BOAC_TRY(ensure_t(ctx, "gs_poolv", (size_t)npool, &poolv));
    BOAC_TRY(ensure_t(ctx, "gs_C", (size_t)nc_max * d, &C));
    BOAC_TRY(ensure_t(ctx, "gs_Ce", (size_t)nc_max, &Ce));
    BOAC_TRY(ensure_t(ctx, "gs_idx", (size_t)std::max(q, nc_max), &idx));
    BOAC_TRY(ensure_t(ctx, "gs_cnt", 2, &cnt));
    BOAC_TRY(ensure_t(ctx, "gs_max", 2, &vmax));
    BOAC_TRY(gp_ei_scratch(ctx, &ag));
    // global stage: the chains' points of n_global rounds, their EI in one launch, each round's pool
    HIP_TRY(launch_copy_f64(d_z0, z, P * d, st));
    for (int t = 0; t < n_global; ++t) {
        HIP_TRY(launch_copy_f64(z, gpts + (size_t)t * P * d, P * d, st));
        HIP_TRY(launch_chaos_step(z, P * d, st));
    }
    ag.q = gpts;
    ag.ei = gvals;
    ag.mu = ag.sd = nullptr;
    BOAC_TRY(timed(ctx, BOAC_K_GP, 0.0, st, [&] { return launch_gp_ei(ag, st); }));
    HIP_TRY(launch_pool_top(gpts, gvals, n_global, P, d, per_step, pool, poolv, st));
    // centres: the greedy choice over the global pool; their count fixes the local stage's split
    const int ng = (int)(kept * n_global);
    HIP_TRY(launch_greedy(pool, poolv, ng, d, nullptr, 0, nc_max, exclusion * exclusion, idx, cnt, vmax, st));
    int nc = 0;
    HIP_TRY(hipMemcpyAsync(&nc, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nc < 1) return fail(BOAC_EINVAL, "no finite acquisition value in the global stage");
    HIP_TRY(launch_take_rows(pool, poolv, idx, cnt, nc, d, C, Ce, st));
    // local stage and its pools
    const int M = (P / nc) * nc;
    long long nq = (long long)n_global * P;
    int nl_pool = 0;
    if (n_local > 0) {
        GpEiArgs al{};
        BOAC_TRY(gp_ei_args(info, d_u, d_linv, d_alpha, M, best, xi, &al));
        BOAC_TRY(gp_ei_scratch(ctx, &al));
        BOAC_TRY(chaos_local_rounds(ctx, al, z, P, C, Ce, nc, radius0, shrink, n_local, lpts, lvals, st));
        HIP_TRY(launch_pool_top(lpts, lvals, n_local, M, d, per_step, pool + (size_t)ng * d, poolv + ng, st));
        nl_pool = std::min(M, per_step) * n_local;
        nq += (long long)n_local * M;
    }
    // proposals: the greedy choice over every pool, away from the points taken
    HIP_TRY(launch_greedy(pool, poolv, ng + nl_pool, d, d_taken, T, q, exclusion * exclusion, idx, cnt + 1, vmax + 1,
                          st));
    HIP_TRY(launch_take_rows(pool, nullptr, idx, cnt + 1, q, d, d_props, nullptr, st));
    int count = 0;
    double mx = 0.0;
    HIP_TRY(hipMemcpyAsync(&count, cnt + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&mx, vmax + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *h_count = count;
    *h_max = mx;
    *h_queries = nq;
    return BOAC_OK;
}

// Relative cost of a slice (algorithmic attenuation-tensor passes x tensor size x candidates).
static double slice_cost(const boac_slice &s, int K, int ck) {
    const double V = (double)s.geom.n_angles * s.geom.n_bins * s.geom.n_samples;
    double passes = 2.0 * K + 3.0;
    if (s.d_grad) passes += 2.0 * K * (ck - 1) / std::max(ck, 1) + 4.0 * K + 6.0;
    return V * passes * s.C;
}

// Concurrent stream lanes of a batch (BOAC_BATCH_LANES overrides). Measured on the 48-slice uneven
// batch (graph replays): 2 lanes 1.54 s, 4 lanes 1.45 s, 6 lanes 1.33 s, 8 and 12 lanes 1.26 s.
static int batch_lanes() {
    const char *e = std::getenv("BOAC_BATCH_LANES");
    int n = e ? std::atoi(e) : 8;
    return std::min(std::max(n, 1), 16);
}

static boac_status eval_slice(boac_ctx *ctx, const boac_slice &s, float delta_r, int K, int ck, hipStream_t st) {
    if (s.d_grad)
        return eval_grad(ctx, s.geom, s.d_meas, (const float *)s.d_cand, s.C, delta_r, K, ck, s.d_obj, s.d_grad,
                         s.d_status, st);
    return eval_forward(ctx, s.geom, s.d_meas, (const float *)s.d_cand, s.C, delta_r, K, s.d_obj, nullptr,
                        s.d_status, st);
}

// Batch scheduler: slices are assigned longest-first to the least-loaded of L concurrent stream
// lanes (each with its own scratch namespace); the lanes fork from and join back into the caller's
// stream through events, so a captured batch is one graph with L parallel branches.
// A slice of many candidates can be evaluated as several parts on different lanes, so that a
// projection of one part (bandwidth-bound) overlaps a gather of another (compute-bound). Parts hold at
// least kSplitMinPart candidates (a multiple of 4, which keeps their pointers 16-byte aligned); a slice
// is cut into at most batch_split() of them (BOAC_BATCH_SPLIT, default 1: whole slices). Per-candidate
// arithmetic does not depend on the grouping, so the results are unchanged. Graph replays of the
// 256-candidate batch as one slice: 17.9 ms per step whole, 18.0 ms in 2 parts, 18.6 ms in 4, 18.7 ms
// in 8 (halves gained 5% before opposed-ray pairing halved the projections).
constexpr int kSplitMinPart = 64;

static int batch_split() {
    const char *e = std::getenv("BOAC_BATCH_SPLIT");
    int n = e ? std::atoi(e) : 1;
    return std::min(std::max(n, 1), 16);
}

static std::vector<boac_slice> batch_parts(const boac_slice *h_in, int32_t ns_in, bool split) {
    std::vector<boac_slice> parts;
    for (int i = 0; i < ns_in; ++i) {
        const boac_slice &s = h_in[i];
        const int np = split ? std::min(batch_split(), s.C / kSplitMinPart) : 1;
        if (np < 2) {
            parts.push_back(s);
            continue;
        }
        int c = 0;
        for (int k = 0; k < np; ++k) {
            const int c1 = (k == np - 1) ? s.C : (int)(((long)s.C * (k + 1) / np) & ~3L);
            boac_slice p = s;
            p.C = c1 - c;
            p.d_cand = s.d_cand + c;
            p.d_obj = s.d_obj + c;
            if (s.d_grad) p.d_grad = s.d_grad + (size_t)8 * c;
            if (s.d_status) p.d_status = s.d_status + c;
            parts.push_back(p);
            c = c1;
        }
    }
    return parts;
}

static boac_status batch_body(boac_ctx *ctx, const boac_slice *h_in, int32_t ns_in, float delta_r, int32_t K,
                              int32_t ck, hipStream_t st) {
    const std::vector<boac_slice> parts = batch_parts(h_in, ns_in, batch_lanes() >= 2);
    const boac_slice *h = parts.data();
    const int32_t ns = (int32_t)parts.size();
    const int L = std::min(batch_lanes(), (int)ns);
    if (L <= 1) {
        // the first lane's scratch, not the eager entry points' (a batch and an eager call issued on
        // different streams without ordering between them then do not share buffers)
        ctx->ns = "L0:";
        boac_status rs = BOAC_OK;
        for (int i = 0; i < ns && rs == BOAC_OK; ++i) rs = eval_slice(ctx, h[i], delta_r, K, ck, st);
        ctx->ns.clear();
        return rs;
    }
    while ((int)ctx->lanes.size() < L) {
        if (ctx->capturing) return fail(BOAC_EDEVICE, "lane streams must exist before graph capture");
        hipStream_t s2 = nullptr;
        hipEvent_t e2 = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
        ctx->lanes.push_back(s2);
        ctx->lane_done.push_back(e2);
    }
    if (!ctx->fork) HIP_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    std::vector<int> order(ns);
    for (int i = 0; i < ns; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return slice_cost(h[a], K, ck) > slice_cost(h[b], K, ck); });
    std::vector<double> load(L, 0.0);
    std::vector<std::vector<int>> assign(L);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        assign[l].push_back(i);
        load[l] += slice_cost(h[i], K, ck);
    }
    HIP_TRY(hipEventRecord(ctx->fork, st));
    boac_status rs = BOAC_OK;
    for (int l = 0; l < L && rs == BOAC_OK; ++l) {
        HIP_TRY(hipStreamWaitEvent(ctx->lanes[l], ctx->fork, 0));
        ctx->ns = "L" + std::to_string(l) + ":";
        for (int i : assign[l]) {
            rs = eval_slice(ctx, h[i], delta_r, K, ck, ctx->lanes[l]);
            if (rs != BOAC_OK) break;
        }
        ctx->ns.clear();
    }
    // join every lane back into the caller's stream (also after a failure, so no branch dangles)
    for (int l = 0; l < L; ++l) {
        HIP_TRY(hipEventRecord(ctx->lane_done[l], ctx->lanes[l]));
        HIP_TRY(hipStreamWaitEvent(st, ctx->lane_done[l], 0));
    }
    return rs;
}

// ------------------------------------------------------------------ persistent batch execution
static void drop_stale_graphs(boac_ctx *ctx);

static int persist_lanes() {
    const char *e = std::getenv("BOAC_PERSIST_LANES");
    int n = e ? std::atoi(e) : 8;
    return std::min(std::max(n, 1), 64);
}

// Longest-first assignment of the parts to L lanes.
static std::vector<std::vector<int>> assign_lanes(const std::vector<boac_slice> &h, int L, int K, int ck) {
    std::vector<int> order(h.size());
    for (size_t i = 0; i < h.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return slice_cost(h[a], K, ck) > slice_cost(h[b], K, ck); });
    std::vector<double> load(L, 0.0);
    std::vector<std::vector<int>> assign(L);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        assign[l].push_back(i);
        load[l] += slice_cost(h[i], K, ck);
    }
    return assign;
}

// Records the batch as tasks: the parts are assigned to lanes (each with its own scratch namespace),
// every lane's launches are recorded in order, and the lanes' tasks are interleaved round-robin, each
// task waiting for its predecessor on its lane. lds: the largest item's dynamic LDS.
static boac_status persist_record(boac_ctx *ctx, const boac_slice *h_in, int32_t ns_in, float delta_r, int32_t K,
                                  int32_t ck, std::vector<TaskRec> &out, unsigned &lds) {
    const std::vector<boac_slice> h = batch_parts(h_in, ns_in, true);
    const int L = std::min(persist_lanes(), (int)h.size());
    const auto assign = assign_lanes(h, L, K, ck);
    TaskRecorder rec;
    std::vector<std::vector<TaskRec>> lane_tasks(L);
    task_recorder() = &rec;
    ctx->recording = true;
    ctx->persist_plans = true;
    boac_status rs = BOAC_OK;
    // two passes: the first sizes every scratch buffer (a buffer that grows is reallocated, which would
    // leave earlier tasks with freed pointers), the second records against the final buffers
    for (int pass = 0; pass < 2 && rs == BOAC_OK; ++pass) {
        const uint64_t gen = ctx->scratch_gen;
        rec.unsupported = false;
        for (int l = 0; l < L && rs == BOAC_OK; ++l) {
            rec.tasks.clear();
            rec.lane = l;
            ctx->ns = "P" + std::to_string(l) + ":";
            for (int i : assign[l]) {
                rs = eval_slice(ctx, h[i], delta_r, K, ck, nullptr);
                if (rs != BOAC_OK) break;
            }
            lane_tasks[l] = rec.tasks;
        }
        if (pass == 1 && rs == BOAC_OK && ctx->scratch_gen != gen)
            rs = fail(BOAC_EDEVICE, "internal: scratch grew while recording the persistent batch");
    }
    ctx->ns.clear();
    ctx->recording = false;
    ctx->persist_plans = false;
    task_recorder() = nullptr;
    BOAC_TRY(rs);
    if (rec.unsupported) return fail(BOAC_ENOTSUP, "persistent batch: %s", rec.why);
    out.clear();
    lds = 0;
    std::vector<int> prev(L, -1);
    for (size_t k = 0;; ++k) {
        bool any = false;
        for (int l = 0; l < L; ++l) {
            if (k >= lane_tasks[l].size()) continue;
            any = true;
            TaskRec t = lane_tasks[l][k];
            t.dep = prev[l];
            prev[l] = (int)out.size();
            lds = std::max(lds, t.lds);
            out.push_back(t);
        }
        if (!any) break;
    }
    if (lds > kLdsBudget - 1024)
        return fail(BOAC_ENOTSUP, "persistent batch: an item needs %u bytes of LDS", lds);
    return BOAC_OK;
}

// Waits for the persistent launch and reports an expired dependency wait (or an abort).
static boac_status persist_finish(boac_ctx *ctx, int *state, hipStream_t st) {
    HIP_TRY(hipStreamSynchronize(st));
    int err = 0;
    HIP_TRY(hipMemcpy(&err, state + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (err) return fail(BOAC_ETIMEOUT, "persistent batch: a dependency wait exceeded %lld polls (or was aborted); "
                                        "results are incomplete", ctx->spin_limit);
    return BOAC_OK;
}

static long long persist_spin_limit(const boac_ctx *ctx) { return ctx->spin_limit > 0 ? ctx->spin_limit : (1ll << 26); }

// One persistent launch for the batch; captured into a graph per batch shape and replayed (as the lane
// schedule is). The call waits for the launch, to report BOAC_ETIMEOUT.
static boac_status persist_batch(boac_ctx *ctx, const boac_slice *h_slices, int32_t n_slices, float delta_r,
                                 int32_t K, int32_t ck, hipStream_t st, const std::vector<uint64_t> &key) {
    drop_stale_graphs(ctx);
    for (auto &g : ctx->graphs) {
        if (g.key == key && g.exec) {
            HIP_TRY(hipGraphLaunch(g.exec, st));
            ++ctx->graph_replays;
            return persist_finish(ctx, (int *)g.aux, st);
        }
    }
    std::vector<TaskRec> tasks;
    unsigned lds = 0;
    BOAC_TRY(persist_record(ctx, h_slices, n_slices, delta_r, K, ck, tasks, lds));
    TaskRec *d_tasks = nullptr;
    int *d_state = nullptr;
    BOAC_TRY(ensure_t(ctx, "#persist_tasks", tasks.size(), &d_tasks));
    BOAC_TRY(ensure_t(ctx, "#persist_state", 8 + 9 * tasks.size(), &d_state));
    HIP_TRY(hipMemcpy(d_tasks, tasks.data(), sizeof(TaskRec) * tasks.size(), hipMemcpyHostToDevice));
    PersistArgs pa{d_tasks, (int)tasks.size(), d_state, persist_spin_limit(ctx)};
    HIP_TRY(launch_persist(pa, ctx->n_cu, lds, st));
    BOAC_TRY(persist_finish(ctx, d_state, st));
    if (st == nullptr) return BOAC_OK;  // the null stream cannot be captured
    drop_stale_graphs(ctx);
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    const hipError_t le = launch_persist(pa, ctx->n_cu, lds, st);
    ctx->capturing = false;
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(BOAC_EDEVICE, "persistent batch capture: %s", hipGetErrorString(le != hipSuccess ? le : ce));
    }
    GraphEntry ge;
    ge.key = key;
    ge.scratch_gen = ctx->scratch_gen;
    ge.aux = d_state;
    hipError_t ie = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(BOAC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    if (ctx->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(ge);
    ++ctx->graph_captures;
    return BOAC_OK;
}

// Destroy every cached graph captured under an older scratch generation (its kernels may address
// buffers that were freed when scratch grew since).
static void drop_stale_graphs(boac_ctx *ctx) {
    auto stale = [&](const GraphEntry &g) { return g.scratch_gen != ctx->scratch_gen; };
    for (auto &g : ctx->graphs)
        if (stale(g) && g.exec) (void)hipGraphExecDestroy(g.exec);
    ctx->graphs.erase(std::remove_if(ctx->graphs.begin(), ctx->graphs.end(), stale), ctx->graphs.end());
}

boac_status boac_evaluate_batch(boac_ctx *ctx, const boac_slice *h_slices, int32_t n_slices, float delta_r_cm,
                                int32_t n_iter, int32_t ckpt_every, void *stream) {
    if (!h_slices) return fail(BOAC_EINVAL, "h_slices is NULL");
    if (n_slices < 1 || n_slices > 65536) return fail(BOAC_EINVAL, "n_slices = %d outside [1, 65536]", n_slices);
    for (int i = 0; i < n_slices; ++i) {
        const boac_slice &s = h_slices[i];
        boac_status r = check_geom(&s.geom);
        if (r != BOAC_OK) return fail(r, "slice %d: %s", i, g_last_error.c_str());
        BOAC_TRY(check_count(s.C));
        BOAC_TRY(check_ptr(s.d_meas, "slice d_meas"));
        BOAC_TRY(check_ptr(s.d_cand, "slice d_cand"));
        BOAC_TRY(check_ptr(s.d_obj, "slice d_obj"));
        BOAC_TRY(check_ptr(s.d_grad, "slice d_grad", true));
        BOAC_TRY(check_ptr(s.d_status, "slice d_status", true));
    }
    if (n_iter < 0 || n_iter > 100000) return fail(BOAC_EINVAL, "n_iter = %d outside [0, 100000]", n_iter);
    if (ckpt_every < 1) return fail(BOAC_EINVAL, "ckpt_every = %d must be >= 1", ckpt_every);
    if (!(delta_r_cm > 0.f) || !std::isfinite(delta_r_cm)) return fail(BOAC_EINVAL, "delta_r_cm must be > 0");
    CTX_CHECK();
    hipStream_t st = (hipStream_t)stream;

    // graph key: every pointer and shape of the batch
    std::vector<uint64_t> key;
    key.push_back((uint64_t)n_slices);
    key.push_back((uint64_t)n_iter);
    key.push_back((uint64_t)ckpt_every);
    uint32_t dr;
    std::memcpy(&dr, &delta_r_cm, 4);
    key.push_back(dr);
    key.push_back((uint64_t)(uintptr_t)st);
    for (int i = 0; i < n_slices; ++i) {
        const boac_slice &s = h_slices[i];
        uint32_t px;
        std::memcpy(&px, &s.geom.pixel_cm, 4);
        key.insert(key.end(), {(uint64_t)s.geom.n, (uint64_t)s.geom.n_angles, (uint64_t)s.geom.n_bins,
                               (uint64_t)s.geom.n_samples, px, (uint64_t)s.C, (uint64_t)(uintptr_t)s.d_meas,
                               (uint64_t)(uintptr_t)s.d_cand, (uint64_t)(uintptr_t)s.d_obj,
                               (uint64_t)(uintptr_t)s.d_grad, (uint64_t)(uintptr_t)s.d_status});
    }
    key.push_back((uint64_t)ctx->batch_mode);
    key.push_back((uint64_t)persist_spin_limit(ctx));
    // the schedule's settings (read from the environment on every call)
    key.push_back((uint64_t)batch_lanes());
    key.push_back((uint64_t)batch_split());
    key.push_back((uint64_t)persist_lanes());
    key.push_back(plan_switch_bits());
    if (ctx->batch_mode == BOAC_BATCH_PERSISTENT)
        return persist_batch(ctx, h_slices, n_slices, delta_r_cm, n_iter, ckpt_every, st, key);
    const bool use_graph = (st != nullptr) && !ctx->profiling && std::getenv("BOAC_NO_GRAPH") == nullptr;
    if (!use_graph) return batch_body(ctx, h_slices, n_slices, delta_r_cm, n_iter, ckpt_every, st);

    drop_stale_graphs(ctx);
    for (auto &g : ctx->graphs) {
        if (g.key == key && g.exec) {
            HIP_TRY(hipGraphLaunch(g.exec, st));
            ++ctx->graph_replays;
            return BOAC_OK;
        }
    }
    // first call for this shape: run eagerly (sizes scratch, uploads tables), then capture; graphs of
    // other shapes whose scratch the eager run reallocated are dropped
    BOAC_TRY(batch_body(ctx, h_slices, n_slices, delta_r_cm, n_iter, ckpt_every, st));
    drop_stale_graphs(ctx);
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    boac_status bs = batch_body(ctx, h_slices, n_slices, delta_r_cm, n_iter, ckpt_every, st);
    ctx->capturing = false;
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (bs != BOAC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return bs;
    }
    if (ce != hipSuccess) return fail(BOAC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ce));
    GraphEntry ge;
    ge.key = key;
    ge.scratch_gen = ctx->scratch_gen;
    hipError_t ie = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(BOAC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    if (ctx->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(ge);
    ++ctx->graph_captures;
    // the eager run above already produced this call's results
    return BOAC_OK;
}

boac_status boac_ctx_set_batch_mode(boac_ctx *ctx, int32_t mode, int64_t spin_limit) {
    if (!ctx) return fail(BOAC_EINVAL, "context is NULL");
    if (mode != BOAC_BATCH_LANES && mode != BOAC_BATCH_PERSISTENT)
        return fail(BOAC_EINVAL, "batch mode %d is neither BOAC_BATCH_LANES nor BOAC_BATCH_PERSISTENT", mode);
    ctx->batch_mode = mode;
    ctx->spin_limit = spin_limit > 0 ? (long long)spin_limit : 0;
    return BOAC_OK;
}

boac_status boac_ctx_set_profiling(boac_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(BOAC_EINVAL, "context is NULL");
    ctx->profiling = enable != 0;
    return BOAC_OK;
}

boac_status boac_ctx_kernel_stats(boac_ctx *ctx, int32_t kind, int64_t *count, double *total_ms,
                                  double *total_bytes) {
    if (!ctx) return fail(BOAC_EINVAL, "context is NULL");
    if (kind < 0 || kind >= BOAC_K_COUNT) return fail(BOAC_EINVAL, "kernel kind %d outside [0, %d)", kind, BOAC_K_COUNT);
    HIP_TRY(hipSetDevice(ctx->device));
    BOAC_TRY(drain_timings(ctx));
    if (count) *count = ctx->stat_count[kind];
    if (total_ms) *total_ms = ctx->stat_ms[kind];
    if (total_bytes) *total_bytes = ctx->stat_bytes[kind];
    return BOAC_OK;
}

boac_status boac_ctx_graph_stats(boac_ctx *ctx, int64_t *graphs, int64_t *captures, int64_t *replays,
                                 int64_t *scratch_generation) {
    if (!ctx) return fail(BOAC_EINVAL, "context is NULL");
    if (graphs) *graphs = (int64_t)ctx->graphs.size();
    if (captures) *captures = ctx->graph_captures;
    if (replays) *replays = ctx->graph_replays;
    if (scratch_generation) *scratch_generation = (int64_t)ctx->scratch_gen;
    return BOAC_OK;
}

boac_status boac_ctx_reset_stats(boac_ctx *ctx) {
    if (!ctx) return fail(BOAC_EINVAL, "context is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    BOAC_TRY(drain_timings(ctx));
    for (int k = 0; k < BOAC_K_COUNT; ++k) {
        ctx->stat_count[k] = 0;
        ctx->stat_ms[k] = 0;
        ctx->stat_bytes[k] = 0;
    }
    return BOAC_OK;
}

}  // extern "C"
