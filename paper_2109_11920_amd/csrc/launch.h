// Host-side launch descriptors shared between the kernel translation units and the runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "device_common.h"

namespace boac {

// Row bands of an n x n image, uniform: band i is assigned rows [-1 + i rows, -1 + (i + 1) rows),
// clipped to n + 1; one band (rows = n + 2) when the whole image fits one LDS stage.
struct Bands {
    int count;
    int rows;
    __host__ __device__ Band band(int i, int n) const {
        const int lo = -1 + i * rows;
        const int hi = lo + rows < n + 1 ? lo + rows : n + 1;
        return Band{lo, hi, i == 0, i == count - 1};
    }
};

// A ray-kernel launch covers `cand` candidates of one slice, each with n_angles * n_bins rays split
// in chunks of block * rpt rays.
struct RayCfg {
    int block;   // threads per workgroup (64..1024, multiple of 64)
    int rpt;     // rays per thread (1..4)
    int chunks;  // workgroups per candidate (per candidate pair when pair)
    size_t lds;  // dynamic LDS bytes of one image stage
    bool single; // whole image staged at once
    bool pair;   // forward projection of two candidates per workgroup (single stage, 2 lds bytes)
    int split_chunks;  // > 0: few candidates: the projection (not the likelihood) splits each ray over 8
                       // lanes, 32 rays per 256-thread workgroup, split_chunks workgroups per candidate
    // attenuation build with the scan over 8 lanes per ray (single stage; scan_passes 0 = one thread per
    // ray): scan_block threads, scan_passes rays per lane group, scan_chunks workgroups per candidate
    int scan_block, scan_passes, scan_chunks;
};

enum FwdMode { FWD_PROJ = 0, FWD_RATIO = 1, FWD_NLL = 2 };

struct FwdArgs {
    const float *att;     // [C] attenuation tensors (4 x 8-block slabs, att_row / att_col)
    const float *E;       // opposed-ray pairing: [C][nah][nb] exp(-T) per ray, else null
    const float *img;     // [C][n][n] x img_comps interleaved (component 0 is sampled)
    const float *meas;    // [na][nb]
    float *y_out;         // [C][na][nb] or null
    float *r_out;         // RATIO: r
    float2 *partial;      // NLL: [C][chunks]
    uint32_t *status;     // NLL: [C] or null
    size_t att_cs, img_cs, sino_cs;
    size_t e_cs;          // E stride per candidate
    int img_comps;        // 1 or 2
};

struct SweepArgs {
    const float *att;     // [C] attenuation tensors (4 x 8-block slabs)
    float *attbar;        // [C] adjoint tensors, same layout; written (accumulate = 0) or accumulated
    const float *pair;    // [C][n][n] float2: (bbar^n, F^{n+1})
    const float *r;       // r^n [C][na][nb]
    const float *y;       // y^n
    const float *ybar_in; // pending ybar^{n+1}
    float *ybar_out;      // ybar^n
    size_t att_cs, img_cs, sino_cs;  // img_cs in floats (2 n^2 per candidate)
    int accumulate;
    // opposed-ray pairing (else null): exp(-T) per held ray and its adjoint Ebar (same layout),
    // written (accumulate = 0) or accumulated
    const float *E;
    float *Ebar;
    size_t e_cs;
};

struct TailArgs {
    const float *att;
    float *attbar;        // in: att_bar, out: m_bar
    const float *pair;    // [C][n][n] float2: (s_bar, F^0)
    const float *rho;     // ybar^0 [C][na][nb]
    size_t att_cs, img_cs, sino_cs;
    int accumulate;       // 0: att_bar starts at zero (no MLEM iterations)
    // opposed-ray pairing (else null): exp(-T) per held ray; Ebar in: its accumulated adjoint,
    // out: dx Tbar, the per-ray term every sample of the held ray adds to m_bar
    const float *E;
    float *Ebar;
    size_t e_cs;
};

enum BackMode { BACK_PLAIN = 0, BACK_SENS = 1, BACK_MLEM = 2, BACK_FIELD = 3, BACK_ADJ = 4 };

struct BackCfg {
    int tw, th;           // tile (pixels)
    int ppt;              // pixels per thread (tw*th/256)
    int cg;               // candidates per workgroup
    int hb;               // bin half-window
    int wbmax, wkmax;     // footprint rectangle bound
    int tiles_x, tiles_y; // tiles per image
    size_t lds;
    const int4 *rects;    // [tiles][n_angles] footprint rectangles (b_lo, k_lo, wb, wk)
    const float4 *rectf;  // slid blocks: [tiles][n_angles][2] block origin as floats, (b0 + 1, k0 + 1,
                          // b0 + P - 2, k0 + P - 2) and ((k0 + 1) kSlidPitch + b0 + 1, 0, 0, 0)
    const float4 *angt;   // slid blocks: [n_angles][2] (c, s, c bscale, s bscale), (c / bscale, s / bscale,
                          // 0, 0), each the FP32 product the kernels would form
    int xcd_remap;        // keep a candidate group's tiles on one XCD
    int slid;             // 16 x 16 tiles, one-bin half window: fixed 32 x 32 staging block slid inside
                          // the sinogram; rects then hold (b0, k0, u0 bits, v0 bits). 1: staging by
                          // 4-byte slots; 2: by aligned 4-sample column groups (k0 a multiple of 4)
    int asplit;           // column-group gather: workgroups per (tile, candidate group) splitting the held
                          // angles in whole 8-angle blocks (1 = none; > 1 needs BackArgs::blk_out)
};

constexpr int kSlidBlock = 32;  // staged bins and samples of the slid-block backprojection
constexpr int kSlidPitch = 34;  // its LDS row pitch, in slots

struct BackArgs {
    const float *att;     // [C] attenuation tensors (4 x 8-block slabs)
    const float *E;       // opposed-ray pairing: [C][nah][nb] exp(-T) per ray, else null
    const float *z;       // PLAIN/MLEM/ADJ: per-ray weights [C][na][nb]; FIELD: [C] per-sample field, att layout
    const float *F;       // MLEM: current image
    const float *s;       // MLEM: sensitivity
    const float *aux;     // ADJ: direct part of F_bar
    float *out;           // [C][n][n]
    float *q_out;         // MLEM: update factor b/s (nullable)
    float *blk_out;       // angle split: [ceil(nah / 8)][C][img_cs] per-8-angle-block sums (else null)
    size_t att_cs, sino_cs, img_cs;
    size_t e_cs;          // E stride per candidate
    int C;
};

struct AdjElemArgs {
    const float *fbar;    // F_bar^{n+1}
    const float *F;       // F^n
    const float *Q;       // Q^n
    const float *s;       // sensitivity
    float *sbar;          // accumulated s_bar (read-modify-write)
    float2 *pair;         // out: (bbar^n, F^{n+1}) interleaved
    float *fbar_direct;   // out
    size_t img_cs;
    int npix, C;
};

// Acquisition of the surrogate at M queries (kernels_gp.hip), FP64.
struct GpEiArgs {
    const double *u;      // [n][d] observations, unit-box coordinates
    const double *linv;   // [n][n] inverse of the Cholesky factor (lower)
    const double *alpha;  // [n] K^-1 z
    const double *q;      // [M][d] queries
    int n, d, M;
    int npad;             // K* row stride (n rounded up to 64)
    int nti;              // row blocks of 64 in X
    double inv2l2, amp, m0, s, best, xi;
    double *ks;           // scratch [M][npad]
    double *part;         // scratch [nti][M]
    double *mu, *sd;      // [M] or NULL
    double *ei;           // [M]
};

// Raster-adjoint components per candidate: c_0..c_5, mu_b, mu_c, dR.
constexpr int kGradComps = 9;

// ---- persistent execution of a recorded launch sequence (kernels_persist.hip) ----
// While a TaskRecorder is installed on the calling thread, every launcher below records its launch as a
// task instead of launching it. The persistent executor then runs the tasks in one launch: workgroups
// of kPersistThreads threads take work items from a queue in device memory, each task waiting for its
// predecessor on the same lane (the order a stream would give). Ray-kernel tasks run a recorded
// 1024-thread workgroup per item; 256-thread tasks run four recorded workgroups per item.
constexpr int kPersistThreads = 1024;
constexpr int kPersistElems = 16384;  // elements per item of an elementwise task

enum TaskKind : int {
    T_RASTER = 0, T_RASTER_ADJ, T_ATT, T_ATT_SCAN, T_FWD, T_FWD_PAIR, T_SWEEP, T_TAIL, T_BACK_COL4,
    T_FILL, T_FILL_U32, T_MUL_COPY, T_COPY, T_YBAR, T_LGAMMA, T_NLL_FINISH, T_ADJ_ELEM, T_PACK_PAIR,
    T_GRAD_FINISH, T_KINDS
};

struct RayTask {
    DevGeom g;
    Bands bands;
    int rpt, chunks, C;
};

struct TaskRec {
    int kind;
    int variant;       // template switches of the recorded kernel (see kernels_persist.hip)
    int grid;          // workgroups of the recorded launch
    int items;         // work items of the persistent executor
    int dep;           // task whose completion this one waits for (-1: none)
    int lane;          // lane of the recorded sequence
    unsigned lds;      // dynamic LDS bytes of one item (all of its recorded workgroups)
    unsigned sub_lds;  // 256-thread tasks: dynamic LDS bytes of one recorded workgroup
    union {
        struct { DevGeom g; const float *cand; float delta_r; float *mu; size_t img_cs; uint32_t *status; int nbx; } raster;
        struct { DevGeom g; const float *cand; float delta_r; const float *mubar; size_t img_cs; float *grad; } raster_adj;
        struct { RayTask r; const float *mu; float *att; size_t img_cs, att_cs; float *E; size_t e_cs; int passes; } att;
        struct { RayTask r; FwdArgs A; } fwd;
        struct { RayTask r; SweepArgs A; } sweep;
        struct { RayTask r; TailArgs A; } tail;
        struct { DevGeom g; BackCfg T; BackArgs A; int mode; } back;
        struct { void *out; const void *a; const void *b; size_t count; float fa, fb; uint32_t u; } elem;
        struct { const float *meas; const float *yK; float *ybar; int C, nrays; size_t sino_cs; } ybar;
        struct { const float *meas; int count; float2 *out; uint32_t *flag; } lgamma;
        struct { const float2 *partial; int chunks, C; const float2 *lg; const uint32_t *flag; float *obj; uint32_t *status; } nll;
        AdjElemArgs adj;
        struct { const float *grad; int C, ncomp; float *d_grad; uint32_t *status; } gfin;
    } u;
};

struct TaskRecorder {
    std::vector<TaskRec> tasks;
    int lane = 0;
    bool unsupported = false;  // a launch the executor cannot run was requested
    const char *why = "";
};
// The calling thread's recorder (null: launchers launch).
TaskRecorder *&task_recorder();
// Records t (dep and lane are set by the recorder's owner); always hipSuccess.
hipError_t record_task(TaskRecorder *r, const TaskRec &t);
hipError_t record_unsupported(TaskRecorder *r, const char *why);

struct PersistArgs {
    const TaskRec *tasks;
    int ntasks;
    int *state;            // [8 + 9 ntasks]: queue head, error, abort, ...; per-XCD claims [8 ntasks]; done [ntasks]
    long long spin_limit;  // polls of an unfinished dependency before the executor gives up (error 1)
};
// Zeroes the queue state and runs the recorded tasks in one persistent launch of `workgroups`
// workgroups with `lds` bytes of dynamic LDS each.
hipError_t launch_persist(const PersistArgs &a, int workgroups, unsigned lds, hipStream_t st);

// ---- launchers (each returns the hipError_t of the launch) ----
hipError_t launch_raster(const DevGeom &g, const float *cand, int C, float delta_r, float *mu, size_t img_cs,
                         uint32_t *status, hipStream_t st);
// grad: [C][kGradComps] partial gradients
hipError_t launch_raster_adj(const DevGeom &g, const float *cand, int C, float delta_r, const float *mubar,
                             size_t img_cs, float *grad, hipStream_t st);
// E: with opposed-ray pairing (g.nah < g.na) exp(-T) per ray [C][nah][nb] (stride e_cs), else null
hipError_t launch_att(const DevGeom &g, const RayCfg &rc, const Bands &bands, const float *mu, float *att,
                      size_t img_cs, size_t att_cs, float *E, size_t e_cs, int C, hipStream_t st);
hipError_t launch_fwd(int mode, const DevGeom &g, const RayCfg &rc, const Bands &bands, const FwdArgs &a, int C,
                      hipStream_t st);
hipError_t launch_adj_sweep(const DevGeom &g, const RayCfg &rc, const Bands &bands, const SweepArgs &a, int C,
                            hipStream_t st);
hipError_t launch_pack_pair(const float *a, float a_const, const float *b, float b_const, float2 *out, size_t count,
                            hipStream_t st);
hipError_t launch_tail(const DevGeom &g, const RayCfg &rc, const Bands &bands, const TailArgs &a, int C,
                       hipStream_t st);
hipError_t launch_back(int mode, const DevGeom &g, const BackCfg &bc, const BackArgs &a, hipStream_t st);
hipError_t launch_fill(float *p, size_t count, float v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t st);
// The likelihood's measurement-only constant (FP64). out holds kLgammaOut float2: out[0] receives the
// constant as (value, remainder), the rest the per-workgroup partial sums (doubles).
constexpr int kLgammaParts = 32;
constexpr int kLgammaOut = 2 + 2 * kLgammaParts;
hipError_t launch_lgamma_sum(const float *meas, int count, float2 *out, uint32_t *flag, hipStream_t st);
hipError_t launch_nll_finish(const float2 *partial, int chunks, int C, const float2 *lg, const uint32_t *meas_flag,
                             float *obj, uint32_t *status, hipStream_t st);
hipError_t launch_adj_elem(const AdjElemArgs &a, hipStream_t st);
hipError_t launch_grad_finish(const float *grad, int C, int ncomp, float *d_grad, uint32_t *status, hipStream_t st);
hipError_t launch_mul_copy(const float *a, const float *b, float *out, size_t count, hipStream_t st);
hipError_t launch_copy(const float *src, float *dst, size_t count, hipStream_t st);
hipError_t launch_gp_ei(const GpEiArgs &a, hipStream_t st);
hipError_t launch_chaos_points(const double *z, const double *C, double r, int per, int nc, int d, double *U,
                               hipStream_t st);
hipError_t launch_chaos_centres(const double *U, const double *e, int per, int nc, int d, double *C, double *Ce,
                                hipStream_t st);
hipError_t launch_chaos_step(double *z, int count, hipStream_t st);
// Pools and greedy choice of the acquisition search (kernels_gp.hip)
constexpr int kPoolMax = 8192;     // values per round a pool is taken from
constexpr int kGreedyMax = 32768;  // pool entries of one greedy choice
hipError_t launch_pool_top(const double *pts, const double *vals, int rounds, int M, int d, int keep, double *pool_pts,
                           double *pool_vals, hipStream_t st);
hipError_t launch_greedy(const double *pts, const double *vals, int N, int d, const double *taken, int T, int q,
                         double ex2, int *idx, int *count, double *vmax, hipStream_t st);
hipError_t launch_take_rows(const double *src, const double *vsrc, const int *idx, const int *count, int rows, int d,
                            double *dst, double *vdst, hipStream_t st);
hipError_t launch_copy_f64(const double *src, double *dst, int n, hipStream_t st);
hipError_t launch_ybar_final(const float *meas, const float *yK, float *ybar, int C, int nrays, size_t sino_cs,
                             hipStream_t st);

}  // namespace boac
