// Persistent executor of a recorded launch sequence (BOAC step 3 for many candidate sets in one launch).
//
// This translation unit includes the kernel sources for their bodies only (BOAC_BODIES_ONLY: the
// kernels and launchers themselves are compiled in their own translation units, whose code generation
// the persistent kernel must not change), so every body can be inlined into one persistent kernel. The runtime records a batch's launches as tasks (TaskRecorder, launch.h), each
// with the task it must wait for (its predecessor on the same lane). k_persist then runs them all in one
// launch of one 1024-thread workgroup per CU:
//
//   queue    tasks are taken in order: a workgroup claims an item of the task at the queue head with a
//            vector atomic on that task's claim counter for its XCD (items are split over the 8 XCDs by
//            index; a workgroup takes its own XCD's items first, then another's), and moves the head
//            past a task once all its items are claimed;
//   waiting  before running an item the workgroup waits until its task's predecessor has completed
//            every item (a done counter per task, incremented with release semantics after an item's
//            writes; read with acquire semantics). A predecessor always sits earlier in the queue, and a
//            workgroup claims only from the head, so every item it waits for was claimed by a running
//            workgroup: the wait ends. It is bounded all the same: after spin_limit polls, or when the
//            host sets the abort word, the executor records an error and every workgroup leaves;
//   items    a ray-kernel item is one recorded 1024-thread workgroup; a gather or rasteriser item is
//            four recorded 256-thread workgroups, each on its own quarter of the threads and of the LDS
//            (a stand-in takes part in the barriers when the grid runs out); elementwise items cover
//            kPersistElems elements; the small reductions run on the whole workgroup.
#define BOAC_BODIES_ONLY
#include "kernels_ray.hip"
#include "kernels_back.hip"
#include "kernels_misc.hip"

namespace boac {

TaskRecorder *&task_recorder() {
    static thread_local TaskRecorder *r = nullptr;
    return r;
}

hipError_t record_task(TaskRecorder *r, const TaskRec &t) {
    TaskRec c = t;
    c.lane = r->lane;
    c.dep = -1;
    r->tasks.push_back(c);
    return hipSuccess;
}

hipError_t record_unsupported(TaskRecorder *r, const char *why) {
    r->unsupported = true;
    r->why = why;
    return hipSuccess;
}

__device__ __forceinline__ int ld_acquire(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One 256-thread recorded workgroup per quarter of the executor's threads: its index among the task's
// workgroups, or -1 beyond the grid.
__device__ __forceinline__ int quarter_block(int item, int grid) {
    const int vb = item * 4 + (int)(threadIdx.x >> 8);
    return vb < grid ? vb : -1;
}

template <int CG, bool W, bool P>
__device__ __forceinline__ void run_col4(const TaskRec &T, int item, float *lds) {
    const int vb = quarter_block(item, T.grid);
    float *l = lds + (threadIdx.x >> 8) * (T.sub_lds / 4);
    k_back_col4_body<CG, W, P, false>(vb >= 0 ? vb : T.grid - 1, threadIdx.x & 255, l, vb >= 0, T.u.back.g,
                                      T.u.back.T, T.u.back.A, T.u.back.mode);
}

template <bool W, bool P>
__device__ __forceinline__ void run_col4_cg(const TaskRec &T, int item, float *lds) {
    switch (T.variant & 3) {
        case 0: run_col4<1, W, P>(T, item, lds); break;
        case 1: run_col4<2, W, P>(T, item, lds); break;
        default: run_col4<4, W, P>(T, item, lds); break;
    }
}

template <int MODE>
__device__ __forceinline__ void run_fwd(const TaskRec &T, int item, float *lds, float *red) {
    const RayTask &r = T.u.fwd.r;
    const bool single = (T.variant & 4) != 0, paired = (T.variant & 8) != 0;
    if (T.kind == T_FWD_PAIR) {
        if (paired)
            k_fwd_pair_body<MODE, true>(item, lds, red, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.fwd.A);
        else
            k_fwd_pair_body<MODE, false>(item, lds, red, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.fwd.A);
    } else if (single) {
        if (paired)
            k_fwd_body<MODE, true, true>(item, lds, red, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.fwd.A);
        else
            k_fwd_body<MODE, true, false>(item, lds, red, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.fwd.A);
    } else {
        if (paired)
            k_fwd_body<MODE, false, true>(item, lds, red, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.fwd.A);
        else
            k_fwd_body<MODE, false, false>(item, lds, red, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.fwd.A);
    }
}

// Elements [e0, e1) of an elementwise task, strided over the workgroup.
__device__ __forceinline__ void run_elem(const TaskRec &T, size_t e0, size_t e1) {
    const auto &E = T.u.elem;
    for (size_t e = e0 + threadIdx.x; e < e1; e += kPersistThreads) {
        switch (T.kind) {
            case T_FILL: static_cast<float *>(E.out)[e] = E.fa; break;
            case T_FILL_U32: static_cast<uint32_t *>(E.out)[e] = E.u; break;
            case T_MUL_COPY:
                static_cast<float *>(E.out)[e] = static_cast<const float *>(E.a)[e] * static_cast<const float *>(E.b)[e];
                break;
            case T_COPY: static_cast<float *>(E.out)[e] = static_cast<const float *>(E.a)[e]; break;
            case T_PACK_PAIR:
                static_cast<float2 *>(E.out)[e] =
                    make_float2(E.a ? static_cast<const float *>(E.a)[e] : E.fa, E.b ? static_cast<const float *>(E.b)[e] : E.fb);
                break;
            default: break;
        }
    }
}

__device__ void run_task(const TaskRec &T, int item, float *lds, float *red) {
    switch (T.kind) {
        case T_RASTER: {
            const int vb = quarter_block(item, T.grid);
            const auto &R = T.u.raster;
            if (vb >= 0) {
                const int cidx = vb / R.nbx;
                raster_at(R.g, R.cand, R.delta_r, R.mu, R.img_cs, R.status, cidx,
                          (vb - cidx * R.nbx) * 256 + (int)(threadIdx.x & 255));
            }
            break;
        }
        case T_RASTER_ADJ: {
            const auto &R = T.u.raster_adj;
            k_raster_adj_body(item, red, R.g, R.cand, R.delta_r, R.mubar, R.img_cs, R.grad);
            break;
        }
        case T_ATT: {
            const auto &A = T.u.att;
            if (T.variant & 1)
                k_att_body<true>(item, lds, A.r.g, A.r.bands, A.r.rpt, A.r.chunks, A.r.C, A.mu, A.att, A.img_cs,
                                 A.att_cs, A.E, A.e_cs);
            else
                k_att_body<false>(item, lds, A.r.g, A.r.bands, A.r.rpt, A.r.chunks, A.r.C, A.mu, A.att, A.img_cs,
                                  A.att_cs, A.E, A.e_cs);
            break;
        }
        case T_ATT_SCAN: {
            const auto &A = T.u.att;
            k_att_scan_body(item, lds, A.r.g, A.r.bands.band(0, A.r.g.n), A.passes, A.r.chunks, A.r.C, A.mu, A.att, A.img_cs,
                            A.att_cs, A.E, A.e_cs);
            break;
        }
        case T_FWD:
        case T_FWD_PAIR:
            switch (T.variant & 3) {
                case FWD_PROJ: run_fwd<FWD_PROJ>(T, item, lds, red); break;
                case FWD_RATIO: run_fwd<FWD_RATIO>(T, item, lds, red); break;
                default: run_fwd<FWD_NLL>(T, item, lds, red); break;
            }
            break;
        case T_SWEEP: {
            const RayTask &r = T.u.sweep.r;
            switch (T.variant & 3) {
                case 0: k_adj_sweep_body<false, false>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.sweep.A); break;
                case 1: k_adj_sweep_body<true, false>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.sweep.A); break;
                case 2: k_adj_sweep_body<false, true>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.sweep.A); break;
                default: k_adj_sweep_body<true, true>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.sweep.A); break;
            }
            break;
        }
        case T_TAIL: {
            const RayTask &r = T.u.tail.r;
            switch (T.variant & 3) {
                case 0: k_tail_body<false, false>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.tail.A); break;
                case 1: k_tail_body<true, false>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.tail.A); break;
                case 2: k_tail_body<false, true>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.tail.A); break;
                default: k_tail_body<true, true>(item, lds, r.g, r.bands, r.rpt, r.chunks, r.C, T.u.tail.A); break;
            }
            break;
        }
        case T_BACK_COL4:
            switch ((T.variant >> 2) & 3) {
                case 0: run_col4_cg<false, false>(T, item, lds); break;
                case 1: run_col4_cg<true, false>(T, item, lds); break;
                case 2: run_col4_cg<false, true>(T, item, lds); break;
                default: run_col4_cg<true, true>(T, item, lds); break;
            }
            break;
        case T_YBAR: {
            const auto &Y = T.u.ybar;
            const size_t total = (size_t)Y.C * Y.nrays;
            const size_t e0 = (size_t)item * kPersistElems, e1 = min(total, e0 + kPersistElems);
            for (size_t e = e0 + threadIdx.x; e < e1; e += kPersistThreads)
                ybar_final_at(Y.meas, Y.yK, Y.ybar, Y.nrays, Y.sino_cs, e);
            break;
        }
        case T_ADJ_ELEM: {
            const size_t total = (size_t)T.u.adj.npix * T.u.adj.C;
            const size_t e0 = (size_t)item * kPersistElems, e1 = min(total, e0 + kPersistElems);
            for (size_t e = e0 + threadIdx.x; e < e1; e += kPersistThreads) adj_elem_at(T.u.adj, e);
            break;
        }
        case T_LGAMMA:
            k_lgamma_sum_body(red, T.u.lgamma.meas, T.u.lgamma.count, T.u.lgamma.out, T.u.lgamma.flag);
            break;
        case T_NLL_FINISH: {
            const auto &N = T.u.nll;
            nll_finish_at(N.partial, N.chunks, N.C, N.lg, N.flag, N.obj, N.status,
                          item * kPersistThreads + (int)threadIdx.x);
            break;
        }
        case T_GRAD_FINISH: {
            const auto &G = T.u.gfin;
            grad_finish_at(G.grad, G.C, G.ncomp, G.d_grad, G.status, item * kPersistThreads + (int)threadIdx.x);
            break;
        }
        default: {
            const size_t e0 = (size_t)item * kPersistElems;
            run_elem(T, e0, min(T.u.elem.count, e0 + kPersistElems));
            break;
        }
    }
}

__global__ __launch_bounds__(kPersistThreads) void k_persist(const TaskRec *__restrict__ tasks, int ntasks,
                                                            int *__restrict__ state, long long spin_limit) {
    extern __shared__ float lds[];
    __shared__ __align__(8) float red[32];  // 32 floats or 16 doubles
    __shared__ int s_task, s_item;
    int *head = state, *err = state + 1, *abort_word = state + 2;
    int *claimed = state + 8, *done = state + 8 + 8 * ntasks;
    const int xcd = (int)(blockIdx.x & 7);
    while (true) {
        if (threadIdx.x == 0) {
            int t = -1, item = -1;
            int c = ld_relaxed(head);
            while (c < ntasks) {
                if (ld_relaxed(err) || ld_relaxed(abort_word)) break;
                const int items = tasks[c].items;
                for (int d = 0; d < 8 && item < 0; ++d) {
                    const int x = (xcd + d) & 7;
                    const int cnt = (items - x + 7) >> 3;  // items x, x + 8, ... of the task
                    if (cnt <= 0 || ld_relaxed(&claimed[8 * c + x]) >= cnt) continue;
                    const int k = atomicAdd(&claimed[8 * c + x], 1);
                    if (k < cnt) item = x + 8 * k;
                }
                if (item >= 0) {
                    t = c;
                    break;
                }
                atomicCAS(head, c, c + 1);  // every item of task c is claimed: the head moves on
                c = ld_relaxed(head);
            }
            if (t >= 0) {
                const int dep = tasks[t].dep;
                if (dep >= 0) {
                    const int need = tasks[dep].items;
                    long long polls = 0;
                    while (ld_acquire(&done[dep]) < need) {
                        if (ld_relaxed(err) || ld_relaxed(abort_word)) {
                            t = -1;
                            break;
                        }
                        if (++polls > spin_limit) {
                            atomicOr(err, 1);
                            t = -1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(4);
                    }
                }
            }
            s_task = t;
            s_item = item;
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_task), item = __builtin_amdgcn_readfirstlane(s_item);
        if (t < 0) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the predecessor's results, seen by every wave
        run_task(tasks[t], item, lds, red);
        __syncthreads();  // every wave's writes of this item are issued
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&done[t], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // s_task and s_item are rewritten only after every wave has read them
    }
}

// Zeroes the executor's queue state (a kernel, not a memset: the launch may be captured into a graph).
__global__ void k_persist_zero(int *state, size_t words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        state[i] = 0;
}

hipError_t launch_persist(const PersistArgs &a, int workgroups, unsigned lds, hipStream_t st) {
    const size_t words = 8 + 9 * (size_t)a.ntasks;
    hipLaunchKernelGGL(k_persist_zero, dim3((unsigned)std::min<size_t>(1024, (words + 255) / 256)), dim3(256), 0, st,
                       a.state, words);
    hipLaunchKernelGGL(k_persist, dim3((unsigned)workgroups), dim3(kPersistThreads), lds, st, a.tasks, a.ntasks, a.state,
                       a.spin_limit);
    return hipGetLastError();
}

}  // namespace boac
