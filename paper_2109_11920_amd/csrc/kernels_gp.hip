// Acquisition of the BOAC outer loop on the device, FP64: posterior mean, standard deviation and
// expected improvement (Eqs. 7-10, minimisation) of a fitted GP at M query points.
//
// With k*_m = k(q_m, u_.) (Eq. 8), the GP weights alpha = K^-1 z and X = L^-1 (K = L L^T):
//   mu_m = m0 + s k*_m . alpha,   var_m = s^2 (amp - |X k*_m|^2),
//   gamma = (J_best - mu - xi) / sigma,  EI = sigma (gamma Phi(gamma) + phi(gamma)).
// |X k*_m|^2 for all m is a triangular matrix product Z = X K*^T (n x M) reduced over its rows:
//   k_gp_kstar  K* [M][npad] (zero past n)
//   k_gp_zsq    per (64-row block of X, 64-query block): the Z block over j <= i on the FP64 matrix
//               cores, squared and summed over its rows -> part [n/64][M] (fixed order, no atomics)
//   k_gp_ei     one wave per query: k* . alpha, sum of the row-block partials, EI
#include "launch.h"

namespace boac {

constexpr int kGpT = 64;   // rows of X and queries per block
constexpr int kGpJ = 16;   // columns per staging step

__global__ __launch_bounds__(256) void k_gp_kstar(GpEiArgs A) {
    const size_t total = (size_t)A.M * A.npad;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(t / A.npad), j = (int)(t - (size_t)m * A.npad);
        double k = 0.0;
        if (j < A.n) {
            double d2 = 0.0;
            for (int c = 0; c < A.d; ++c) {
                const double e = A.q[(size_t)m * A.d + c] - A.u[(size_t)j * A.d + c];
                d2 = fma(e, e, d2);
            }
            k = A.amp * exp(-d2 * A.inv2l2);
        }
        A.ks[t] = k;
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Z block on the FP64 matrix cores: D[16 x 16] += A[16 x 4] B[4 x 16] per v_mfma_f64_16x16x4f64, with
// lane l holding A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4 v][l % 16] (v = 0..3).
// Wave w of the 4 takes queries m0 + 16 w .. + 15 and all 64 rows (4 row tiles of 16): A = X rows,
// B = K*^T, so D[i][m] = sum_j X[i][j] K*[m][j]. X and K* pass through LDS 16 columns at a time.
__global__ __launch_bounds__(256) void k_gp_zsq(GpEiArgs A) {
    __shared__ double Xs[kGpJ][kGpT + 1];  // X[i0 + r][j0 + c] at [c][r]
    __shared__ double Ks[kGpJ][kGpT + 1];  // K*[m0 + r][j0 + c] at [c][r]
    __shared__ double red[4][kGpT];
    const int i0 = blockIdx.x * kGpT, m0 = blockIdx.y * kGpT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    v4d acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    // X is lower triangular: row block [i0, i0 + 64) needs columns j < min(i0 + 64, n)
    const int jend = min(i0 + kGpT, A.n);
    for (int j0 = 0; j0 < jend; j0 += kGpJ) {
        for (int e = threadIdx.x; e < kGpT * kGpJ; e += blockDim.x) {
            const int r = e / kGpJ, c = e - r * kGpJ;
            const int i = i0 + r, m = m0 + r, j = j0 + c;
            Xs[c][r] = (i < A.n && j < A.n) ? A.linv[(size_t)i * A.n + j] : 0.0;
            Ks[c][r] = (m < A.M && j < A.npad) ? A.ks[(size_t)m * A.npad + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGpJ; kk += 4) {
            const double b = Ks[kk + lk][16 * w + lr];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[kk + lk][16 * t + lr], b, acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    // this lane: query m0 + 16 w + lr, rows 16 t + lk + 4 v; sum of squares over its 16 rows
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) s = fma(acc[t][v], acc[t][v], s);
    red[lk][16 * w + lr] = s;
    __syncthreads();
    if (threadIdx.x < kGpT) {
        const double q = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
        const int m = m0 + threadIdx.x;
        if (m < A.M) A.part[(size_t)blockIdx.x * A.M + m] = q;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(256) void k_gp_ei(GpEiArgs A) {
    const int lane = threadIdx.x & 63;
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= A.M) return;  // uniform per wave
    double a = 0.0;
    for (int j = lane; j < A.n; j += 64) a = fma(A.ks[(size_t)m * A.npad + j], A.alpha[j], a);
    a = wave_sum(a);
    double q = 0.0;
    for (int t = lane; t < A.nti; t += 64) q += A.part[(size_t)t * A.M + m];
    q = wave_sum(q);
    if (lane == 0) {
        const double mu = A.m0 + A.s * a;
        const double var = A.amp - q;
        const double sd = A.s * sqrt(var > 0.0 ? var : 0.0);
        const double imp = A.best - mu - A.xi;
        double ei;
        if (sd > 0.0) {
            const double g = imp / sd;
            const double cdf = 0.5 * erfc(-g * 0.70710678118654752440);
            const double pdf = 0.39894228040143267794 * exp(-0.5 * g * g);
            // g Phi(g) + phi(g) > 0, but for g far below 0 its two terms cancel and rounding can leave a
            // tiny negative: EI, the mean of a non-negative improvement, is clamped at 0
            ei = sd * fma(g, cdf, pdf);
            if (!(ei > 0.0)) ei = 0.0;
        } else {
            ei = imp > 0.0 ? imp : 0.0;
        }
        if (A.mu) A.mu[m] = mu;
        if (A.sd) A.sd[m] = sd;
        A.ei[m] = ei;
    }
}

// ------------------------------------------------------------------ acquisition search, local stage
// (Bayesian Optimization, step 5: chaotic search). Per round: the query points of every centre's chains,
// U = clip(C_c + r (2 z - 1), 0, 1) in FP64 with the host search's operation order (no contraction), so
// the device search takes the same points as one run on the host; after the EI kernels, each centre
// moves to the first of its chains' best points when that beats its value; then z <- 4 z (1 - z).
__global__ __launch_bounds__(256) void k_chaos_points(const double *__restrict__ z, const double *__restrict__ C,
                                                      double r, int per, int d, int count, double *__restrict__ U) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;  // element of U [nc * per][d]; z rows match U rows
    if (t >= count) return;
    const int row = t / d, k = t - row * d;
    const double w = 2.0 * z[t] - 1.0;
    const double v = C[(row / per) * d + k] + r * w;
    const double m = v > 0.0 ? v : 0.0;  // clip to [0, 1] as max then min, comparisons only
    U[t] = m < 1.0 ? m : 1.0;
}

__global__ __launch_bounds__(256) void k_chaos_centres(const double *__restrict__ U, const double *__restrict__ e,
                                                       int per, int nc, int d, double *__restrict__ C,
                                                       double *__restrict__ Ce) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *ec = e + (size_t)c * per;
    int j = 0;
    double best = ec[0];
    for (int k = 1; k < per; ++k)
        if (ec[k] > best) {
            best = ec[k];
            j = k;
        }
    if (best > Ce[c]) {
        Ce[c] = best;
        for (int k = 0; k < d; ++k) C[(size_t)c * d + k] = U[((size_t)c * per + j) * d + k];
    }
}

__global__ __launch_bounds__(256) void k_chaos_step(double *__restrict__ z, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double v = z[t];
    z[t] = (4.0 * v) * (1.0 - v);
}

// ------------------------------------------------------------------ pools and greedy choice
// The order of the search's selections: larger value first, lower index on ties (as a stable sort in
// decreasing value). Values are taken to be finite.
__device__ __forceinline__ bool ranks_before(double va, int ia, double vb, int ib) {
    return va > vb || (va == vb && ia < ib);
}

// Bitonic sort of n = 2^k (value, index) pairs in LDS by ranks_before (by_index: indices ascending).
__device__ void lds_bitonic(double *sv, int *si, int n, bool by_index) {
    for (int k = 2; k <= n; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < n; t += blockDim.x) {
                const int u = t ^ j;
                if (u <= t) continue;
                const bool asc = (t & k) == 0;  // this pair's run is ordered ascending in rank
                const bool ut = by_index ? si[u] < si[t] : ranks_before(sv[u], si[u], sv[t], si[t]);
                const bool tu = by_index ? si[t] < si[u] : ranks_before(sv[t], si[t], sv[u], si[u]);
                if (asc ? ut : tu) {
                    const double v = sv[t];
                    sv[t] = sv[u];
                    sv[u] = v;
                    const int i = si[t];
                    si[t] = si[u];
                    si[u] = i;
                }
            }
            __syncthreads();
        }
}

// One workgroup per round: the `keep` highest-ranked of the round's M values, written in index order
// (values and their points) to the round's pool slot of min(M, keep) entries. M <= kPoolMax.
__global__ __launch_bounds__(1024) void k_pool_top(const double *__restrict__ pts, const double *__restrict__ vals,
                                                   int M, int d, int keep, double *__restrict__ pool_pts,
                                                   double *__restrict__ pool_vals) {
    __shared__ double sv[kPoolMax];
    __shared__ int si[kPoolMax];
    const int r = blockIdx.x;
    const int kept = M < keep ? M : keep;
    const double *v = vals + (size_t)r * M;
    const double *p = pts + (size_t)r * M * d;
    double *ov = pool_vals + (size_t)r * kept;
    double *op = pool_pts + (size_t)r * kept * d;
    if (M > keep) {
        int n = 1;
        while (n < M) n <<= 1;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            sv[t] = t < M ? v[t] : -INFINITY;
            si[t] = t < M ? t : 0x7fffffff;
        }
        __syncthreads();
        lds_bitonic(sv, si, n, false);
        // the first `keep` are the selection; put them back in index order
        int m = 1;
        while (m < keep) m <<= 1;
        for (int t = keep + threadIdx.x; t < m; t += blockDim.x) si[t] = 0x7fffffff;
        __syncthreads();
        lds_bitonic(sv, si, m, true);
    } else {
        for (int t = threadIdx.x; t < M; t += blockDim.x) si[t] = t;
        __syncthreads();
    }
    for (int t = threadIdx.x; t < kept * d; t += blockDim.x) {
        const int row = t / d, k = t - row * d;
        op[t] = p[(size_t)si[row] * d + k];
    }
    for (int t = threadIdx.x; t < kept; t += blockDim.x) ov[t] = v[si[t]];
}

// Squared distance of two d-vectors, in coordinate order.
__device__ __forceinline__ double dist2(const double *a, const double *b, int d) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        const double e = a[k] - b[k];
        s += e * e;
    }
    return s;
}

// One workgroup: up to q pool entries in rank order, each at least sqrt(ex2) from the rows of `taken`
// and from the entries chosen before it (a greedy choice: the best remaining entry is chosen and every
// entry nearer than the exclusion to it is dropped). idx[0..count) receive the choices in order; *vmax
// the largest pool value. N <= kGreedyMax.
__global__ __launch_bounds__(1024) void k_greedy(const double *__restrict__ pts, const double *__restrict__ vals,
                                                 int N, int d, const double *__restrict__ taken, int T, int q,
                                                 double ex2, int *__restrict__ idx, int *__restrict__ count,
                                                 double *__restrict__ vmax) {
    __shared__ unsigned char alive[kGreedyMax];
    __shared__ double wv[32];
    __shared__ int wi[32];
    __shared__ int pick;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    double mx = -INFINITY;
    for (int i = tid; i < N; i += blockDim.x) {
        const double *pi = pts + (size_t)i * d;
        bool ok = true;
        for (int t = 0; ok && t < T; ++t) ok = !(dist2(pi, taken + (size_t)t * d, d) < ex2);
        alive[i] = ok ? 1 : 0;
        mx = fmax(mx, vals[i]);
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (lane == 0) wv[wave] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = wv[0];
        for (int w = 1; w < nw; ++w) m = fmax(m, wv[w]);
        *vmax = m;
    }
    int n = 0;
    for (int it = 0; it < q; ++it) {
        __syncthreads();  // alive[] updated, wv[] free
        double bv = -INFINITY;
        int bi = 0x7fffffff;
        for (int i = tid; i < N; i += blockDim.x)
            if (alive[i] && ranks_before(vals[i], i, bv, bi)) {
                bv = vals[i];
                bi = i;
            }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (ranks_before(ov, oi, bv, bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            wv[wave] = bv;
            wi[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double v = wv[0];
            int i = wi[0];
            for (int w = 1; w < nw; ++w)
                if (ranks_before(wv[w], wi[w], v, i)) {
                    v = wv[w];
                    i = wi[w];
                }
            pick = (i == 0x7fffffff) ? -1 : i;
            if (i != 0x7fffffff) idx[n] = i;
        }
        __syncthreads();
        const int pk = pick;
        if (pk < 0) break;
        ++n;
        const double *pp = pts + (size_t)pk * d;
        for (int i = tid; i < N; i += blockDim.x)
            if (alive[i] && (i == pk || dist2(pts + (size_t)i * d, pp, d) < ex2)) alive[i] = 0;
    }
    if (tid == 0) *count = n;
}

// dst rows r = src rows idx[r] (r < *count, at most rows), and the matching values if vdst.
__global__ __launch_bounds__(256) void k_take_rows(const double *__restrict__ src, const double *__restrict__ vsrc,
                                                   const int *__restrict__ idx, const int *__restrict__ count,
                                                   int rows, int d, double *__restrict__ dst, double *__restrict__ vdst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * d) return;
    const int r = t / d, k = t - r * d;
    if (r >= *count) return;
    dst[t] = src[(size_t)idx[r] * d + k];
    if (vdst && k == 0) vdst[r] = vsrc[idx[r]];
}

__global__ __launch_bounds__(256) void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = src[t];
}

hipError_t launch_pool_top(const double *pts, const double *vals, int rounds, int M, int d, int keep, double *pool_pts,
                           double *pool_vals, hipStream_t st) {
    if (M > kPoolMax || keep < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pool_top, dim3((unsigned)rounds), dim3(1024), 0, st, pts, vals, M, d, keep, pool_pts,
                       pool_vals);
    return hipGetLastError();
}

hipError_t launch_greedy(const double *pts, const double *vals, int N, int d, const double *taken, int T, int q,
                         double ex2, int *idx, int *count, double *vmax, hipStream_t st) {
    if (N > kGreedyMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(1024), 0, st, pts, vals, N, d, taken, T, q, ex2, idx, count, vmax);
    return hipGetLastError();
}

hipError_t launch_take_rows(const double *src, const double *vsrc, const int *idx, const int *count, int rows, int d,
                            double *dst, double *vdst, hipStream_t st) {
    const int n = rows * d;
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_take_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, vsrc, idx, count, rows,
                       d, dst, vdst);
    return hipGetLastError();
}

hipError_t launch_copy_f64(const double *src, double *dst, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_chaos_points(const double *z, const double *C, double r, int per, int nc, int d, double *U,
                               hipStream_t st) {
    const int count = per * nc * d;
    hipLaunchKernelGGL(k_chaos_points, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, z, C, r, per, d,
                       count, U);
    return hipGetLastError();
}

hipError_t launch_chaos_centres(const double *U, const double *e, int per, int nc, int d, double *C, double *Ce,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_chaos_centres, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, U, e, per, nc, d, C,
                       Ce);
    return hipGetLastError();
}

hipError_t launch_chaos_step(double *z, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_chaos_step, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, z, count);
    return hipGetLastError();
}

hipError_t launch_gp_ei(const GpEiArgs &a, hipStream_t st) {
    size_t blocks = ((size_t)a.M * a.npad + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_gp_kstar, dim3((unsigned)blocks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gp_zsq, dim3((unsigned)a.nti, (unsigned)((a.M + kGpT - 1) / kGpT)), dim3(256), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gp_ei, dim3((unsigned)((a.M + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace boac
