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
            ei = sd * fma(g, cdf, pdf);
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
