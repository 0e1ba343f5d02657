// Acquisition of the BOAC outer loop on the device, FP64: posterior mean, standard deviation and
// expected improvement (Eqs. 7-10, minimisation) of a fitted GP at M query points.
//
// With k*_m = k(q_m, u_.) (Eq. 8), the GP weights alpha = K^-1 z and X = L^-1 (K = L L^T):
//   mu_m = m0 + s k*_m . alpha,   var_m = s^2 (amp - |X k*_m|^2),
//   gamma = (J_best - mu - xi) / sigma,  EI = sigma (gamma Phi(gamma) + phi(gamma)).
// |X k*_m|^2 for all m is a triangular matrix product Z = X K*^T (n x M) reduced over its rows:
//   k_gp_kstar  K* [M][npad] (zero past n)
//   k_gp_zsq    per (64-row block of X, 64-query block): the Z block over j <= i, squared and summed
//               over its rows -> part [n/64][M] (fixed order, no atomics)
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

__global__ __launch_bounds__(256) void k_gp_zsq(GpEiArgs A) {
    __shared__ double Xs[kGpJ][kGpT + 1];  // X[i0 + r][j0 + c] at [c][r]
    __shared__ double Ks[kGpJ][kGpT + 1];  // K*[m0 + r][j0 + c] at [c][r]
    __shared__ double red[kGpT / 4][kGpT];
    const int i0 = blockIdx.x * kGpT, m0 = blockIdx.y * kGpT;
    const int tm = threadIdx.x & 15, ti = threadIdx.x >> 4;  // 4 queries x 4 rows per thread
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
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
        for (int c = 0; c < kGpJ; ++c) {
            double a[4], b[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[x] = Xs[c][ti * 4 + x];
                b[x] = Ks[c][tm * 4 + x];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        double s = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) s = fma(acc[x][y], acc[x][y], s);
        red[ti][tm * 4 + y] = s;
    }
    __syncthreads();
    if (threadIdx.x < kGpT) {
        double s = 0.0;
        for (int r = 0; r < kGpT / 4; ++r) s += red[r][threadIdx.x];
        const int m = m0 + threadIdx.x;
        if (m < A.M) A.part[(size_t)blockIdx.x * A.M + m] = s;
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
