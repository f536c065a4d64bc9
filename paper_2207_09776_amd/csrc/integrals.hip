// Lebesgue integrals of the fine Brownian path per Magnus step and the
// weights of eq. (MagnusFormulas).
//
// One workgroup per path walks its K sub-intervals in order (K the same for
// every path, or one count per path with the rows beyond it zero).  On sub-interval
// k the path restarts (W~_0 = 0) and the integrals int W~, int W~^2,
// int r W~ dr are taken exactly for the piecewise-linear path through the fine
// nodes r_i = i delta:
//   int W~      = sum delta (W_i + W_{i+1}) / 2
//   int W~^2    = sum delta (W_i^2 + W_i W_{i+1} + W_{i+1}^2) / 3
//   int r W~ dr = sum delta (r_i (2 W_i + W_{i+1}) + r_{i+1} (W_i + 2 W_{i+1})) / 6
// Each thread owns a contiguous chunk of the n = Nf/K increments; an exclusive
// scan of the chunk sums gives every thread its starting value W~.  All
// arithmetic is FP64.

#include "mg_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ inline double block_sum(double v, double* red) {
    // wave reduction then one LDS pass
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
    return s;
}

// Kp (nullable): steps of each path; path p then fills rows 0 .. Kp[p]-1 of
// its Kstride rows and zeros the rest (a zero step is the identity), or fills
// every row with NaN when Kp[p] is not a divisor of Nf in 1 .. Kstride.
__global__ __launch_bounds__(kThreads) void iterated_integrals_kernel(
    const double* __restrict__ dW, int64_t Nf, double T, int Kuni, const int32_t* __restrict__ Kp,
    int Kstride, int order, double* __restrict__ coef, double* __restrict__ pathstat) {
    __shared__ double scan[kThreads];
    __shared__ double red[kThreads / 64];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const int K = Kp ? Kp[p] : Kuni;
    if (K < 1 || K > Kstride || Nf % K != 0) {
        for (int64_t i = t; i < (int64_t)Kstride * 6; i += kThreads)
            coef[p * Kstride * 6 + i] = NAN;
        if (t == 0 && pathstat) pathstat[2 * p] = pathstat[2 * p + 1] = NAN;
        return;
    }
    for (int64_t i = (int64_t)K * 6 + t; i < (int64_t)Kstride * 6; i += kThreads)
        coef[p * Kstride * 6 + i] = 0.0;
    const int64_t n = Nf / K;
    const double h = T / K;
    const double delta = T / (double)Nf;
    const double* path = dW + p * Nf;
    // chunk of this thread within a sub-interval
    const int64_t per = (n + kThreads - 1) / kThreads;
    const int64_t i0 = min<int64_t>((int64_t)t * per, n), i1 = min<int64_t>(i0 + per, n);

    double Wstart = 0.0;     // W at the left end of the sub-interval (global path)
    double IT = 0.0;         // int_0^{t_k} W
    for (int k = 0; k < K; ++k) {
        const double* seg = path + (int64_t)k * n;
        double csum = 0.0;
        for (int64_t i = i0; i < i1; ++i) csum += seg[i];
        // exclusive scan of the chunk sums
        __syncthreads();
        scan[t] = csum;
        __syncthreads();
        for (int o = 1; o < kThreads; o <<= 1) {
            double add = (t >= o) ? scan[t - o] : 0.0;
            __syncthreads();
            scan[t] += add;
            __syncthreads();
        }
        const double total = scan[kThreads - 1];
        double Wl = scan[t] - csum;              // W~ at node i0
        double s1 = 0.0, s2 = 0.0, sj = 0.0;
        for (int64_t i = i0; i < i1; ++i) {
            const double Wr = Wl + seg[i];
            const double rl = (double)i * delta, rr = (double)(i + 1) * delta;
            s1 += Wl + Wr;
            s2 += Wl * Wl + Wl * Wr + Wr * Wr;
            sj += rl * (2.0 * Wl + Wr) + rr * (Wl + 2.0 * Wr);
            Wl = Wr;
        }
        const double I1 = block_sum(s1, red) * (delta / 2.0);
        const double I2 = block_sum(s2, red) * (delta / 3.0);
        const double J = block_sum(sj, red) * (delta / 6.0);
        const double DW = total;
        if (t == 0) {
            double* c = coef + ((int64_t)p * Kstride + k) * 6;
            c[0] = h;
            c[1] = DW;
            c[2] = order >= 2 ? -0.5 * h : 0.0;
            c[3] = order >= 2 ? I1 - 0.5 * h * DW : 0.0;
            c[4] = order >= 3 ? 0.5 * I2 - 0.5 * DW * I1 + h * DW * DW / 12.0 : 0.0;
            c[5] = order >= 3 ? J - 0.5 * h * I1 - h * h * DW / 12.0 : 0.0;
        }
        IT += Wstart * h + I1;
        Wstart += DW;
    }
    if (t == 0 && pathstat) {
        pathstat[2 * p] = Wstart;
        pathstat[2 * p + 1] = IT;
    }
}

// Euler increments: one thread per (p, n) sums its Nf/NE fine increments in
// order.
__global__ __launch_bounds__(256) void euler_increments_kernel(const double* __restrict__ dW,
                                                                int64_t P, int64_t Nf, int NE,
                                                                double* __restrict__ dWE) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= P * NE) return;
    const int64_t p = idx / NE, n = idx % NE, len = Nf / NE;
    const double* src = dW + p * Nf + n * len;
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += src[i];
    dWE[idx] = s;
}

}  // namespace

hipError_t launch_euler_increments(const double* dW, int64_t P, int64_t Nf, int NE, double* dWE,
                                   hipStream_t s) {
    const int64_t n = P * NE;
    hipLaunchKernelGGL(euler_increments_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       dW, P, Nf, NE, dWE);
    return hipGetLastError();
}

hipError_t launch_iterated_integrals(const double* dW, int64_t P, int64_t Nf, double T, int K,
                                     int order, double* coef, double* pathstat, hipStream_t s) {
    hipLaunchKernelGGL(iterated_integrals_kernel, dim3((unsigned)P), dim3(kThreads), 0, s, dW, Nf,
                       T, K, (const int32_t*)nullptr, K, order, coef, pathstat);
    return hipGetLastError();
}

hipError_t launch_iterated_integrals_steps(const double* dW, int64_t P, int64_t Nf, double T,
                                           const int32_t* Kp, int Kmax, int order, double* coef,
                                           double* pathstat, hipStream_t s) {
    hipLaunchKernelGGL(iterated_integrals_kernel, dim3((unsigned)P), dim3(kThreads), 0, s, dW, Nf,
                       T, Kmax, Kp, Kmax, order, coef, pathstat);
    return hipGetLastError();
}
