// Relative Frobenius error on the central kappa window, eq. (meanErr), against
// a reference array or the closed-form constant-coefficient Langevin solution.
//
// Closed form (Section 3.1, fundamental solution Gamma integrated against the
// Gaussian initial density N(0, s0sq I)): with c = a - sigma^2,
//   y = (x + sigma * int_0^T W, v + sigma * W_T),
//   S = s0sq [[1+T^2, T], [T, 1]] + c [[T^3/3, T^2/2], [T^2/2, T]],
//   u(x, v) = exp(-y^T S^{-1} y / 2) / (2 pi sqrt(det S)).
// One workgroup per path; FP64 sums reduced within the workgroup.

#include <cmath>

#include "mg_internal.h"

namespace {

constexpr int kThreads = 256;

struct ErrArgs {
    const double* pathstat;
    const double* u;
    const double* uref;
    double* err;
    int nx, nv;
    int wx0, wv0, wx, wv;     // window origin and width per axis
    double ax, dx, av, dv;
    double sigma, S00, S01, S11, det;
};

__global__ __launch_bounds__(kThreads) void error_kernel(ErrArgs a) {
    __shared__ double red[2][kThreads / 64];
    const int64_t p = blockIdx.x;
    const size_t N = (size_t)a.nx * a.nv;
    const double* up = a.u + p * N;
    double WT = 0.0, IT = 0.0;
    if (!a.uref) {
        WT = a.pathstat[2 * p];
        IT = a.pathstat[2 * p + 1];
    }
    const double norm = 1.0 / (2.0 * M_PI * sqrt(a.det));
    double num = 0.0, den = 0.0;
    const int cnt = a.wx * a.wv;
    for (int idx = threadIdx.x; idx < cnt; idx += kThreads) {
        const int jj = a.wv0 + idx / a.wx, ii = a.wx0 + idx % a.wx;
        const size_t off = (size_t)jj * a.nx + ii;
        double ref;
        if (a.uref) {
            ref = a.uref[p * N + off];
        } else {
            const double x = a.ax + (ii + 1) * a.dx, v = a.av + (jj + 1) * a.dv;
            const double y1 = x + a.sigma * IT, y2 = v + a.sigma * WT;
            const double q = (a.S11 * y1 * y1 - 2.0 * a.S01 * y1 * y2 + a.S00 * y2 * y2) / a.det;
            ref = norm * exp(-0.5 * q);
        }
        const double diff = up[off] - ref;
        num += diff * diff;
        den += ref * ref;
    }
    for (int o = 32; o > 0; o >>= 1) {
        num += __shfl_xor(num, o, 64);
        den += __shfl_xor(den, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = num;
        red[1][w] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double n = 0.0, d = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) {
            n += red[0][i];
            d += red[1][i];
        }
        a.err[p] = sqrt(n) / sqrt(d);
    }
}

void window(int n, int kappa, int& i0, int& w) {
    w = n >> kappa;
    i0 = (int)std::floor(n / 2.0 - n / std::ldexp(1.0, kappa + 1));
}

}  // namespace

hipError_t launch_error_vs_exact(const mg_grid* g, const mg_exact* ex, const double* pathstat,
                                 const double* u, const double* uref, int64_t P, int kappa,
                                 double* err, hipStream_t s) {
    ErrArgs a{};
    a.pathstat = pathstat;
    a.u = u;
    a.uref = uref;
    a.err = err;
    a.nx = g->nx;
    a.nv = g->nv;
    window(g->nx, kappa, a.wx0, a.wx);
    window(g->nv, kappa, a.wv0, a.wv);
    a.ax = g->ax;
    a.av = g->av;
    a.dx = (g->bx - g->ax) / (g->nx + 1);
    a.dv = (g->bv - g->av) / (g->nv + 1);
    if (!uref) {
        const double T = ex->T, c = ex->a - ex->sigma * ex->sigma, s0 = ex->s0sq;
        a.sigma = ex->sigma;
        a.S00 = s0 * (1.0 + T * T) + c * T * T * T / 3.0;
        a.S01 = s0 * T + c * T * T / 2.0;
        a.S11 = s0 + c * T;
        a.det = a.S00 * a.S11 - a.S01 * a.S01;
    } else {
        a.det = 1.0;
    }
    hipLaunchKernelGGL(error_kernel, dim3((unsigned)P), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}
