// Per-(path, step) assembly of the Magnus logarithm, its 1-norm and the
// Taylor parameters (m, s).
//
// Y_{p,k} = sum_l coef[p][k][l] M_l (eq. (MagnusFormulas)) is formed row by
// row from the factored basis tables.  mu = tr(Y)/N is removed from the
// diagonal, ||Y - mu I||_1 (maximum absolute column sum) is computed exactly
// from the factored form, and (m, s) minimise m * s subject to
// ||Y - mu I||_1 / s <= theta_m (truncated-Taylor thresholds of Al-Mohy and
// Higham for the requested tolerance).  The table written for (p, k) holds the
// header (s, m, exp(mu/s), mu, norm, flag) and the rows of (Y - mu I)/s, in
// FP64, or rounded to FP32 for the compensated FP32 form (with the rounding
// residual of every band moved into its centre entry, see below).
//
// Column sums.  With M = sum_q V_q (x) Dt^q (Dt = tridiag(-1,0,1)), column
// (i', j') of Y - mu I has entries in rows (i, j), |j - j'| <= R, i - i' in
// {-2..2}:   i'-2: a2,  i'-1: a1,  i': a0 + a2 * diag(Dt^2)_{i'},  i'+1: -a1,
// i'+2: a2, with a_q = V_q[j][j' - j] (entries outside the grid are absent).
// Columns i' = 2 .. nx-3 share one pattern, so the classes
// i' in {0, 1, 2, nx-3, nx-2, nx-1} cover all columns.  Terms W_t (x) diag(a_t)
// (x-dependent coefficients) add w_t a_t(i') to the entry in row i'; there the
// sum uses |c + sum_t w_t m_t| + sum_t |w_t| h_t with m_t, h_t the midpoint and
// half-width of the values of a_t, an upper bound of the exact column sum, so
// (m, s) stay admissible (at worst s is larger than needed).  Chain terms
// C (x) diag(alpha) Dt diag(beta) add at most |C| max|alpha| max|beta| per x
// neighbour of the column.

#include <cmath>

#include "mg_internal.h"
#include "theta_table.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxS = 1 << 14;   // beyond this the path is flagged (MG_FLAG_NORM)

struct AsmArgs {
    const double* basis;       // [6][nv][NBP]
    const double* coef;        // [P][K][6]
    char* tables;              // [P][K] records of tbytes
    size_t tbytes;
    int f32;                   // rows in FP32 (compensated form) instead of FP64
    int nx, nv, nv_pad, K, NBP, nact;
    int R0, R1, R2;
    int qmax;                  // V2 (Dt^2) entries are in the row only for qmax >= 2
    int ND, RW;                // x-dependent factors (0: none) and their band radius
    const double* xstat;       // per factor {sum, midpoint, half-width, 0}
    int use24;                 // theta table for 2^-24 instead of 2^-53
    int NC, NCB;               // x-terms and their coefficients per row (FP64 only)
    const double* basis_c;     // x-term section of the basis [6][nv_pad][NCB]
    const double* cstat;       // per x-term X {||X||_1, tr X, 0, 0} (raw differences)
};

__device__ inline double coeff(const AsmArgs& a, const double* c, int j, int idx) {
    double v = 0.0;
    for (int l = 0; l < a.nact; ++l) v += c[l] * a.basis[((size_t)l * a.nv_pad + j) * a.NBP + idx];
    return v;
}
__device__ inline double coeff_c(const AsmArgs& a, const double* c, int j, int idx) {
    double v = 0.0;
    for (int l = 0; l < a.nact; ++l) v += c[l] * a.basis_c[((size_t)l * a.nv_pad + j) * a.NCB + idx];
    return v;
}

__device__ inline double block_reduce(double v, double* red, bool is_max) {
    for (int o = 32; o > 0; o >>= 1) {
        double u = __shfl_xor(v, o, 64);
        v = is_max ? fmax(v, u) : v + u;
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < kThreads / 64; ++i) s = is_max ? fmax(s, red[i]) : s + red[i];
    return s;
}

// diagonal of Dt^2 at column/row i (Dt = tridiag(-1,0,1) with zero boundary)
__device__ inline double dt2_diag(int i, int nx) {
    int cnt = (i + 1 < nx ? 1 : 0) + (i > 0 ? 1 : 0);
    return -(double)cnt;
}

__global__ __launch_bounds__(kThreads) void assemble_kernel(AsmArgs a) {
    __shared__ double red[kThreads / 64];
    __shared__ double hdr[4];
    const int64_t pk = blockIdx.x;
    const double* c = a.coef + pk * 6;
    const int t = threadIdx.x;
    const bool v2 = a.qmax >= 2;
    const int o0 = 0, o1 = 2 * a.R0 + 1, o2 = o1 + 2 * a.R1 + 1, o3 = o2 + (v2 ? 2 * a.R2 + 1 : 0);
    const int wl = 2 * a.RW + 1;
    const int nx = a.nx, nv = a.nv;

    // trace: sum_j (nx * V0[j][0] + tr(Dt^2) * V2[j][0] + sum_t W_t[j][0] * sum_i a_t(i)
    //              + sum_k C_k[j][0] * tr X_k)
    const double trDt2 = nx >= 2 ? -(2.0 * nx - 2.0) : 0.0;
    double tr = 0.0;
    for (int j = t; j < nv; j += kThreads) {
        tr += nx * coeff(a, c, j, o0 + a.R0) + (v2 ? trDt2 * coeff(a, c, j, o2 + a.R2) : 0.0);
        for (int f = 0; f < a.ND; ++f) tr += coeff(a, c, j, o3 + f * wl + a.RW) * a.xstat[4 * f];
        for (int f = 0; f < a.NC; ++f) tr += coeff_c(a, c, j, f * wl + a.RW) * a.cstat[4 * f + 1];
    }
    tr = block_reduce(tr, red, false);
    const double mu = tr / ((double)nx * nv);

    // column sums of |Y - mu I| over the x column classes
    int cls[6] = {0, 1, 2, nx - 3, nx - 2, nx - 1};
    double best = 0.0;
    for (int idx = t; idx < nv * 6; idx += kThreads) {
        const int jp = idx / 6;
        const int ip = cls[idx % 6];
        if (ip < 0 || ip >= nx) continue;
        double sum = 0.0;
        const int R = max(max(a.R0, a.R1), max(a.R2, a.ND > 0 ? a.RW : 0));
        for (int j = max(0, jp - R); j <= min(nv - 1, jp + R); ++j) {
            const int b = jp - j;
            const double a0 = (b >= -a.R0 && b <= a.R0) ? coeff(a, c, j, o0 + b + a.R0) : 0.0;
            const double a1 = (b >= -a.R1 && b <= a.R1) ? coeff(a, c, j, o1 + b + a.R1) : 0.0;
            const double a2 = (v2 && b >= -a.R2 && b <= a.R2) ? coeff(a, c, j, o2 + b + a.R2) : 0.0;
            double d0 = a0 - (b == 0 ? mu : 0.0), spread = 0.0;
            if (b >= -a.RW && b <= a.RW)
                for (int f = 0; f < a.ND; ++f) {
                    const double w = coeff(a, c, j, o3 + f * wl + b + a.RW);
                    d0 += w * a.xstat[4 * f + 1];
                    spread += fabs(w) * a.xstat[4 * f + 2];
                }
            if (ip - 2 >= 0) sum += fabs(a2);
            if (ip - 1 >= 0) sum += fabs(a1);
            sum += fabs(d0 + a2 * dt2_diag(ip, nx)) + spread;
            if (ip + 1 < nx) sum += fabs(a1);
            if (ip + 2 < nx) sum += fabs(a2);
            // x-terms C (x) X: a column of X sums to at most ||X||_1
            if (b >= -a.RW && b <= a.RW)
                for (int f = 0; f < a.NC; ++f)
                    sum += fabs(coeff_c(a, c, j, f * wl + b + a.RW)) * a.cstat[4 * f];
        }
        best = fmax(best, sum);
        if (sum != sum) best = sum;   // keep NaN visible
    }
    const double norm = block_reduce(best, red, true);

    if (t == 0) {
        int s = 1, m = 0, flag = 0;
        if (!isfinite(norm) || !isfinite(mu)) {
            flag = MG_FLAG_NONFINITE;
        } else if (norm > 0.0) {
            const double* th = a.use24 ? kTheta24 : kTheta53;
            long long bestc = -1;
            for (int mm = 1; mm <= MG_THETA_MMAX; ++mm) {
                double sd = ceil(norm / th[mm]);
                if (sd > (double)kMaxS) continue;
                long long ss = (long long)fmax(sd, 1.0);
                long long cost = (long long)mm * ss;
                if (bestc < 0 || cost < bestc) { bestc = cost; m = mm; s = (int)ss; }
            }
            if (bestc < 0) { flag = MG_FLAG_NORM; m = MG_THETA_MMAX; s = kMaxS; }
        }
        hdr[0] = s;
        hdr[1] = m;
        hdr[2] = flag;
        double* tab = reinterpret_cast<double*>(a.tables + pk * a.tbytes);
        int32_t* itab = reinterpret_cast<int32_t*>(tab);
        itab[0] = s;                   // [0] s      (int32 in the first word)
        itab[1] = 0;
        itab[2] = m;                   // [1] m
        itab[3] = 0;
        tab[2] = flag == MG_FLAG_NONFINITE ? NAN : exp(mu / s);
        tab[3] = mu;
        tab[4] = norm;
        itab[10] = flag;               // [5] flag
        itab[11] = 0;
        tab[6] = 0.0;
        tab[7] = 0.0;
    }
    __syncthreads();
    const double inv_s = 1.0 / hdr[0];
    char* rows = a.tables + pk * a.tbytes + 64;
    if (!a.f32) {
        for (int idx = t; idx < a.nv_pad * a.NBP; idx += kThreads) {
            const int j = idx / a.NBP, e = idx % a.NBP;
            double v = 0.0;
            if (j < nv) {
                v = coeff(a, c, j, e);
                if (e == o0 + a.R0) v -= mu;
            }
            reinterpret_cast<double*>(rows)[idx] = v * inv_s;
        }
        // x-term section (the trace shift is taken from the V0 centre only)
        double* crows = reinterpret_cast<double*>(rows) + (size_t)a.nv_pad * a.NBP;
        for (int idx = t; idx < a.nv_pad * a.NCB; idx += kThreads) {
            const int j = idx / a.NCB, e = idx % a.NCB;
            crows[idx] = j < nv ? coeff_c(a, c, j, e) * inv_s : 0.0;
        }
        return;
    }
    // FP32 rows.  Rounding every entry on its own would change the sum of each
    // band by up to 2^-24 times the sum of its magnitudes; on smooth data the
    // operator acts through these sums (the large entries of a second
    // difference cancel), so that change becomes a spurious growth rate of
    // the order of 2^-24 ||Y||, the same in every sub-step of a Magnus step.
    // Each band's centre entry therefore takes up the rounding residual of
    // the others: the FP32 band sums equal the FP64 ones to one rounding of
    // the (small, trace-shifted) centre.
    for (int j = t; j < a.nv_pad; j += kThreads) {
        float* row = reinterpret_cast<float*>(rows) + (size_t)j * a.NBP;
        if (j >= nv) {
            for (int e = 0; e < a.NBP; ++e) row[e] = 0.0f;
            continue;
        }
        auto band = [&](int off, int rad, double shift) {
            double resid = 0.0;
            for (int b = -rad; b <= rad; ++b) {
                if (b == 0) continue;
                const double v = coeff(a, c, j, off + b + rad) * inv_s;
                const float f = (float)v;
                row[off + b + rad] = f;
                resid += v - (double)f;
            }
            row[off + rad] = (float)((coeff(a, c, j, off + rad) - shift) * inv_s + resid);
        };
        band(o0, a.R0, mu);
        band(o1, a.R1, 0.0);
        if (v2) band(o2, a.R2, 0.0);
        for (int f = 0; f < a.ND; ++f) band(o3 + f * wl, a.RW, 0.0);
        for (int e = o3 + a.ND * wl; e < a.NBP; ++e) row[e] = 0.0f;
    }
}

}  // namespace

hipError_t launch_assemble(const mg_ops* ops, const double* coef, int64_t P, int K, double tol,
                           int precision, char* tables, hipStream_t s) {
    AsmArgs a;
    a.basis = ops->basis_dev;
    a.coef = coef;
    a.tables = tables;
    a.tbytes = mg_table_bytes(ops, precision);
    a.f32 = precision == MG_FP32C ? 1 : 0;
    a.nx = ops->grid.nx;
    a.nv = ops->grid.nv;
    a.nv_pad = ops->nv_pad;
    a.K = K;
    a.NBP = ops->NBP;
    a.nact = ops->nactive;
    a.R0 = ops->R[0];
    a.R1 = ops->R[1];
    a.R2 = ops->R[2];
    a.qmax = ops->qmax;
    a.ND = ops->ND;
    a.RW = ops->RW;
    a.xstat = ops->ND > 0 ? ops->xdiag_dev + (size_t)ops->ND * ops->grid.nx : nullptr;
    a.use24 = tol >= 0x1p-24 ? 1 : 0;
    a.NC = ops->NC;
    a.NCB = ops->NCB;
    a.basis_c = ops->basis_dev + (size_t)MG_NBASIS * ops->nv_pad * ops->NBP;
    a.cstat = ops->NC > 0 ? mg_cstat_dev(ops) : nullptr;
    const int64_t blocks = P * K;
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}
