// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "magnus.h"

// ---------------------------------------------------------------------------
// Factored operator form.
//
// Every matrix of the Magnus basis M_l (B, A, A^2, [B,A], [[B,A],A], [[B,A],B])
// is stored as  M_l = sum_{q=0..2} V_{l,q} (x) Dt^q  where Dt = tridiag(-1,0,1)
// is the raw x difference (D^x = Dt / (2 dx)); the factor (1/(2dx))^q is folded
// into V_{l,q}.  V_{l,q} is an nv x nv band matrix with radius R[q]; row j is
// stored as 2R[q]+1 entries for columns j-R[q] .. j+R[q].  The bands of the
// three q are concatenated per row: NB = sum_q (2R[q]+1) doubles, padded to NBP.
// ---------------------------------------------------------------------------
constexpr int MG_NBASIS = 6;
constexpr int MG_HDR = 8;          // table header entries (doubles)

struct mg_ops {
    mg_grid grid;
    int order;
    int R[3];                      // band radius of the V tables per x-power q
    int qmax;                      // highest x-power the kernels apply (1 or 2)
    int NB, NBP;                   // coefficients per row, padded row stride
    int nactive;                   // basis matrices used by `order` (2, 4 or 6)
    int nv_pad;                    // table rows: nv rounded up to the kernel's rows (zeros)
    // basis tables, host copy and device copy: [MG_NBASIS][nv_pad][NBP]
    std::vector<double> basis_host;
    double* basis_dev = nullptr;
    int device = 0;
};

// Per-(path, step) table of the scaled Magnus logarithm (written by the
// assemble kernel, read by the Taylor kernels).  Layout per (p,k), FP64:
//   [0] s (int32)  [1] m (int32)  [2] exp(mu/s)  [3] mu  [4] ||Y - mu I||_1
//   [5] flag (int32)  then nv rows of NBP coefficients of (Y - mu I)/s.
inline size_t mg_table_stride(const mg_ops* ops) {
    size_t s = (size_t)MG_HDR + (size_t)ops->nv_pad * ops->NBP;
    return (s + 7) & ~(size_t)7;   // 64-byte aligned records
}

// error state (thread local, defined in api.hip)
mg_status mg_fail(mg_status code, const std::string& msg);

// kernel launchers (defined next to the kernels)
hipError_t launch_iterated_integrals(const double* dW, int64_t P, int64_t Nf, double T, int K,
                                     int order, double* coef, double* pathstat, hipStream_t s);
hipError_t launch_euler_increments(const double* dW, int64_t P, int64_t Nf, int NE, double* dWE,
                                   hipStream_t s);
hipError_t launch_assemble(const mg_ops* ops, const double* coef, int64_t P, int K, double tol,
                           int precision, double* tables, hipStream_t s);
// Taylor chain over all K steps for paths whose state fits on one workgroup.
// Returns hipErrorInvalidValue (without launching) if no kernel shape fits.
hipError_t launch_expmv_resident(const mg_ops* ops, const double* tables, int64_t P, int K,
                                 const double* u0, int u0_broadcast, double* uT, double tol,
                                 int32_t* stats, int32_t* flags, hipStream_t s, bool dry_run);
hipError_t launch_euler_resident(const mg_ops* ops, double* u, int64_t P, const double* dWE,
                                 int NE, double dt, int32_t* flags, hipStream_t s, bool dry_run);
hipError_t launch_error_vs_exact(const mg_grid* grid, const mg_exact* ex, const double* pathstat,
                                 const double* u, const double* uref, int64_t P, int kappa,
                                 double* err, hipStream_t s);

// rows covered by the resident kernel shape for this grid (0: no shape)
int resident_rows(int nx, int nv);

// host operator build (ops_build.cpp)
mg_status mg_build_host(const mg_grid* grid, const mg_coeffs* coeffs, int order, mg_ops* ops);
