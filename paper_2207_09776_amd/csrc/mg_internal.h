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
// q <= qmax are concatenated per row: NB = sum_{q <= qmax} (2R[q]+1) doubles,
// padded to NBP (a row holds no V2 band where Dt^2 does not occur).
//
// Coefficients that depend on x add terms W_{l,t} (x) diag(a_t) (t < ND, the
// x vectors a_t shared by all l); their bands (radius RW) follow the three V
// bands in each row, so NB = sum_{q <= qmax} (2R[q]+1) + ND (2RW+1).  ND is 0, 3 (for
// one to three factors) or MG_MAX_XDIAG (unused factors are zero).
// ---------------------------------------------------------------------------
constexpr int MG_NBASIS = 6;
constexpr int MG_HDR = 8;          // table header entries (doubles)
constexpr int MG_MAX_XDIAG = 4;    // most x-dependent factors the kernels take
constexpr int MG_XDIAG_RADIUS = 2; // band radius of their v factors (and of the x-term factors)
constexpr int MG_MAX_XTERM = 32;   // x-terms C (x) diag(x_0) D^x ... diag(x_d) (d <= 2)
constexpr int MG_MAX_XVEC = 16;    // distinct x vectors of the x-terms

struct mg_ops {
    mg_grid grid;
    int order;
    int R[3];                      // band radius of the V tables per x-power q
    int qmax;                      // highest x-power the kernels apply (1 or 2)
    int NB, NBP;                   // coefficients per row, padded row stride
    int nactive;                   // basis matrices used by `order` (2, 4 or 6)
    int nv_pad;                    // table rows: nv rounded up to the kernel's rows (zeros)
    int ND = 0, RW = 0;            // x-dependent factors and their band radius
    int NC = 0, NCB = 0;           // x-terms C (x) X with X = diag(x_0) D^x diag(x_1)
                                   // ... D^x diag(x_d), d <= 2, that the diagonal
                                   // x-factors cannot hold, and their coefficients
                                   // per row (NC bands of radius MG_XDIAG_RADIUS)
    int NXV = 0;                   // distinct x vectors of the x-terms
    bool xt_in_ba = false;         // B or A holds x-terms (the Euler kernels read them)
    // basis tables, host copy and device copy: [MG_NBASIS][nv_pad][NBP], then
    // the x-term section [MG_NBASIS][nv_pad][NCB]
    std::vector<double> basis_host;
    double* basis_dev = nullptr;
    // x vectors a_t [ND][nx] and per factor {sum, midpoint, half-width, 0};
    // x-term vectors [NXV][nx] (vector 0 is the unit vector) and per x-term
    // {||X||_1, tr X, 0, 0} with D^x taken without its 1/(2 dx);
    // x-term descriptors [NC][4] = {d + 4 L_1 + 8 L_2, slot of x_0, slot of x_1,
    // slot of x_d} (letters L: 0 Dt, 1 Dxx)
    std::vector<double> xdiag_host, xstat_host, xchain_host, cstat_host;
    std::vector<int32_t> xdesc_host;
    double* xdiag_dev = nullptr;   // xdiag, xstat, xchain, cstat, xdesc in one allocation
    size_t xdesc_off = 0;          // offset of xdesc in it (doubles, even)
    int device = 0;
    // register-resident kernel shape (PX, RJ, NW) recorded by the autotuner
    // per precision (FP64, FP32C); zeros: the default shape
    int tuned[2][3] = {{0, 0, 0}, {0, 0, 0}};
    // cooperative-kernel shape variant per precision (0: the default)
    int tuned_coop[2] = {0, 0};
};

// Per-(path, step) table of the scaled Magnus logarithm (written by the
// assemble kernel, read by the Taylor kernels).  Layout per (p,k):
//   64-byte header: [int32 s, pad] [int32 m, pad] [f64 exp(mu/s)] [f64 mu]
//                   [f64 ||Y - mu I||_1] [int32 flag, pad] [2 x f64 reserved]
//   then nv_pad rows of NBP coefficients of (Y - mu I)/s, FP64 (MG_FP64) or
//   FP32 rounded from FP64 with each band's rounding residual in its centre
//   entry (MG_FP32C), then nv_pad rows of the NCB x-term coefficients (FP64
//   only); records are 64-byte aligned.
inline size_t mg_table_bytes(const mg_ops* ops, int precision) {
    const size_t elem = precision == MG_FP32C ? 4 : 8;
    size_t b = 64 + (size_t)ops->nv_pad * (ops->NBP + ops->NCB) * elem;
    return (b + 63) & ~(size_t)63;
}

// device copies of the per-factor statistics and of the x-term vectors,
// statistics and descriptors, which follow the x vectors in the xdiag_dev
// allocation
inline const double* mg_xstat_dev(const mg_ops* ops) {
    return ops->xdiag_dev + ops->xdiag_host.size();
}
inline const double* mg_xchain_dev(const mg_ops* ops) {
    return ops->xdiag_dev + ops->xdiag_host.size() + ops->xstat_host.size();
}
inline const double* mg_cstat_dev(const mg_ops* ops) {
    return mg_xchain_dev(ops) + ops->xchain_host.size();
}
inline const int4* mg_xdesc_dev(const mg_ops* ops) {
    return reinterpret_cast<const int4*>(ops->xdiag_dev + ops->xdesc_off);
}

// error state (thread local, defined in api.hip)
mg_status mg_fail(mg_status code, const std::string& msg);

// kernel launchers (defined next to the kernels)
hipError_t launch_iterated_integrals(const double* dW, int64_t P, int64_t Nf, double T, int K,
                                     int order, double* coef, double* pathstat, hipStream_t s);
hipError_t launch_iterated_integrals_steps(const double* dW, int64_t P, int64_t Nf, double T,
                                           const int32_t* Kp, int Kmax, int order, double* coef,
                                           double* pathstat, hipStream_t s);
hipError_t launch_euler_increments(const double* dW, int64_t P, int64_t Nf, int NE, double* dWE,
                                   hipStream_t s);
hipError_t launch_assemble(const mg_ops* ops, const double* coef, int64_t P, int K, double tol,
                           int precision, char* tables, hipStream_t s);
// Taylor chain over all K steps for paths whose state fits on one workgroup.
// Returns hipErrorInvalidValue (without launching) if no kernel shape fits.
// `shape` (PX, RJ, NW) overrides the shape (autotuner candidates), else the
// default or the autotuner's record in ops.
hipError_t launch_expmv_resident(const mg_ops* ops, const char* tables, size_t tbytes, int64_t P,
                                 int K, const double* u0, int u0_broadcast, double* uT, double tol,
                                 int precision, int32_t* stats, int32_t* flags, hipStream_t s,
                                 bool dry_run, const int* shape = nullptr);
hipError_t launch_euler_resident(const mg_ops* ops, double* u, int64_t P, const double* dWE,
                                 int NE, double dt, int32_t* flags, hipStream_t s, bool dry_run);
hipError_t launch_error_vs_exact(const mg_grid* grid, const mg_exact* ex, const double* pathstat,
                                 const double* u, const double* uref, int64_t P, int kappa,
                                 double* err, hipStream_t s);

// rows covered by the resident kernel shape for this grid (0: no shape)
int resident_rows(int nx, int nv);
// resident kernel shapes the autotuner may time for this grid (the default
// first); returns their number (<= max)
int resident_candidates(int nx, int nv, int (*shapes)[3], int max);
// the most rows per workgroup any cooperative kernel shape for this nx uses
// (operator tables are padded to a multiple of it; 0: no shape)
int coop_rows_max(int nx);
// table rows the cooperative kernels for this grid need: nv rounded up to
// the rows of a workgroup (0: no kernel)
int coop_table_rows(int nx, int nv);
// cooperative kernels: the Taylor chain and Euler-Maruyama (FP64)
enum class CoopKind { Expmv, Euler };
// a cooperative kernel of this kind exists for this operator and precision
bool coop_supported(const mg_ops* ops, int precision, CoopKind kind = CoopKind::Expmv);

// Cooperative launch plan: G workgroups per path, ngroups resident groups and
// the exchange area they need (placed after the tables in the workspace).
struct CoopPlan {
    int G = 0, ngroups = 0, xcd_map = 0, threads = 0, per_cu = -1, cus = -1;
    int stage = 0;   // how far planning got (diagnostics)
    size_t lds = 0, xh_bytes = 0, xn_bytes = 0, fl_bytes = 0, bytes = 0;
};
// variant: the kernel variant (coop_variant_valid), -1 the one the operator
// records
hipError_t coop_plan(const mg_ops* ops, int precision, int64_t P, CoopPlan* plan,
                     CoopKind kind = CoopKind::Expmv, int variant = -1);
// Variants of the cooperative Taylor kernel for an operator and precision;
// all apply the same arithmetic per point in the same order with the same
// rows per workgroup.  Bit 0 selects the alternative workgroup shape, bit 1
// the exchange overlapped with the term's rows; variant 0 is the default.
constexpr int MG_COOP_VARIANTS = 4;
bool coop_variant_valid(const mg_ops* ops, int precision, int variant);
// private (spill) bytes per lane of a variant's kernel (-1: no such kernel)
int coop_variant_scratch(const mg_ops* ops, int precision, int variant);
// waves and rows per workgroup of a variant (false: none)
bool coop_variant_shape(const mg_ops* ops, int precision, int variant, int* nw, int* rows);
hipError_t launch_expmv_coop(const mg_ops* ops, const char* tables, size_t tbytes, int64_t P,
                             int K, const double* u0, int u0_broadcast, double* uT, double tol,
                             int precision, int32_t* stats, int32_t* flags, char* xarea,
                             const CoopPlan& plan, hipStream_t s);
// Euler-Maruyama for grids beyond the register-resident kernel (plan of kind Euler)
hipError_t launch_euler_coop(const mg_ops* ops, double* u, int64_t P, const double* dWE, int NE,
                             double dt, int32_t* flags, char* xarea, const CoopPlan& plan,
                             hipStream_t s);

// host operator build (ops_build.cpp)
mg_status mg_build_host(const mg_grid* grid, const mg_coeffs* coeffs, int order, mg_ops* ops);
