// Register-resident Taylor chain of the iterated Magnus scheme (FP64 and the
// compensated FP32 form) and the Euler-Maruyama baseline, for grids whose
// per-path state fits on one workgroup (nx <= 128, nv <= 128).
//
// Work decomposition (one workgroup = one path, all K Magnus steps):
//   lane l of every wave owns the PX consecutive x points l*PX .. l*PX+PX-1;
//   wave w owns the RJ consecutive v rows w*RJ .. w*RJ+RJ-1.
// The Taylor term and the partial sum (which is also the state u between
// sub-steps) stay in VGPRs for the whole launch; HBM is touched only to read
// u0 and the per-step coefficient tables and to write uT.
//
// Applying Y = sum_q V_q (x) Dt^q (Dt = tridiag(-1,0,1) along x) to d:
//   y_q(j) = sum_b V_q[j][b] d(j + b)       (band along v: own registers,
//                                             plus RH halo rows per side that
//                                             neighbouring waves publish in LDS)
//   Y d    = y_0 + Dt (y_1 + Dt y_2)         (x differences: the neighbour
//                                             values come from adjacent lanes
//                                             through DPP wave shifts)
// The band coefficients of a row are the same for every lane of the wave: the
// FP64 kernel reads them with scalar loads, the FP32 kernel from a copy of
// the step's rows in LDS (scalar loads at one point per lane).  One barrier
// per Taylor term orders the halo
// exchange; the same barrier publishes the per-wave inf-norms used by the
// early-termination test of the Taylor sum.
//
// FP64 chain: with Y' = (Y - mu I)/s from the table, the chain is kept
// unscaled, d_j = Y'^j u, and F = sum_j d_j / j!; after each of the s sub-steps
// u <- exp(mu/s) F.
// FP32 compensated chain: c_j = Y' c_{j-1} / j in FP32 (FP32 tables), the sum
// F = hi + lo is accumulated with Kahan compensation in FP32; at the end of a
// sub-step u = exp(mu/s) (hi + lo) is formed in FP64 and split again, so the
// state between sub-steps and Magnus steps keeps ~48 significant bits.
// Both stop a sub-step after term j when
// ||c_{j-1}||_inf + ||c_j||_inf <= tol ||F||_inf.

#include <cmath>

#include "kernel_common.h"
#include "theta_table.h"   // MG_THETA_MMAX

namespace {

using namespace mgk;

// Early termination without a norm of F at every term.  The test after term j
// needs ||F_j||, but it can only pass if ||c_{j-1}|| <= tol ||F_j||, and
// ||F_j|| <= ||F_{j-1}|| + ||c_j|| with ||c_j|| <= tol ||F_j|| give
// ||F_j|| <= ||F_{j-1}|| / (1 - tol).  With fnest an upper bound of ||F_{j-1}||
// (the exact norm when it was formed, else the previous bound plus ||c_{j-1}||),
// ||F_j|| is therefore formed only when ||c_{j-1}|| <= tol fnest / (1 - tol)
// (times a margin for rounding).  Whenever the test could pass it is evaluated
// on the exact norms, so the term counts are those of the plain rule.
template <class T>
struct StopRule {
    T tol, kpred;
    T cprev, fnest;
    bool wantf;
    __device__ StopRule(T tol_, T margin) : tol(tol_), kpred(tol_ / (T(1) - tol_) * margin) {}
    __device__ void start(T unorm) {
        cprev = unorm;
        fnest = unorm;
        wantf = cprev <= kpred * fnest;
    }
    // norms of the latest term (c) and, when it was formed, of the partial sum
    // (fn); true when the series stops before the next term
    template <class ReadF>
    __device__ bool stop(T c, ReadF read_fn) {
        if (wantf) {
            const T fn = read_fn();
            if (cprev + c <= tol * fn) return true;
            fnest = fn;
        } else {
            fnest = fnest + c;
        }
        cprev = c;
        wantf = cprev <= kpred * fnest;
        return false;
    }
};

// Max over the NW per-wave partial maxima when lane l holds the entry of wave
// l mod NW (NW a power of two <= 16): row shifts reduce lanes 0..NW-1 and lane
// NW-1 holds the result.  With one LDS read per lane this keeps a single LDS
// round trip between the barrier and the next term.
template <class T, int NW>
__device__ inline T waves_max(T x) {
    static_assert(NW >= 1 && NW <= 16 && (NW & (NW - 1)) == 0, "NW must be a power of two");
    if (NW > 1) x = max_abs(x, dpp_pull<0x111, 0xf>(x));
    if (NW > 2) x = max_abs(x, dpp_pull<0x112, 0xf>(x));
    if (NW > 4) x = max_abs(x, dpp_pull<0x114, 0xf>(x));
    if (NW > 8) x = max_abs(x, dpp_pull<0x118, 0xf>(x));
    return lane_value<NW - 1>(x);
}

// 1/j! (FP64 chain) for j <= 63, formed by the same sequence of correctly
// rounded operations the chain would use at run time, and 1/j for the FP32
// chain as a float plus its residual: c_j = y (1/j) is formed as
// fma(y, inv_j, y * inv_j_lo), so the scaling carries no systematic bias (a
// single rounded 1/j would scale every term j of every sub-step by the same
// factor 1 + O(2^-24), which adds up over the sub-steps of a path).
struct FactorTables {
    double inv_fact[64];
    float inv_j[64];
    float inv_j_lo[64];
};
constexpr FactorTables make_factor_tables() {
    FactorTables t{};
    t.inv_fact[0] = 1.0;
    t.inv_j[0] = 1.0f;
    t.inv_j_lo[0] = 0.0f;
    for (int j = 1; j < 64; ++j) {
        t.inv_fact[j] = t.inv_fact[j - 1] / (double)j;
        t.inv_j[j] = (float)(1.0 / (double)j);
        t.inv_j_lo[j] = (float)(1.0 / (double)j - (double)t.inv_j[j]);
    }
    return t;
}
__constant__ FactorTables kFactors = make_factor_tables();
static_assert(MG_THETA_MMAX < 64, "factor tables too short");

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, int ND, int NC>
__global__ __launch_bounds__(64 * NW) void expmv_resident_kernel(
    const char* __restrict__ tables, size_t tbytes, int K, int nx, int nv,
    const double* __restrict__ u0, int u0_bcast, double* __restrict__ uT, double tol,
    int32_t* __restrict__ stats, int32_t* __restrict__ flags, const double* __restrict__ xdiag,
    const double* __restrict__ xvecs, const int4* __restrict__ xdesc, int nxt, int nxv) {
    using T = double;
    using BD = Bands<R0, R1, R2, QMAX>;
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, ND>();
    // x-term coefficients per row (NC > 0: the operator has x-terms)
    const int ncb = NC > 0 ? nxt * (2 * MG_XDIAG_RADIUS + 1) : 0;
    extern __shared__ double lds_d[];
    T* lds = reinterpret_cast<T*>(lds_d);
    Halo<PX, RJ, NW, RH, T> halo{lds};
    T* red = lds + halo_bytes<PX, NW, RH, T>() / sizeof(T);   // [2][NW][2] term norms
    T* red2 = red + 2 * NW * 2;                                 // [2][NW] state norms
    int* sflag = reinterpret_cast<int*>(red2 + 2 * NW);
    // x-term vectors [nxv][64*PX] after the flag word (16 bytes)
    T* cvl = red2 + 2 * NW + 2;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p = blockIdx.x;
    const int row0 = w * RJ;
    const int nrows = min(RJ, max(0, nv - row0));
    const size_t N = (size_t)nx * nv;
    if (threadIdx.x == 0) *sflag = 0;
    halo.zero_guards(threadIdx.x, 64 * NW);
    // x-dependent factors at this lane's points (zero beyond nx)
    constexpr int NDX = ND > 0 ? ND : 1;
    T xa[NDX][PX];
#pragma unroll
    for (int t = 0; t < NDX; ++t)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            xa[t][q] = (ND > 0 && i < nx) ? (T)xdiag[(size_t)t * nx + i] : T(0);
        }
    // x-term vectors at every lane's points into LDS (zero beyond nx; read
    // after the first barrier of the term loop)
    if constexpr (NC > 0) {
        for (int idx = threadIdx.x; idx < nxv * 64 * PX; idx += 64 * NW) {
            const int v = idx / (64 * PX), i = idx % (64 * PX);
            cvl[idx] = i < nx ? xvecs[(size_t)v * nx + i] : 0.0;
        }
    }
    const XTerms<PX, T> cvec{nxt, xdesc, cvl, lane};

    T F[RJ][PX];
    {
        const double* src = u0 + (u0_bcast ? 0 : (size_t)p * N);
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const int i = lane * PX + q;
                F[r][q] = (r < nrows && i < nx) ? src[(size_t)(row0 + r) * nx + i] : 0.0;
            }
    }
    // per-wave ||u||_inf into red2[par2]; read after the next barrier
    auto post_state_norm = [&](int par2) {
        T mx = 0;
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) mx = max_abs(mx, F[r][q]);
        mx = wave_max_dpp(mx);
        if (lane == 0) red2[par2 * NW + w] = mx;
    };

    int sub_par = 0;
    post_state_norm(sub_par);
    int tpar = 0;
    int pflag = 0;
    StopRule<T> rule(tol, 1.0 + 0x1p-30);

    for (int k = 0; k < K; ++k) {
        const TableView tv{tables + ((size_t)p * K + k) * tbytes};
        const int s = tv.s();
        const int m = tv.m();
        const double es = tv.es();
        pflag |= tv.flag();
        const T* rows = tv.rows<T>() + (size_t)row0 * NBP;
        // x-term section: after the NW*RJ main rows (the table's padded rows)
        const T* crows = tv.rows<T>() + (size_t)NW * RJ * NBP + (size_t)row0 * ncb;
        int terms = 0;
        for (int sub = 0; sub < s; ++sub) {
            // the Taylor terms alternate between A and B (no copies between terms)
            T A[RJ][PX], B[RJ][PX];
#pragma unroll
            for (int r = 0; r < RJ; ++r)
#pragma unroll
                for (int q = 0; q < PX; ++q) A[r][q] = F[r][q];
            // a sub-step without terms still orders the state-norm slots
            if (m == 0) __syncthreads();
            // term j from `in` into `out`; false when the series stopped before it
            auto step = [&](T (&in)[RJ][PX], T (&out)[RJ][PX], int j) -> bool {
                halo.publish(tpar, w, lane, in);
                __syncthreads();
                if (j == 1) {
                    rule.start(waves_max<T, NW>(red2[sub_par * NW + (lane & (NW - 1))]));
                } else {
                    // norms of the previous term (both read at once)
                    const T* rr = red + (size_t)(tpar ^ 1) * NW * 2 + 2 * (lane & (NW - 1));
                    const T cw = rr[0], fw = rr[1];
                    if (rule.stop(waves_max<T, NW>(cw), [&] { return waves_max<T, NW>(fw); }))
                        return false;
                }
                T top[RH][PX], bot[RH][PX];
                const int hp = tpar;
                auto fb = [&] { halo.fetch_bot(hp, w, lane, bot); };
                auto ft = [&] { halo.fetch_top(hp, w, lane, top); };
                auto coef = [&](int r, int e) -> T { return rows[r * NBP + e]; };
                const T fj = kFactors.inv_fact[j];   // 1/j!
                T mc = 0, mf = 0;
                auto emit = [&](int r, T (&y)[PX]) {
#pragma unroll
                    for (int q = 0; q < PX; ++q) {
                        F[r][q] = fma(y[q], fj, F[r][q]);
                        mc = max_abs(mc, y[q]);
                    }
                };
                if constexpr (NC > 0) {
                    auto ccoef = [crows, ncb](int r, int e) -> T { return crows[r * ncb + e]; };
                    apply_rows_any<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, T, NDX, decltype(coef),
                                   decltype(fb), decltype(ft), decltype(emit), NC,
                                   decltype(ccoef), decltype(cvec)>(
                        in, out, top, bot, fb, ft, coef, xa, lane, nx, emit, ccoef, cvec);
                } else {
                    apply_rows_any<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, T>(
                        in, out, top, bot, fb, ft, coef, xa, lane, nx, emit);
                }
                if (rule.wantf) {
#pragma unroll
                    for (int r = 0; r < RJ; ++r)
#pragma unroll
                        for (int q = 0; q < PX; ++q) mf = max_abs(mf, F[r][q]);
                    mf = wave_max_dpp(mf);
                }
                mc = wave_max_dpp(mc) * fj;
                if (lane == 0) {
                    red[(size_t)tpar * NW * 2 + 2 * w] = mc;
                    red[(size_t)tpar * NW * 2 + 2 * w + 1] = mf;
                }
                tpar ^= 1;
                ++terms;
                return true;
            };
            for (int j = 1; j <= m; j += 2) {
                if (!step(A, B, j)) break;
                if (j + 1 > m || !step(B, A, j + 1)) break;
            }
#pragma unroll
            for (int r = 0; r < RJ; ++r)
#pragma unroll
                for (int q = 0; q < PX; ++q) F[r][q] *= es;
            sub_par ^= 1;
            post_state_norm(sub_par);
        }
        if (stats && threadIdx.x == 0) {
            stats[((size_t)p * K + k) * 2] = terms;
            stats[((size_t)p * K + k) * 2 + 1] = s;
        }
    }

    bool bad = false;
    double* dst = uT + (size_t)p * N;
#pragma unroll
    for (int r = 0; r < RJ; ++r)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            if (r < nrows && i < nx) {
                dst[(size_t)(row0 + r) * nx + i] = F[r][q];
                bad |= !isfinite(F[r][q]);
            }
        }
    if (bad) atomicOr(sflag, MG_FLAG_NONFINITE);
    __syncthreads();
    if (flags && threadIdx.x == 0) flags[p] = *sflag | pflag;
}

// The FP32C kernel copies a step's coefficient rows into LDS when a lane
// holds two or more points per row.
template <int PX>
constexpr bool f32c_stages_rows() {
    return PX >= 2;
}

// Compensated FP32 form (see the file header).
template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, int ND>
__global__ __launch_bounds__(64 * NW) void expmv_resident_f32c_kernel(
    const char* __restrict__ tables, size_t tbytes, int K, int nx, int nv,
    const double* __restrict__ u0, int u0_bcast, double* __restrict__ uT, float tol,
    int32_t* __restrict__ stats, int32_t* __restrict__ flags, const double* __restrict__ xdiag) {
    using T = float;
    using BD = Bands<R0, R1, R2, QMAX>;
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, ND>();
    extern __shared__ double lds_d[];
    T* lds = reinterpret_cast<T*>(lds_d);
    Halo<PX, RJ, NW, RH, T> halo{lds};
    T* red = lds + halo_bytes<PX, NW, RH, T>() / sizeof(T);
    T* red2 = red + 2 * NW * 2;
    int* sflag = reinterpret_cast<int*>(red2 + 2 * NW);
    // coefficient rows staged in LDS from two points per lane on
    constexpr bool kStageRows = f32c_stages_rows<PX>();
    T* ctab = reinterpret_cast<T*>(reinterpret_cast<char*>(lds_d) +
                                   resident_ctab_offset<PX, NW, RH, T>());

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p = blockIdx.x;
    const int row0 = w * RJ;
    const int nrows = min(RJ, max(0, nv - row0));
    const size_t N = (size_t)nx * nv;
    if (threadIdx.x == 0) *sflag = 0;
    halo.zero_guards(threadIdx.x, 64 * NW);
    // x-dependent factors at this lane's points (zero beyond nx)
    constexpr int NDX = ND > 0 ? ND : 1;
    T xa[NDX][PX];
#pragma unroll
    for (int t = 0; t < NDX; ++t)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            xa[t][q] = (ND > 0 && i < nx) ? (T)xdiag[(size_t)t * nx + i] : T(0);
        }

    // F = hi + lo (hi carries the FP32 value, lo the compensation)
    T hi[RJ][PX], lo[RJ][PX];
    {
        const double* src = u0 + (u0_bcast ? 0 : (size_t)p * N);
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const int i = lane * PX + q;
                const double u = (r < nrows && i < nx) ? src[(size_t)(row0 + r) * nx + i] : 0.0;
                hi[r][q] = (float)u;
                lo[r][q] = (float)(u - (double)hi[r][q]);
            }
    }
    auto post_state_norm = [&](int par2) {
        T mx = 0;
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) mx = max_abs(mx, hi[r][q]);
        mx = wave_max_dpp(mx);
        if (lane == 0) red2[par2 * NW + w] = mx;
    };

    int sub_par = 0;
    post_state_norm(sub_par);
    int tpar = 0;
    int pflag = 0;
    StopRule<T> rule(tol, 1.0f + 0x1p-10f);

    for (int k = 0; k < K; ++k) {
        const TableView tv{tables + ((size_t)p * K + k) * tbytes};
        const int s = tv.s();
        const int m = tv.m();
        const double es = tv.es();
        pflag |= tv.flag();
        // this step's coefficient rows, staged in LDS and read from there by
        // every term, one row ahead (13 % faster than re-reading them through
        // the scalar cache at 128^2; at one point per lane the copy costs
        // more than it saves, and the FP64 kernel keeps the scalar reads,
        // since the rows in VGPRs make it spill)
        if constexpr (kStageRows) {
            constexpr int n16 = NW * RJ * NBP * (int)sizeof(T) / 16;
            static_assert(NW * RJ * NBP * sizeof(T) % 16 == 0, "row block not in 16-byte units");
            const uint4* src = reinterpret_cast<const uint4*>(tv.rows<T>());
            uint4* dst = reinterpret_cast<uint4*>(ctab);
            __syncthreads();   // the previous step's reads are done
            for (int i = threadIdx.x; i < n16; i += 64 * NW) dst[i] = src[i];
            __syncthreads();
        }
        const T* rows = (kStageRows ? ctab : tv.rows<T>()) + (size_t)row0 * NBP;
        int terms = 0;
        for (int sub = 0; sub < s; ++sub) {
            T A[RJ][PX], B[RJ][PX];
#pragma unroll
            for (int r = 0; r < RJ; ++r)
#pragma unroll
                for (int q = 0; q < PX; ++q) A[r][q] = hi[r][q];
            if (m == 0) __syncthreads();
            auto step = [&](T (&in)[RJ][PX], T (&out)[RJ][PX], int j) -> bool {
                halo.publish(tpar, w, lane, in);
                __syncthreads();
                if (j == 1) {
                    rule.start(waves_max<T, NW>(red2[sub_par * NW + (lane & (NW - 1))]));
                } else {
                    // norms of the previous term (both read at once)
                    const T* rr = red + (size_t)(tpar ^ 1) * NW * 2 + 2 * (lane & (NW - 1));
                    const T cw = rr[0], fw = rr[1];
                    if (rule.stop(waves_max<T, NW>(cw), [&] { return waves_max<T, NW>(fw); }))
                        return false;
                }
                T top[RH][PX], bot[RH][PX];
                const int hp = tpar;
                auto fb = [&] { halo.fetch_bot(hp, w, lane, bot); };
                auto ft = [&] { halo.fetch_top(hp, w, lane, top); };
                const auto coef = [&] {
                    if constexpr (kStageRows)
                        return LdsRows<T, NBP>{rows};
                    else
                        return [rows](int r, int e) -> T { return rows[r * NBP + e]; };
                }();
                const T invj = kFactors.inv_j[j], invj_lo = kFactors.inv_j_lo[j];
                T mc = 0, mf = 0;
                // c_j = Y' c_{j-1} / j goes to `out`; F = hi + lo gains c_j (Kahan)
                auto kahan = [&](int r, T (&y)[PX]) {
#pragma unroll
                    for (int q = 0; q < PX; ++q) {
                        const T x = fma(y[q], invj, y[q] * invj_lo);
                        y[q] = x;
                        const T a = x + lo[r][q];
                        const T t = hi[r][q] + a;
                        lo[r][q] = a - (t - hi[r][q]);
                        hi[r][q] = t;
                        mc = max_abs(mc, x);
                    }
                };
                apply_rows_any<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, T>(
                    in, out, top, bot, fb, ft, coef, xa, lane, nx, kahan);
                if (rule.wantf) {
#pragma unroll
                    for (int r = 0; r < RJ; ++r)
#pragma unroll
                        for (int q = 0; q < PX; ++q) mf = max_abs(mf, hi[r][q]);
                    mf = wave_max_dpp(mf);
                }
                mc = wave_max_dpp(mc);
                if (lane == 0) {
                    red[(size_t)tpar * NW * 2 + 2 * w] = mc;
                    red[(size_t)tpar * NW * 2 + 2 * w + 1] = mf;
                }
                tpar ^= 1;
                ++terms;
                return true;
            };
            for (int j = 1; j <= m; j += 2) {
                if (!step(A, B, j)) break;
                if (j + 1 > m || !step(B, A, j + 1)) break;
            }
            // u = exp(mu/s) (hi + lo) in FP64, split again
#pragma unroll
            for (int r = 0; r < RJ; ++r)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const double u = es * ((double)hi[r][q] + (double)lo[r][q]);
                    hi[r][q] = (float)u;
                    lo[r][q] = (float)(u - (double)hi[r][q]);
                }
            sub_par ^= 1;
            post_state_norm(sub_par);
        }
        if (stats && threadIdx.x == 0) {
            stats[((size_t)p * K + k) * 2] = terms;
            stats[((size_t)p * K + k) * 2 + 1] = s;
        }
    }

    bool bad = false;
    double* dst = uT + (size_t)p * N;
#pragma unroll
    for (int r = 0; r < RJ; ++r)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            if (r < nrows && i < nx) {
                const double u = (double)hi[r][q] + (double)lo[r][q];
                dst[(size_t)(row0 + r) * nx + i] = u;
                bad |= !isfinite(u);
            }
        }
    if (bad) atomicOr(sflag, MG_FLAG_NONFINITE);
    __syncthreads();
    if (flags && threadIdx.x == 0) flags[p] = *sflag | pflag;
}

// Euler-Maruyama: u <- u + (dt B + dW_n A) u for n = 0..NE-1 (FP64).
template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, int ND, int NC>
__global__ __launch_bounds__(64 * NW) void euler_resident_kernel(
    const double* __restrict__ basis, int nx, int nv, int nv_pad, double* __restrict__ u,
    const double* __restrict__ dWE, int NE, double dt, int32_t* __restrict__ flags,
    const double* __restrict__ xdiag, const double* __restrict__ xvecs,
    const int4* __restrict__ xdesc, int nxt, int nxv) {
    using T = double;
    using BD = Bands<R0, R1, R2, QMAX>;
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, ND>();
    extern __shared__ double lds[];
    Halo<PX, RJ, NW, RH, T> halo{lds};
    int* sflag = reinterpret_cast<int*>(lds + halo_bytes<PX, NW, RH, T>() / sizeof(T));
    // x-terms of B and A (NC > 0): vectors [nxv][64*PX] after the flag word,
    // coefficients in the x-term section of basis matrices 0 and 1
    T* cvl = lds + halo_bytes<PX, NW, RH, T>() / sizeof(T) + 2;
    const int ncb = NC > 0 ? nxt * (2 * MG_XDIAG_RADIUS + 1) : 0;
    if constexpr (NC > 0) {
        for (int idx = threadIdx.x; idx < nxv * 64 * PX; idx += 64 * NW) {
            const int v = idx / (64 * PX), i = idx % (64 * PX);
            cvl[idx] = i < nx ? xvecs[(size_t)v * nx + i] : 0.0;
        }
    }
    const XTerms<PX, T> xt{nxt, xdesc, cvl, (int)(threadIdx.x & 63)};

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p = blockIdx.x;
    const int row0 = w * RJ;
    const int nrows = min(RJ, max(0, nv - row0));
    const size_t N = (size_t)nx * nv;
    if (threadIdx.x == 0) *sflag = 0;
    halo.zero_guards(threadIdx.x, 64 * NW);
    // x-dependent factors at this lane's points (zero beyond nx)
    constexpr int NDX = ND > 0 ? ND : 1;
    T xa[NDX][PX];
#pragma unroll
    for (int t = 0; t < NDX; ++t)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            xa[t][q] = (ND > 0 && i < nx) ? (T)xdiag[(size_t)t * nx + i] : T(0);
        }

    T d[RJ][PX];
    double* src = u + (size_t)p * N;
#pragma unroll
    for (int r = 0; r < RJ; ++r)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            d[r][q] = (r < nrows && i < nx) ? src[(size_t)(row0 + r) * nx + i] : 0.0;
        }
    const double* Brows = basis + (size_t)row0 * NBP;             // basis matrix 0: B
    const double* Arows = basis + ((size_t)nv_pad + row0) * NBP;  // basis matrix 1: A
    const double* Bc = basis + (size_t)MG_NBASIS * nv_pad * NBP + (size_t)row0 * ncb;
    const double* Ac = Bc + (size_t)nv_pad * ncb;
    const double* dw = dWE + (size_t)p * NE;
    int tpar = 0;
    for (int n = 0; n < NE; ++n) {
        const double wn = dw[n];
        auto coef = [&](int r, int e) -> T {
            return fma(dt, Brows[r * NBP + e], wn * Arows[r * NBP + e]);
        };
        halo.publish(tpar, w, lane, d);
        __syncthreads();
        T top[RH][PX], bot[RH][PX];
        halo.fetch(tpar, w, lane, top, bot);
        auto din = [&](int rr, int q) -> T {
            if (rr < 0) return top[rr + RH][q];
            if (rr >= RJ) return bot[rr - RJ][q];
            return d[rr][q];
        };
        T dn[RJ][PX];
        apply_operator<PX, RJ, R0, R1, R2, QMAX, FULLX, T>(din, coef, lane, nx, dn);
        if constexpr (ND > 0) {
            // x-dependent factors: dn += a_t(x) * sum_b W_t[j][b] d(j+b)
            constexpr int WL = 2 * MG_XDIAG_RADIUS + 1;
            constexpr int NBM = BD::NB;
#pragma unroll
            for (int r = 0; r < RJ; ++r)
#pragma unroll
                for (int t = 0; t < ND; ++t) {
                    T z[PX];
#pragma unroll
                    for (int q = 0; q < PX; ++q) z[q] = T(0);
#pragma unroll
                    for (int b = 0; b < WL; ++b)
#pragma unroll
                        for (int q = 0; q < PX; ++q)
                            z[q] = fma(coef(r, NBM + t * WL + b), din(r - MG_XDIAG_RADIUS + b, q), z[q]);
#pragma unroll
                    for (int q = 0; q < PX; ++q) dn[r][q] = fma(xa[t][q], z[q], dn[r][q]);
                    // one row and factor at a time (the coefficient sums are VALU work)
                    __builtin_amdgcn_sched_barrier(0);
                }
        }
        if constexpr (NC > 0) {
            auto ccoef = [&](int r, int e) -> T {
                return fma(dt, Bc[r * ncb + e], wn * Ac[r * ncb + e]);
            };
#pragma unroll
            for (int r = 0; r < RJ; ++r) add_xterms<PX, MG_XDIAG_RADIUS, T>(r, dn[r], din, ccoef, xt);
        }
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) d[r][q] += dn[r][q];
        tpar ^= 1;
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < RJ; ++r)
#pragma unroll
        for (int q = 0; q < PX; ++q) {
            const int i = lane * PX + q;
            if (r < nrows && i < nx) {
                src[(size_t)(row0 + r) * nx + i] = d[r][q];
                bad |= !isfinite(d[r][q]);
            }
        }
    if (bad) atomicOr(sflag, MG_FLAG_NONFINITE);
    __syncthreads();
    if (flags && threadIdx.x == 0) flags[p] = *sflag;
}

// ---- dispatch ----------------------------------------------------------------
struct Shape {
    int PX, RJ, NW;
};

bool pick_shape(int nx, int nv, Shape& sh) {
    if (nx <= 64) {
        sh.PX = 1;
        if (nv <= 32) { sh.RJ = 16; sh.NW = 2; return true; }
        if (nv <= 64) { sh.RJ = 16; sh.NW = 4; return true; }
        if (nv <= 128) { sh.RJ = 16; sh.NW = 8; return true; }
        return false;
    }
    if (nx <= 128) {
        sh.PX = 2;
        if (nv <= 64) { sh.RJ = 16; sh.NW = 4; return true; }
        if (nv <= 128) { sh.RJ = 16; sh.NW = 8; return true; }
        return false;
    }
    return false;
}

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, int ND, int NC>
hipError_t run_expmv(const mg_ops* ops, const char* tables, size_t tbytes, int64_t P, int K,
                     const double* u0, int bc, double* uT, double tol, int precision,
                     int32_t* stats, int32_t* flags, hipStream_t s) {
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    // the tables must have the row layout the kernel reads
    if (ops->NBP != table_stride<R0, R1, R2, QMAX, ND>() || (ops->NC > 0) != (NC > 0) ||
        (NC > 0 && ops->nv_pad != NW * RJ))
        return hipErrorInvalidValue;
    if (precision == MG_FP64) {
        const size_t lds = resident_lds_bytes<PX, NW, RH, double>() +
                           (NC > 0 ? (size_t)ops->NXV * 64 * PX * sizeof(double) : 0);
        auto kern = expmv_resident_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX, ND, NC>;
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)P), dim3(64 * NW), lds, s, tables, tbytes, K,
                           ops->grid.nx, ops->grid.nv, u0, bc, uT, tol, stats, flags,
                           ops->xdiag_dev, NC > 0 ? mg_xchain_dev(ops) : nullptr,
                           NC > 0 ? mg_xdesc_dev(ops) : nullptr, ops->NC, ops->NXV);
    } else if constexpr (NC > 0) {
        return hipErrorInvalidValue;   // x-terms: FP64 only
    } else {
        constexpr size_t lds =
            f32c_stages_rows<PX>()
                ? resident_lds_with_ctab<PX, RJ, NW, RH, table_stride<R0, R1, R2, QMAX, ND>(),
                                         float>()
                : resident_lds_bytes<PX, NW, RH, float>();
        auto kern = expmv_resident_f32c_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX, ND>;
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)P), dim3(64 * NW), lds, s, tables, tbytes, K,
                           ops->grid.nx, ops->grid.nv, u0, bc, uT, (float)tol, stats, flags,
                           ops->xdiag_dev);
    }
    return hipGetLastError();
}

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, int ND, int NC>
hipError_t run_euler(const mg_ops* ops, double* u, int64_t P, const double* dWE, int NE,
                     double dt, int32_t* flags, hipStream_t s) {
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    if (ops->NBP != table_stride<R0, R1, R2, QMAX, ND>() || (NC > 0) != ops->xt_in_ba)
        return hipErrorInvalidValue;
    const size_t lds = halo_bytes<PX, NW, RH, double>() + 16 +
                       (NC > 0 ? (size_t)ops->NXV * 64 * PX * sizeof(double) : 0);
    auto kern = euler_resident_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX, ND, NC>;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)P), dim3(64 * NW), lds, s, ops->basis_dev,
                       ops->grid.nx, ops->grid.nv, ops->nv_pad, u, dWE, NE, dt, flags,
                       ops->xdiag_dev, NC > 0 ? mg_xchain_dev(ops) : nullptr,
                       NC > 0 ? mg_xdesc_dev(ops) : nullptr, ops->NC, ops->NXV);
    return hipGetLastError();
}

// Instantiated band shapes (R0, R1, R2, QMAX), matching the table layouts the
// host builder rounds to: (1,0,0,1) and (2,1,0,1) cover orders 1 and 2 of the
// constant-coefficient Langevin operator, (2,1,1,2) its order 3, (3,3,3,2)
// v-dependent coefficients.  B and A (Euler) only carry Dt^0 and Dt^1.
#define MG_FOR_SHAPE(PX, RJ, NW, FULLX, CALL)                                                  \
    if (ops->ND == 3) {                                                                        \
        if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 1, 0, 0, 1, FULLX, 3, 0); \
        if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, 3, 0); \
        return hipErrorInvalidValue;                                                           \
    }                                                                                          \
    if (ops->ND == MG_MAX_XDIAG) {                                                             \
        if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 1, 0, 0, 1, FULLX, MG_MAX_XDIAG, 0); \
        if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, MG_MAX_XDIAG, 0); \
        return hipErrorInvalidValue;                                                           \
    }                                                                                          \
    if (ops->ND > 0) return hipErrorInvalidValue;                                              \
    if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 1, 0, 0, 1, FULLX, 0, 0); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, 0, 0); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 1 && qmax == 2) return CALL(PX, RJ, NW, 2, 1, 1, 2, FULLX, 0, 0); \
    if (R[0] == 3 && R[1] == 3 && R[2] == 3 && qmax == 2) return CALL(PX, RJ, NW, 3, 3, 3, 2, FULLX, 0, 0); \
    return hipErrorInvalidValue;
// operators with x-terms (x-dependent noise meeting D^x): four x-factors, any
// number of x-terms (a run-time loop), the order-2 band shape (FP64)
#define MG_FOR_SHAPE_CHAINS(PX, RJ, NW, FULLX, CALL)                                           \
    if (ops->ND == MG_MAX_XDIAG && ops->NC > 0 && R[0] == 2 && R[1] == 1 && R[2] == 0 &&       \
        qmax == 1)                                                                             \
        return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, MG_MAX_XDIAG, 1);                           \
    return hipErrorInvalidValue;

#define MG_SHAPE_CASE(SPX, SRJ, SNW, CALL)                                                     \
    if (sh.PX == SPX && sh.RJ == SRJ && sh.NW == SNW) {                                        \
        if (full) { MG_FOR_SHAPE(SPX, SRJ, SNW, true, CALL) } else { MG_FOR_SHAPE(SPX, SRJ, SNW, false, CALL) } \
    }
#define MG_SHAPE_CASE_CHAINS(SPX, SRJ, SNW, CALL)                                              \
    if (sh.PX == SPX && sh.RJ == SRJ && sh.NW == SNW) {                                        \
        if (full) { MG_FOR_SHAPE_CHAINS(SPX, SRJ, SNW, true, CALL) } else { MG_FOR_SHAPE_CHAINS(SPX, SRJ, SNW, false, CALL) } \
    }
#define MG_DISPATCH_CHAINS(CALL)                                                               \
    {                                                                                          \
        const bool full = (nx == 64 * sh.PX);                                                  \
        MG_SHAPE_CASE_CHAINS(1, 16, 2, CALL)                                                   \
        MG_SHAPE_CASE_CHAINS(1, 16, 4, CALL)                                                   \
        MG_SHAPE_CASE_CHAINS(1, 16, 8, CALL)                                                   \
        MG_SHAPE_CASE_CHAINS(2, 16, 4, CALL)                                                   \
        MG_SHAPE_CASE_CHAINS(2, 16, 8, CALL)                                                   \
        return hipErrorInvalidValue;                                                           \
    }
// the default shapes (pick_shape)
#define MG_DISPATCH(CALL)                                                                      \
    {                                                                                          \
        const bool full = (nx == 64 * sh.PX);                                                  \
        MG_SHAPE_CASE(1, 16, 2, CALL)                                                          \
        MG_SHAPE_CASE(1, 16, 4, CALL)                                                          \
        MG_SHAPE_CASE(1, 16, 8, CALL)                                                          \
        MG_SHAPE_CASE(2, 16, 4, CALL)                                                          \
        MG_SHAPE_CASE(2, 16, 8, CALL)                                                          \
        return hipErrorInvalidValue;                                                           \
    }
// the default shapes and the alternatives the autotuner may pick (half the
// rows per wave, twice the waves; the same rows per workgroup)
#define MG_DISPATCH_TUNED(CALL)                                                                \
    {                                                                                          \
        const bool full = (nx == 64 * sh.PX);                                                  \
        MG_SHAPE_CASE(1, 16, 2, CALL)                                                          \
        MG_SHAPE_CASE(1, 16, 4, CALL)                                                          \
        MG_SHAPE_CASE(1, 16, 8, CALL)                                                          \
        MG_SHAPE_CASE(2, 16, 4, CALL)                                                          \
        MG_SHAPE_CASE(2, 16, 8, CALL)                                                          \
        MG_SHAPE_CASE(1, 8, 4, CALL)                                                           \
        MG_SHAPE_CASE(1, 8, 8, CALL)                                                           \
        MG_SHAPE_CASE(1, 8, 16, CALL)                                                          \
        MG_SHAPE_CASE(2, 8, 8, CALL)                                                           \
        MG_SHAPE_CASE(2, 8, 16, CALL)                                                          \
        return hipErrorInvalidValue;                                                           \
    }

// The shape a launch uses: the default, or the one the autotuner recorded in
// the operator for this precision (same x width and rows per workgroup).
bool launch_shape(const mg_ops* ops, int precision, Shape& sh) {
    if (!pick_shape(ops->grid.nx, ops->grid.nv, sh)) return false;
    const int* t = ops->tuned[precision == MG_FP32C ? 1 : 0];
    if (t[0] == sh.PX && t[1] * t[2] == sh.RJ * sh.NW) {
        sh.RJ = t[1];
        sh.NW = t[2];
    }
    return true;
}

}  // namespace

int resident_rows(int nx, int nv) {
    Shape sh;
    return pick_shape(nx, nv, sh) ? sh.NW * sh.RJ : 0;
}

int resident_candidates(int nx, int nv, int (*shapes)[3], int max) {
    Shape sh;
    if (!pick_shape(nx, nv, sh) || max < 1) return 0;
    int n = 0;
    shapes[n][0] = sh.PX, shapes[n][1] = sh.RJ, shapes[n][2] = sh.NW, ++n;
    if (n < max && sh.RJ == 16 && sh.NW <= 8) {
        shapes[n][0] = sh.PX, shapes[n][1] = 8, shapes[n][2] = 2 * sh.NW, ++n;
    }
    return n;
}

hipError_t launch_expmv_resident(const mg_ops* ops, const char* tables, size_t tbytes, int64_t P,
                                 int K, const double* u0, int u0_broadcast, double* uT, double tol,
                                 int precision, int32_t* stats, int32_t* flags, hipStream_t s,
                                 bool dry_run, const int* shape) {
    Shape sh;
    const int nx = ops->grid.nx;
    if (!launch_shape(ops, precision, sh)) return hipErrorInvalidValue;
    if (shape) {
        // an explicit candidate (autotuner): same x width and rows per workgroup
        if (shape[0] != sh.PX || shape[1] * shape[2] != sh.RJ * sh.NW) return hipErrorInvalidValue;
        sh.RJ = shape[1];
        sh.NW = shape[2];
    }
    if (dry_run) return hipSuccess;
    const int* R = ops->R;
    const int qmax = ops->qmax;
#define MG_CALL_EXPMV(PX, RJ, NW, R0, R1, R2, QM, FX, ND, NC)                               \
    run_expmv<PX, RJ, NW, R0, R1, R2, QM, FX, ND, NC>(ops, tables, tbytes, P, K, u0, u0_broadcast, \
                                                  uT, tol, precision, stats, flags, s)
    if (ops->NC > 0) MG_DISPATCH_CHAINS(MG_CALL_EXPMV)   // chains: the default shapes
    MG_DISPATCH_TUNED(MG_CALL_EXPMV)
#undef MG_CALL_EXPMV
}

hipError_t launch_euler_resident(const mg_ops* ops, double* u, int64_t P, const double* dWE,
                                 int NE, double dt, int32_t* flags, hipStream_t s, bool dry_run) {
    Shape sh;
    const int nx = ops->grid.nx, nv = ops->grid.nv;
    if (!pick_shape(nx, nv, sh)) return hipErrorInvalidValue;
    if (dry_run) return hipSuccess;
    const int* R = ops->R;
    const int qmax = ops->qmax;
#define MG_CALL_EULER(PX, RJ, NW, R0, R1, R2, QM, FX, ND, NC) \
    run_euler<PX, RJ, NW, R0, R1, R2, 1, FX, ND, NC>(ops, u, P, dWE, NE, dt, flags, s)
    // x-terms in B or A: the x-term kernels of the default shapes
    if (ops->xt_in_ba) MG_DISPATCH_CHAINS(MG_CALL_EULER)
    MG_DISPATCH(MG_CALL_EULER)
#undef MG_CALL_EULER
}
