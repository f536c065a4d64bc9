// Device helpers shared by the Taylor-chain kernels (register-resident and
// cooperative): DPP lane shifts, wave reductions, the banded-Kronecker row
// operator, LDS halo slots and the per-(path, step) table view.
#pragma once

#include <type_traits>
#include <cmath>

#include "mg_internal.h"

namespace mgk {

// ---- per-type lane shifts, max and broadcast ---------------------------------
// wave_shr:1 (lane l receives lane l-1) and wave_shl:1 (lane l receives l+1),
// zero fill beyond the wave.
template <class T> __device__ T from_left(T x);
template <class T> __device__ T from_right(T x);
template <> __device__ inline double from_left<double>(double x) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <> __device__ inline double from_right<double>(double x) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <> __device__ inline float from_left<float>(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
template <> __device__ inline float from_right<float>(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}

// max(acc, |x|) as one v_max with an abs source modifier (fmax() adds an IEEE
// canonicalisation per operand).  NaN inputs may be dropped; non-finite
// states are detected separately at the end of the launch.
__device__ inline double max_abs(double acc, double x) {
    double r;
    asm("v_max_f64 %0, %1, |%2|" : "=v"(r) : "v"(acc), "v"(x));
    return r;
}
__device__ inline float max_abs(float acc, float x) {
    float r;
    asm("v_max_f32 %0, %1, |%2|" : "=v"(r) : "v"(acc), "v"(x));
    return r;
}

template <class T>
__device__ inline T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) v = max_abs(v, __shfl_xor(v, o, 64));
    return v;
}

// Wave-uniform copy of a value every lane holds identically.
__device__ inline double uniform(double x) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ inline float uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Dt y at this lane's PX points: y[q+1] - y[q-1] with neighbours from the
// adjacent lanes (zero beyond the wave, which is the zero boundary).
template <int PX, class T>
__device__ inline void dt_apply(const T (&y)[PX], T (&out)[PX]) {
    const T left = from_left<T>(y[PX - 1]);
    const T right = from_right<T>(y[0]);
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        const T a = (q + 1 < PX) ? y[q + 1] : right;
        const T b = (q > 0) ? y[q - 1] : left;
        out[q] = a - b;
    }
}

// The raw second difference Dxx = tridiag(1, -2, 1) along x with zero outside
// the wave, as dt_apply.
template <int PX, class T>
__device__ inline void dxx_apply(const T (&y)[PX], T (&out)[PX]) {
    const T left = from_left<T>(y[PX - 1]);
    const T right = from_right<T>(y[0]);
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        const T a = (q + 1 < PX) ? y[q + 1] : right;
        const T b = (q > 0) ? y[q - 1] : left;
        out[q] = (a + b) - T(2) * y[q];
    }
}
// One letter of an x word: Dt (dxx false) or Dxx (dxx true), wave-uniform.
template <int PX, class T>
__device__ inline void letter_apply(bool dxx, const T (&y)[PX], T (&out)[PX]) {
    if (dxx) dxx_apply<PX, T>(y, out);
    else dt_apply<PX, T>(y, out);
}

// Max over the 64 lanes of non-negative values with DPP row shifts and row
// broadcasts (no LDS traffic); the result is returned wave-uniform (lane 63's
// value read into scalar registers).
template <int CTRL, int ROWMASK>
__device__ inline double dpp_pull(double x) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), CTRL,
                                               ROWMASK, 0xf, CTRL < 0x140);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), CTRL,
                                               ROWMASK, 0xf, CTRL < 0x140);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ inline float dpp_pull(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                      CTRL, ROWMASK, 0xf, CTRL < 0x140));
}
template <int L>
__device__ inline double lane_value(double x) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), L);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), L);
    return __hiloint2double(hi, lo);
}
template <int L>
__device__ inline float lane_value(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), L));
}
// row_shr:1,2,4,8 leave each 16-lane row's maximum in its lane 15 (lanes
// without a source read zero, harmless for non-negative values);
// row_bcast:15 and row_bcast:31 then carry rows 0..2 into lane 63.
template <class T>
__device__ inline T wave_max_dpp(T x) {
    x = max_abs(x, dpp_pull<0x111, 0xf>(x));
    x = max_abs(x, dpp_pull<0x112, 0xf>(x));
    x = max_abs(x, dpp_pull<0x114, 0xf>(x));
    x = max_abs(x, dpp_pull<0x118, 0xf>(x));
    x = max_abs(x, dpp_pull<0x142, 0xa>(x));
    x = max_abs(x, dpp_pull<0x143, 0xc>(x));
    return lane_value<63>(x);
}

template <int R0, int R1, int R2, int Q = 2>
struct Bands {
    static constexpr int RH = (R0 > R1 ? (R0 > R2 ? R0 : R2) : (R1 > R2 ? R1 : R2));
    static constexpr int O1 = 2 * R0 + 1;
    static constexpr int O2 = O1 + 2 * R1 + 1;
    // the V2 band is stored only where Dt^2 occurs (Q = highest power of Dt)
    static constexpr int NB = O2 + (Q >= 2 ? 2 * R2 + 1 : 0);
    static constexpr int NBP = (NB + 1) & ~1;
};

// One application of the banded-Kronecker operator to the RJ rows of this
// wave into a separate output array.  `din(rr, q)` yields the input row rr in
// [-RH, RJ + RH).  `coef(r, e)` is the coefficient e of local row r; rows
// beyond nv have zero coefficients in the (padded) tables, so they produce
// zeros without a branch.  QMAX is the highest power of Dt present.
template <int PX, int RJ, int R0, int R1, int R2, int QMAX, bool FULLX, class T, class In,
          class Coef>
__device__ inline void apply_operator(In din, Coef coef, int lane, int nx, T (&out)[RJ][PX]) {
    using BD = Bands<R0, R1, R2, QMAX>;
    constexpr int NB = BD::NB;
    T cur[NB], nxt[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) cur[e] = coef(0, e);
#pragma unroll
    for (int r = 0; r < RJ; ++r) {
        if (r + 1 < RJ) {
#pragma unroll
            for (int e = 0; e < NB; ++e) nxt[e] = coef(r + 1, e);
        }
        T y0[PX], y1[PX], y2[PX];
#pragma unroll
        for (int q = 0; q < PX; ++q) y0[q] = y1[q] = y2[q] = T(0);
#pragma unroll
        for (int b = -R0; b <= R0; ++b)
#pragma unroll
            for (int q = 0; q < PX; ++q) y0[q] = fma(cur[b + R0], din(r + b, q), y0[q]);
        if (QMAX >= 1) {
#pragma unroll
            for (int b = -R1; b <= R1; ++b)
#pragma unroll
                for (int q = 0; q < PX; ++q)
                    y1[q] = fma(cur[BD::O1 + b + R1], din(r + b, q), y1[q]);
        }
        if (QMAX >= 2) {
#pragma unroll
            for (int b = -R2; b <= R2; ++b)
#pragma unroll
                for (int q = 0; q < PX; ++q)
                    y2[q] = fma(cur[BD::O2 + b + R2], din(r + b, q), y2[q]);
            T t[PX];
            dt_apply<PX, T>(y2, t);
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                y1[q] += t[q];
                // the inner Dt result lives on the grid only (truncated product)
                if (!FULLX && lane * PX + q >= nx) y1[q] = T(0);
            }
        }
        if (QMAX >= 1) {
            T t[PX];
            dt_apply<PX, T>(y1, t);
#pragma unroll
            for (int q = 0; q < PX; ++q) y0[q] += t[q];
        }
#pragma unroll
        for (int q = 0; q < PX; ++q) out[r][q] = (!FULLX && lane * PX + q >= nx) ? T(0) : y0[q];
        if (r + 1 < RJ) {
#pragma unroll
            for (int e = 0; e < NB; ++e) cur[e] = nxt[e];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Default for the x-term accessors of the x-factor operators (no x-terms).
struct NoChains {
    template <class... A>
    __device__ double operator()(A...) const { return 0.0; }
};

// x-terms C_k (x) X_k of row r, added to y.  X_k = diag(x_0) L_1 diag(x_1)
// ... L_d diag(x_d) has depth d <= 2, each letter L_h the raw first difference
// Dt or second difference Dxx (the coefficients carry 1/(2 dx) and 1/dx^2);
// `xt.desc(k)` is {d + 4 [L_1 = Dxx] + 8 [L_2 = Dxx], outer, middle, inner}
// (vector slots of x_0, x_1 and x_d; a depth-0 or depth-1 term has no middle
// one),
// `xt.vec(v, q)` vector v at this lane's point q, zero beyond nx, so the next
// vector cuts every Dt result back to the grid: the truncated matrix product.
// `ccoef(r, e)` is coefficient e of row r in the x-term section of the table
// (xt.n bands of 2 RC + 1).  The term count is a run-time value: one loop
// iteration per term.
template <int PX, int RC, class T, class Din, class CCoef, class XT>
__device__ inline void add_xterms(int r, T (&y)[PX], Din din, CCoef ccoef, const XT& xt) {
    constexpr int WL = 2 * RC + 1;
#pragma unroll 1
    for (int k = 0; k < xt.n; ++k) {
        const int4 ds = xt.desc(k);
        T w[PX];
        {
            const T c0 = ccoef(r, k * WL);
#pragma unroll
            for (int q = 0; q < PX; ++q) w[q] = c0 * din(r - RC, q);
        }
#pragma unroll
        for (int b = 1; b < WL; ++b) {
            const T c = ccoef(r, k * WL + b);
#pragma unroll
            for (int q = 0; q < PX; ++q) w[q] = fma(c, din(r - RC + b, q), w[q]);
        }
#pragma unroll
        for (int q = 0; q < PX; ++q) w[q] *= xt.vec(ds.w, q);
        const int depth = ds.x & 3;
        if (depth >= 1) {
            T e[PX];
            // the innermost letter first: L_2 for depth 2, L_1 for depth 1
            letter_apply<PX, T>(depth == 2 ? ((ds.x >> 3) & 1) : ((ds.x >> 2) & 1), w, e);
            if (depth == 2) {
#pragma unroll
                for (int q = 0; q < PX; ++q) e[q] *= xt.vec(ds.z, q);
                letter_apply<PX, T>((ds.x >> 2) & 1, e, w);
            } else {
#pragma unroll
                for (int q = 0; q < PX; ++q) w[q] = e[q];
            }
        }
#pragma unroll
        for (int q = 0; q < PX; ++q) y[q] = fma(xt.vec(ds.y, q), w[q], y[q]);
    }
}

// The x-term accessor of the kernels: descriptors in global memory (read at
// wave-uniform addresses, so through the scalar cache), vectors
// [NXV][64*PX] in LDS.
template <int PX, class T>
struct XTerms {
    int n;
    const int4* __restrict__ descs;
    const T* vecs;
    int lane;
    __device__ int4 desc(int k) const { return descs[k]; }
    __device__ T vec(int v, int q) const { return vecs[v * 64 * PX + lane * PX + q]; }
};

// One application of the banded-Kronecker operator to the RJ rows of this
// wave, in place: d holds the input rows, top/bot the RH halo rows above and
// below.  Row r of the result y is handed to `emit(r, y)`, which returns the
// value that replaces d[r]; the replacement is committed RH rows later, once
// no later row reads the old d[r], so only RH + 1 result rows are live at a
// time.  `coef(r, e)` is the coefficient e of local row r; rows beyond nv have
// zero coefficients in the (padded) tables, so they produce zeros without a
// branch.  QMAX is the highest power of Dt present.
// SEG computes rows RH .. RJ-1 first and rows 0 .. RH-1 last (each row's
// arithmetic is the same; the old values of rows RH .. 2RH-1, which the last
// rows read, are kept when those rows are committed), so that neither halo
// is read before step RJ - 2RH.  `hook(i)` runs before the i-th row computed;
// the cooperative kernel uses it to take part in its group's exchange while
// the rows that do not need the halo rows are computed.  `emit` may take the
// row's input accessor as a third argument (it reads the kept rows).
struct NoHook {
    __device__ void operator()(int) const {}
};
template <int PX, int RJ, int R0, int R1, int R2, int QMAX, bool FULLX, int RH, class T,
          class Coef, class Emit, bool SEG = false, class Hook = NoHook>
__device__ inline void apply_inplace(T (&d)[RJ][PX], const T (&top)[RH][PX],
                                     const T (&bot)[RH][PX], Coef coef, int lane, int nx,
                                     Emit emit, Hook hook = Hook{}) {
    using BD = Bands<R0, R1, R2, QMAX>;
    constexpr int NB = BD::NB;
    static_assert(!SEG || RJ > 2 * RH, "segmented order needs more than 2 RH rows");
    // row computed at step i
    auto row_at = [](int i) -> int {
        return SEG ? (i < RJ - RH ? RH + i : i - (RJ - RH)) : i;
    };
    T res[RJ][PX];
    T keep[RH][PX];   // SEG: old rows RH .. 2RH-1
    // coefficients of the current row; the next row's are loaded while the
    // current one is computed (scheduling barriers keep the scalar loads from
    // being hoisted all at once)
    T cur[NB], nxt[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) cur[e] = coef(row_at(0), e);
#pragma unroll
    for (int i = 0; i < RJ; ++i) {
        const int r = row_at(i);
        const bool last_seg = SEG && i >= RJ - RH;
        auto din = [&](int rr, int q) -> T {
            if (rr < 0) return top[rr + RH][q];
            if (rr >= RJ) return bot[rr - RJ][q];
            if (last_seg && rr >= RH && rr < 2 * RH) return keep[rr - RH][q];
            return d[rr][q];
        };
        hook(i);
        if (i + 1 < RJ) {
#pragma unroll
            for (int e = 0; e < NB; ++e) nxt[e] = coef(row_at(i + 1), e);
        }
        T y0[PX], y1[PX], y2[PX];
#pragma unroll
        for (int q = 0; q < PX; ++q) y0[q] = y1[q] = y2[q] = T(0);
#pragma unroll
        for (int b = -R0; b <= R0; ++b)
#pragma unroll
            for (int q = 0; q < PX; ++q) y0[q] = fma(cur[b + R0], din(r + b, q), y0[q]);
        if (QMAX >= 1) {
#pragma unroll
            for (int b = -R1; b <= R1; ++b)
#pragma unroll
                for (int q = 0; q < PX; ++q)
                    y1[q] = fma(cur[BD::O1 + b + R1], din(r + b, q), y1[q]);
        }
        if (QMAX >= 2) {
#pragma unroll
            for (int b = -R2; b <= R2; ++b)
#pragma unroll
                for (int q = 0; q < PX; ++q)
                    y2[q] = fma(cur[BD::O2 + b + R2], din(r + b, q), y2[q]);
            T t[PX];
            dt_apply<PX, T>(y2, t);
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                y1[q] += t[q];
                // the inner Dt result lives on the grid only (truncated product)
                if (!FULLX && lane * PX + q >= nx) y1[q] = T(0);
            }
        }
        if (QMAX >= 1) {
            T t[PX];
            dt_apply<PX, T>(y1, t);
#pragma unroll
            for (int q = 0; q < PX; ++q) y0[q] += t[q];
        }
#pragma unroll
        for (int q = 0; q < PX; ++q)
            if (!FULLX && lane * PX + q >= nx) y0[q] = T(0);
        if constexpr (std::is_invocable_v<Emit, int, T (&)[PX], decltype(din)>)
            emit(r, y0, din);
        else
            emit(r, y0);
#pragma unroll
        for (int q = 0; q < PX; ++q) res[r][q] = y0[q];
        if constexpr (SEG) {
            // the row is computed here: without this the hook's control flow
            // lets the rows before it sink past it, where their operands
            // then stay live (the register file overflows)
#pragma unroll
            for (int q = 0; q < PX; ++q) asm volatile("" : "+v"(res[r][q]));
        }
        // commit row k once no row still to be computed reads its old value
        auto commit = [&](int k) {
            if (SEG && k >= RH && k < 2 * RH) {
#pragma unroll
                for (int q = 0; q < PX; ++q) keep[k - RH][q] = d[k][q];
            }
#pragma unroll
            for (int q = 0; q < PX; ++q) d[k][q] = res[k][q];
        };
        if (!SEG && r >= RH) commit(r - RH);
        if (SEG && !last_seg) {
            if (r - RH >= RH) commit(r - RH);
            if (i == RJ - RH - 1) {
#pragma unroll
                for (int k = (RJ - RH > RH ? RJ - RH : RH); k < RJ; ++k) commit(k);
            }
        }
        if (i + 1 < RJ) {
#pragma unroll
            for (int e = 0; e < NB; ++e) cur[e] = nxt[e];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    // the last RH rows computed
    constexpr int rlo = SEG ? 0 : (RJ > RH ? RJ - RH : 0);
    constexpr int rhi = SEG ? RH : RJ;
#pragma unroll
    for (int r = rlo; r < rhi; ++r)
#pragma unroll
        for (int q = 0; q < PX; ++q) d[r][q] = res[r][q];
}


// apply_inplace with x-dependent factors: every factor W_t (x) diag(a_t) adds
// a_t(x) * sum_b W_t[j][b] d(j+b) to row j before it is emitted (a_t at this
// lane's point q is xa(t, q)).  The W bands follow the V bands in the table row; their
// coefficients are requested at the start of the row.  Row r is emitted before
// apply_inplace overwrites d[r - RH], so the rows r - RW .. r + RW read here
// are still the input (RW <= RH).
// The rows are read through the accessor apply_inplace hands to the emit
// (in its SEG order it reads the kept rows).
template <int PX, int RJ, int R0, int R1, int R2, int QMAX, bool FULLX, int RH, int ND, int RW,
          class T, class Coef, class XA, class Emit, int NC = 0, class CCoef = NoChains,
          class CVec = NoChains, bool SEG = false, class Hook = NoHook>
__device__ inline void apply_inplace_x(T (&d)[RJ][PX], const T (&top)[RH][PX],
                                       const T (&bot)[RH][PX], Coef coef, XA xa, int lane, int nx,
                                       Emit emit, CCoef ccoef = CCoef{}, CVec cvec = CVec{},
                                       Hook hook = Hook{}) {
    constexpr int NBM = Bands<R0, R1, R2, QMAX>::NB;
    constexpr int WL = 2 * RW + 1;
    static_assert(RW <= RH, "halo narrower than the x-dependent factors");
    auto xemit = [&](int r, T (&y)[PX], auto din) {
            T w[ND][WL];
#pragma unroll
            for (int t = 0; t < ND; ++t)
#pragma unroll
                for (int b = 0; b < WL; ++b) w[t][b] = coef(r, NBM + t * WL + b);
#pragma unroll
            for (int t = 0; t < ND; ++t) {
                T z[PX];
#pragma unroll
                for (int q = 0; q < PX; ++q) z[q] = w[t][0] * din(r - RW, q);
#pragma unroll
                for (int b = 1; b < WL; ++b)
#pragma unroll
                    for (int q = 0; q < PX; ++q) z[q] = fma(w[t][b], din(r - RW + b, q), z[q]);
#pragma unroll
                for (int q = 0; q < PX; ++q) y[q] = fma(xa(t, q), z[q], y[q]);
            }
            if constexpr (NC > 0) add_xterms<PX, RW, T>(r, y, din, ccoef, cvec);
            emit(r, y);
        };
    apply_inplace<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T, Coef, decltype(xemit), SEG, Hook>(
        d, top, bot, coef, lane, nx, xemit, hook);
}

// One application of the banded-Kronecker operator in "difference first" form,
// from d into a separate output.  Because V_q acts along v and Dt along x,
// Coefficient rows copied into LDS: apply_split requests them one row ahead
// instead of two (an LDS read returns far sooner than a scalar-cache miss,
// and every row held ahead costs NB registers per lane).
template <class T, int NBP>
struct LdsRows {
    const T* rows;
    __device__ T operator()(int r, int e) const { return rows[r * NBP + e]; }
};
template <class C>
struct coef_ahead {
    static constexpr int value = 2;
};
template <class T, int NBP>
struct coef_ahead<LdsRows<T, NBP>> {
    static constexpr int value = 1;
};

// V_q (x) Dt^q = (V_q (x) I)(I (x) Dt^q): each row's x differences e1 = Dt d and
// e2 = Dt e1 (truncated to the grid) are formed once, and every output point is
// a single FMA chain over the bands,
//   y(j) = sum_b V0[j][b] d(j+b) + sum_b V1[j][b] e1(j+b) + sum_b V2[j][b] e2(j+b).
// Rows are produced in the order RH .. RJ-1, then 0 .. RH-1, so the halo rows
// (read from LDS by fetch_bot / fetch_top a few rows before their first use)
// arrive while interior rows are computed.  Each row's coefficients are
// requested one row ahead.  Row r of the result goes to emit(r, y), which may
// rescale y before it is stored in out[r].  Rows beyond nv have zero
// coefficients in the padded tables; points beyond nx stay zero because every
// input is zero there.
template <int PX, int RJ, int R0, int R1, int R2, int QMAX, bool FULLX, int RH, class T,
          class Coef, class FetchBot, class FetchTop, class Emit>
__device__ inline void apply_split(const T (&d)[RJ][PX], T (&out)[RJ][PX], T (&top)[RH][PX],
                                   T (&bot)[RH][PX], FetchBot fetch_bot, FetchTop fetch_top,
                                   Coef coef, int lane, int nx, Emit emit) {
    using BD = Bands<R0, R1, R2, QMAX>;
    constexpr int NB = BD::NB;
    constexpr int A2 = QMAX >= 2 ? R2 : 0;                    // e2 rows needed ahead
    constexpr int A1 = QMAX >= 1 ? (A2 > R1 ? A2 : R1) : 0;   // e1 rows needed ahead
    static_assert(A1 <= RH && A2 <= RH, "halo narrower than the difference window");
    static_assert(RJ >= 2 * RH + 1, "too few rows per wave for the halo width");
    // first row of the first pass that reads a bottom halo row, and the fetch
    // points two rows ahead of first use
    constexpr int RB = RJ - (R0 > A1 ? R0 : A1);
    constexpr int FB = (RB - 2 > RH) ? RB - 2 : RH;
    constexpr int FT = (RJ - 2 > RH) ? RJ - 2 : RH;
    auto din = [&](int rr, int q) -> T {
        if (rr < 0) return top[rr + RH][q];
        if (rr >= RJ) return bot[rr - RJ][q];
        return d[rr][q];
    };
    T e1[RJ + 2 * RH][PX], e2[RJ + 2 * RH][PX];   // row rr at index rr + RH
    auto make_e1 = [&](int rr) {
        T v[PX];
#pragma unroll
        for (int q = 0; q < PX; ++q) v[q] = din(rr, q);
        dt_apply<PX, T>(v, e1[rr + RH]);
        if (!FULLX) {
#pragma unroll
            for (int q = 0; q < PX; ++q)
                if (lane * PX + q >= nx) e1[rr + RH][q] = T(0);
        }
    };
    auto make_e2 = [&](int rr) {
        dt_apply<PX, T>(e1[rr + RH], e2[rr + RH]);
        if (!FULLX) {
#pragma unroll
            for (int q = 0; q < PX; ++q)
                if (lane * PX + q >= nx) e2[rr + RH][q] = T(0);
        }
    };
    auto order = [](int i) { return i < RJ - RH ? i + RH : i - (RJ - RH); };
    // coefficients of the current row and of the next AH (requested two rows
    // ahead from the scalar cache, where a miss costs more than one row of
    // work, one row ahead from LDS)
    constexpr int AH = coef_ahead<Coef>::value;
    static_assert(AH == 1 || AH == 2, "coefficients are requested one or two rows ahead");
    T cur[NB], nxt[NB], nx2[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) cur[e] = coef(order(0), e);
    if constexpr (AH == 2) {
#pragma unroll
        for (int e = 0; e < NB; ++e) nxt[e] = coef(order(1), e);
    }
    // differences for the start of the first pass (rows RH - A .. RH + A - 1)
    if (QMAX >= 1) {
#pragma unroll
        for (int rr = RH - A1; rr < RH + A1; ++rr) make_e1(rr);
    }
    if (QMAX >= 2) {
#pragma unroll
        for (int rr = RH - A2; rr < RH + A2; ++rr) make_e2(rr);
    }
#pragma unroll
    for (int i = 0; i < RJ; ++i) {
        const int r = order(i);
        if (i + AH < RJ) {
            const int rn = order(i + AH);
#pragma unroll
            for (int e = 0; e < NB; ++e) (AH == 2 ? nx2 : nxt)[e] = coef(rn, e);
        }
        if (r == FB) fetch_bot();
        if (r == FT) fetch_top();
        __builtin_amdgcn_sched_barrier(0);
        if (i == RJ - RH) {
            // second pass: differences of the rows above the first pass
            if (QMAX >= 1) {
#pragma unroll
                for (int rr = -A1; rr < RH - A1; ++rr) make_e1(rr);
            }
            if (QMAX >= 2) {
#pragma unroll
                for (int rr = -A2; rr < RH - A2; ++rr) make_e2(rr);
            }
        }
        if (i < RJ - RH) {
            if (QMAX >= 1) make_e1(r + A1);
            if (QMAX >= 2) make_e2(r + A2);
        }
        T y[PX];
#pragma unroll
        for (int q = 0; q < PX; ++q) y[q] = cur[0] * din(r - R0, q);
#pragma unroll
        for (int b = -R0 + 1; b <= R0; ++b)
#pragma unroll
            for (int q = 0; q < PX; ++q) y[q] = fma(cur[b + R0], din(r + b, q), y[q]);
        if (QMAX >= 1) {
#pragma unroll
            for (int b = -R1; b <= R1; ++b)
#pragma unroll
                for (int q = 0; q < PX; ++q)
                    y[q] = fma(cur[BD::O1 + b + R1], e1[r + b + RH][q], y[q]);
        }
        if (QMAX >= 2) {
#pragma unroll
            for (int b = -R2; b <= R2; ++b)
#pragma unroll
                for (int q = 0; q < PX; ++q)
                    y[q] = fma(cur[BD::O2 + b + R2], e2[r + b + RH][q], y[q]);
        }
        emit(r, y);
#pragma unroll
        for (int q = 0; q < PX; ++q) out[r][q] = y[q];
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            cur[e] = nxt[e];
            if (AH == 2) nxt[e] = nx2[e];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// apply_split with x-dependent factors: after the V bands, every factor
// W_t (x) diag(a_t) adds a_t(x) * sum_b W_t[j][b] d(j+b) to the row, with
// a_t at this lane's points in xa.  The W bands follow the V bands in the table
// row (NBM coefficients); their coefficients are requested at the start of the
// row.  RH must cover RW.

template <int PX, int RJ, int R0, int R1, int R2, int QMAX, bool FULLX, int RH, int ND, int RW,
          class T, class Coef, class FetchBot, class FetchTop, class Emit, int NC = 0,
          class CCoef = NoChains, class CVec = NoChains>
__device__ inline void apply_split_x(const T (&d)[RJ][PX], T (&out)[RJ][PX], T (&top)[RH][PX],
                                     T (&bot)[RH][PX], FetchBot fetch_bot, FetchTop fetch_top,
                                     Coef coef, const T (&xa)[ND][PX], int lane, int nx,
                                     Emit emit, CCoef ccoef = CCoef{}, CVec cvec = CVec{}) {
    constexpr int NBM = Bands<R0, R1, R2, QMAX>::NB;
    constexpr int WL = 2 * RW + 1;
    static_assert(RW <= RH, "halo narrower than the x-dependent factors");
    auto din = [&](int rr, int q) -> T {
        if (rr < 0) return top[rr + RH][q];
        if (rr >= RJ) return bot[rr - RJ][q];
        return d[rr][q];
    };
    // the first RB row that reads a bottom halo row, with the W bands included
    constexpr int RWB = RW > R0 ? RW : R0;
    apply_split<PX, RJ, (RWB > R0 ? RWB : R0), R1, R2, QMAX, FULLX, RH, T>(
        d, out, top, bot, fetch_bot, fetch_top,
        [&](int r, int e) -> T {
            // the widened V0 band of apply_split: pad with zeros around V0
            constexpr int PAD = (RWB > R0 ? RWB : R0) - R0;
            constexpr int O1W = 2 * (R0 + PAD) + 1;
            if (e < O1W) {
                const int b = e - PAD;
                return (b >= 0 && b < 2 * R0 + 1) ? coef(r, b) : T(0);
            }
            return coef(r, e - 2 * PAD);
        },
        lane, nx, [&](int r, T (&y)[PX]) {
            T w[ND][WL];
#pragma unroll
            for (int t = 0; t < ND; ++t)
#pragma unroll
                for (int b = 0; b < WL; ++b) w[t][b] = coef(r, NBM + t * WL + b);
#pragma unroll
            for (int t = 0; t < ND; ++t) {
                T z[PX];
#pragma unroll
                for (int q = 0; q < PX; ++q) z[q] = w[t][0] * din(r - RW, q);
#pragma unroll
                for (int b = 1; b < WL; ++b)
#pragma unroll
                    for (int q = 0; q < PX; ++q) z[q] = fma(w[t][b], din(r - RW + b, q), z[q]);
#pragma unroll
                for (int q = 0; q < PX; ++q) y[q] = fma(xa[t][q], z[q], y[q]);
            }
            if constexpr (NC > 0) add_xterms<PX, RW, T>(r, y, din, ccoef, cvec);
            emit(r, y);
        });
}

// Halo rows per side a kernel shape needs: the widest band, including the
// bands of the x-dependent factors when there are any.
template <int R0, int R1, int R2, int ND>
constexpr int halo_rows() {
    constexpr int rh = Bands<R0, R1, R2>::RH > 0 ? Bands<R0, R1, R2>::RH : 1;
    return (ND > 0 && MG_XDIAG_RADIUS > rh) ? MG_XDIAG_RADIUS : rh;
}

// Coefficients per table row (padded to an even count): the V bands, then the
// bands of the x-dependent factors.
template <int R0, int R1, int R2, int QMAX, int ND>
constexpr int table_stride() {
    return (Bands<R0, R1, R2, QMAX>::NB + ND * (2 * MG_XDIAG_RADIUS + 1) + 1) & ~1;
}

// apply_split, or apply_split_x when the operator has x-dependent factors.
template <int PX, int RJ, int R0, int R1, int R2, int QMAX, bool FULLX, int RH, int ND, class T,
          int NDX, class Coef, class FetchBot, class FetchTop, class Emit, int NC = 0,
          class CCoef = NoChains, class CVec = NoChains>
__device__ inline void apply_rows_any(const T (&d)[RJ][PX], T (&out)[RJ][PX], T (&top)[RH][PX],
                                      T (&bot)[RH][PX], FetchBot fb, FetchTop ft, Coef coef,
                                      const T (&xa)[NDX][PX], int lane, int nx, Emit emit,
                                      CCoef ccoef = CCoef{}, CVec cvec = CVec{}) {
    if constexpr (ND == 0)
        apply_split<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T>(d, out, top, bot, fb, ft, coef, lane, nx,
                                                            emit);
    else
        apply_split_x<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, MG_XDIAG_RADIUS, T, Coef, FetchBot,
                      FetchTop, Emit, NC, CCoef, CVec>(d, out, top, bot, fb, ft, coef, xa, lane,
                                                      nx, emit, ccoef, cvec);
}

// LDS halo layout: halo[parity][wave + 1][slot][64*PX] for waves -1 .. NW; the
// guard waves -1 and NW are zero rows (the zero boundary in v) so that every
// fetch is unconditional.  Slots 0..RH-1 hold a wave's first RH rows, slots
// RH..2RH-1 its last RH rows.
template <int PX, int RJ, int NW, int RH, class T>
struct Halo {
    T* base;
    __device__ T* slot(int par, int w, int s) const {
        return base + (((size_t)par * (NW + 2) + (w + 1)) * (2 * RH) + s) * (64 * PX);
    }
    __device__ void zero_guards(int tid, int nthreads) const {
        for (int par = 0; par < 2; ++par)
            for (int g = 0; g < 2; ++g) {
                T* p = slot(par, g == 0 ? -1 : NW, 0);
                for (int i = tid; i < 2 * RH * 64 * PX; i += nthreads) p[i] = T(0);
            }
    }
    __device__ void publish(int par, int w, int lane, const T (&d)[RJ][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s) {
            T* top = slot(par, w, s) + lane * PX;
            T* bot = slot(par, w, RH + s) + lane * PX;
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                top[q] = d[s][q];
                bot[q] = d[RJ - RH + s][q];
            }
        }
    }
    // rows -RH..-1 (from wave w-1)
    __device__ void fetch_top(int par, int w, int lane, T (&top)[RH][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) top[s][q] = slot(par, w - 1, RH + s)[lane * PX + q];
    }
    // rows RJ..RJ+RH-1 (from wave w+1)
    __device__ void fetch_bot(int par, int w, int lane, T (&bot)[RH][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) bot[s][q] = slot(par, w + 1, s)[lane * PX + q];
    }
    // rows -RH..-1 (from wave w-1) and RJ..RJ+RH-1 (from wave w+1)
    __device__ void fetch(int par, int w, int lane, T (&top)[RH][PX], T (&bot)[RH][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s) {
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                top[s][q] = slot(par, w - 1, RH + s)[lane * PX + q];
                bot[s][q] = slot(par, w + 1, s)[lane * PX + q];
            }
        }
    }
};

template <int PX, int NW, int RH, class T>
constexpr size_t halo_bytes() {
    return (size_t)2 * (NW + 2) * 2 * RH * 64 * PX * sizeof(T);
}

// LDS: halo | red [2][NW][2] (term norms) | red2 [2][NW] (state norms) | flag
template <int PX, int NW, int RH, class T>
constexpr size_t resident_lds_bytes() {
    return halo_bytes<PX, NW, RH, T>() + (size_t)2 * NW * 2 * sizeof(T) +
           (size_t)2 * NW * sizeof(T) + 16;
}

// LDS of a resident workgroup that also holds the coefficient rows of the
// current (path, step): the halo and reduction area, then NW*RJ rows of NBP.
template <int PX, int NW, int RH, class T>
constexpr size_t resident_ctab_offset() {
    return (resident_lds_bytes<PX, NW, RH, T>() + 15) & ~(size_t)15;
}
template <int PX, int RJ, int NW, int RH, int NBP, class T>
constexpr size_t resident_lds_with_ctab() {
    return resident_ctab_offset<PX, NW, RH, T>() + (size_t)NW * RJ * NBP * sizeof(T);
}

// Table of one (path, step): 64-byte header, then rows of NBP coefficients.
struct TableView {
    const char* base;
    __device__ int s() const { return reinterpret_cast<const int32_t*>(base)[0]; }
    __device__ int m() const { return reinterpret_cast<const int32_t*>(base)[2]; }
    __device__ double es() const { return reinterpret_cast<const double*>(base)[2]; }
    __device__ int flag() const { return reinterpret_cast<const int32_t*>(base)[10]; }
    template <class T>
    __device__ const T* rows() const { return reinterpret_cast<const T*>(base + 64); }
};


}  // namespace mgk
