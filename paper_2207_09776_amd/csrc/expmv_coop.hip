// Cooperative Taylor chain for grids whose per-path state does not fit on one
// workgroup (128 < nx <= 1024).
//
// A path is split along v into G slabs; slab g is held by workgroup g of a
// group of G co-resident workgroups (cooperative launch), in VGPRs, with the
// same lane/row decomposition as the register-resident kernel (lane -> PX
// consecutive x points, wave -> RJ consecutive v rows).  Groups are persistent:
// group q processes paths q, q + ngroups, ...
//
// Per Taylor term the group synchronises once through the workspace:
//   * the first wave publishes its top RH rows and the last wave its bottom RH
//     rows (the halo the neighbouring slabs need), and every wave publishes
//     its inf-norms of the previous term and partial sum (of the state at the
//     start of a sub-step); each wave then waits for its own stores,
//   * after a workgroup barrier wave 0 bumps the workgroup's counter and waits
//     until every member's counter reached the same value,
//   * after a second barrier the edge waves load their neighbours' halo rows
//     and every wave loads the norms of all waves of all members, so every
//     member takes the same early-termination decision.
// Waiting is bounded: after kSpinLimit polls the launch is aborted through a
// shared word, every workgroup leaves its loops and the paths get
// MG_FLAG_ABORT.
//
// Every access to the exchange area (halo rows, norms, counters) is a
// device-coherent (agent-scope) relaxed atomic, which neither hits a stale
// L1 line nor leaves data in a non-coherent cache; a vmcnt(0) wait orders a
// member's data stores before its counter store, and the readers load the
// data after they have seen the counters.  No L2 write-back or invalidation is
// issued, so the per-term synchronisation does not flush the caches that hold
// the coefficient tables.

#include <algorithm>
#include <cmath>

#include "kernel_common.h"

namespace {

using namespace mgk;

constexpr int kSpinLimit = 1 << 22;

struct CoopArgs {
    const char* tables;
    size_t tbytes;
    int K, nx, nv;
    int64_t P;
    const double* u0;
    int u0_bcast;
    double* uT;
    double tol;
    int32_t* stats;
    int32_t* flags;
    // exchange area (in the caller's workspace, zeroed before the launch)
    char* xh;          // halo rows   [ngroups][G][2 parity][2 side][RHX][nx] of T
    double* xn;        // norms       [ngroups][G][2 parity][NW waves][2]
    int* fl;           // counters    [ngroups][G]
    int* abort_word;
    int G;
    int ngroups;
    int xcd_map;       // members of a group on one XCD (blockIdx mod 8)
};

// Stores issued so far by this wave have completed (device-coherent stores
// are then visible to every later device-coherent load).
__device__ inline void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Device-coherent accesses to the exchange area.
template <class T>
__device__ inline T xload(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void xstore(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kRHX = 3;   // halo rows reserved per side in the exchange area

// LDS halo of the cooperative kernel: one buffer, waves 0..NW-1 only; wave w
// writes its first RH rows to slots [w][0..RH) and its last RH rows to
// [w][RH..2RH).  Written before the first barrier of a term and read between
// the two barriers, so one buffer suffices.
template <int PX, int RJ, int NW, int RH, class T>
struct HaloC {
    T* base;
    __device__ T* slot(int w, int s) const { return base + ((size_t)w * (2 * RH) + s) * (64 * PX); }
    __device__ void publish(int w, int lane, const T (&d)[RJ][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                slot(w, s)[lane * PX + q] = d[s][q];
                slot(w, RH + s)[lane * PX + q] = d[RJ - RH + s][q];
            }
    }
    __device__ void fetch(int w, int lane, T (&top)[RH][PX], T (&bot)[RH][PX]) const {
        if (w > 0) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) top[s][q] = slot(w - 1, RH + s)[lane * PX + q];
        }
        if (w + 1 < NW) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) bot[s][q] = slot(w + 1, s)[lane * PX + q];
        }
    }
};

template <int PX, int NW, int RH, class T>
constexpr size_t coop_lds_bytes() {
    return (size_t)NW * 2 * RH * 64 * PX * sizeof(T) + 16;
}

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, bool F32C>
__global__ __launch_bounds__(64 * NW) void expmv_coop_kernel(CoopArgs a) {
    using T = typename std::conditional<F32C, float, double>::type;
    using BD = Bands<R0, R1, R2>;
    constexpr int RH = BD::RH > 0 ? BD::RH : 1;
    constexpr int NBP = BD::NBP;
    constexpr int RW = NW * RJ;
    extern __shared__ double lds_d[];
    T* lds = reinterpret_cast<T*>(lds_d);
    HaloC<PX, RJ, NW, RH, T> halo{lds};
    int* sh = reinterpret_cast<int*>(lds + (size_t)NW * 2 * RH * 64 * PX);   // [0] abort

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = a.G;
    int g, grp;
    {
        const int b = blockIdx.x;
        if (a.xcd_map) {
            const int xcd = b & 7, k = b >> 3;
            g = k % G;
            grp = (k / G) * 8 + xcd;
        } else {
            g = b % G;
            grp = b / G;
        }
    }
    const int nx = a.nx, nv = a.nv;
    const size_t N = (size_t)nx * nv;
    const int row0 = g * RW + w * RJ;                 // first global row of this wave
    const int nrows = min(RJ, max(0, nv - row0));

    int* my_cnt = a.fl + (size_t)grp * G + g;
    const int* grp_cnt = a.fl + (size_t)grp * G;
    T* xh = reinterpret_cast<T*>(a.xh);
    auto xh_row = [&](int member, int par, int side, int s) -> T* {
        return xh + ((((size_t)grp * G + member) * 2 + par) * 2 + side) * (size_t)kRHX * nx +
               (size_t)s * nx;
    };
    // per member and parity: NW pairs (one per wave) of norms
    auto xn_at = [&](int member, int par, int wave) -> double* {
        return a.xn + ((((size_t)grp * G + member) * 2 + par) * NW + wave) * 2;
    };

    int counter = 0;      // group syncs done by this launch
    bool aborted = false;

    // Edge rows of d for the neighbouring slabs (parity of the coming sync).
    auto publish_global = [&](const T (&d)[RJ][PX]) {
        const int par = counter & 1;
        if (w == 0 && g > 0) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    if (i < nx) xstore(xh_row(g, par, 0, s) + i, d[s][q]);
                }
        }
        if (w == NW - 1 && g + 1 < G) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    if (i < nx) xstore(xh_row(g, par, 1, s) + i, d[RJ - RH + s][q]);
                }
        }
    };
    // this wave's pair of norms for the coming sync
    auto publish_pair = [&](double v0, double v1) {
        if (lane == 0) {
            double* x = xn_at(g, counter & 1, w);
            xstore(x, v0);
            xstore(x + 1, v1);
        }
    };

    // One group synchronisation.  Every wave has published its pair and its
    // halo rows and waited for its stores, then the workgroup passed a
    // barrier; wave 0 bumps the counter and waits for the other members.
    auto group_sync = [&]() {
        if (w == 0) {
            if (lane == 0) xstore(my_cnt, counter + 1);
            // wait until every member published this sync (lane m watches member m)
            int spins = 0;
            bool ab = false;
            for (;;) {
                bool ready = true;
                for (int mm = lane; mm < G; mm += 64)
                    if (xload(grp_cnt + mm) < counter + 1) ready = false;
                if (__all(ready)) break;
                if (++spins > kSpinLimit || xload(a.abort_word)) {
                    ab = true;
                    if (lane == 0) xstore(a.abort_word, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0) sh[0] = ab ? 1 : 0;
        }
        __syncthreads();
        // the exchange loads that follow stay after the counter loads
        asm volatile("" ::: "memory");
        aborted = __builtin_amdgcn_readfirstlane(sh[0]) != 0;
    };
    // Maxima over every wave of every member of the pairs of the sync just done.
    auto read_pairs = [&](double (&out)[2]) {
        const int par = counter & 1;
        double o0 = 0.0, o1 = 0.0;
        for (int idx = lane; idx < G * NW; idx += 64) {
            const double* x = xn_at(idx / NW, par, idx % NW);
            o0 = fmax(o0, xload(x));
            o1 = fmax(o1, xload(x + 1));
        }
        for (int o = 32; o > 0; o >>= 1) {
            o0 = fmax(o0, __shfl_xor(o0, o, 64));
            o1 = fmax(o1, __shfl_xor(o1, o, 64));
        }
        out[0] = uniform(o0);
        out[1] = uniform(o1);
        ++counter;
    };

    for (int64_t p = grp; p < a.P && !aborted; p += a.ngroups) {
        // state F (+ compensation L for the FP32 form)
        T F[RJ][PX], L[RJ][PX];
        {
            const double* src = a.u0 + (a.u0_bcast ? 0 : (size_t)p * N);
#pragma unroll
            for (int r = 0; r < RJ; ++r)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    const double u = (r < nrows && i < nx) ? src[(size_t)(row0 + r) * nx + i] : 0.0;
                    F[r][q] = (T)u;
                    L[r][q] = F32C ? (T)(u - (double)F[r][q]) : T(0);
                }
        }
        int pflag = 0;
        for (int k = 0; k < a.K && !aborted; ++k) {
            const TableView tv{a.tables + ((size_t)p * a.K + k) * a.tbytes};
            const int s = tv.s();
            const int m = tv.m();
            const double es = tv.es();
            pflag |= tv.flag();
            const T* rows = tv.rows<T>() + (size_t)row0 * NBP;
            auto coef = [&](int r, int e) -> T { return rows[r * NBP + e]; };
            int terms = 0;
            for (int sub = 0; sub < s && !aborted; ++sub) {
                T d[RJ][PX];
                T sm = 0;
#pragma unroll
                for (int r = 0; r < RJ; ++r)
#pragma unroll
                    for (int q = 0; q < PX; ++q) {
                        d[r][q] = F[r][q];
                        sm = max_abs(sm, F[r][q]);
                    }
                sm = wave_max(sm);
                // this wave's pair for the next sync: the state norm (first
                // term), then the norms of the previous term and partial sum
                double pr0 = (double)uniform(sm), pr1 = 0.0;
                double c1 = 0.0;
                T fj = 1;
                for (int j = 1; j <= m; ++j) {
                    const int par = counter & 1;
                    halo.publish(w, lane, d);
                    publish_global(d);
                    publish_pair(pr0, pr1);
                    wait_stores();
                    __syncthreads();
                    // LDS halo read between the two barriers (the next term
                    // writes it after the second)
                    T top[RH][PX], bot[RH][PX];
                    halo.fetch(w, lane, top, bot);
                    group_sync();
                    if (aborted) break;
                    // neighbours' halo rows and the pairs, loaded together
                    if (w == 0) {
#pragma unroll
                        for (int s2 = 0; s2 < RH; ++s2)
#pragma unroll
                            for (int q = 0; q < PX; ++q) {
                                const int i = lane * PX + q;
                                T v = T(0);
                                if (g > 0 && i < nx) v = xload(xh_row(g - 1, par, 1, s2) + i);
                                top[s2][q] = v;
                            }
                    }
                    if (w == NW - 1) {
#pragma unroll
                        for (int s2 = 0; s2 < RH; ++s2)
#pragma unroll
                            for (int q = 0; q < PX; ++q) {
                                const int i = lane * PX + q;
                                T v = T(0);
                                if (g + 1 < G && i < nx) v = xload(xh_row(g + 1, par, 0, s2) + i);
                                bot[s2][q] = v;
                            }
                    }
                    double got[2];
                    read_pairs(got);
                    if (j == 1) {
                        c1 = got[0];
                    } else {
                        const double c2 = got[0], fn = got[1];
                        if (c1 + c2 <= a.tol * fn) break;
                        c1 = c2;
                    }
                    T mc = 0, mf = 0;
                    if constexpr (F32C) {
                        const T invj = uniform((float)(1.0 / (double)j));
                        auto emit = [&](int r, T (&y)[PX]) {
#pragma unroll
                            for (int q = 0; q < PX; ++q) {
                                const T x = y[q] * invj;
                                y[q] = x;
                                const T yy = x + L[r][q];
                                const T t = F[r][q] + yy;
                                L[r][q] = yy - (t - F[r][q]);
                                F[r][q] = t;
                                mc = max_abs(mc, x);
                                mf = max_abs(mf, t);
                            }
                        };
                        apply_inplace<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T>(d, top, bot, coef,
                                                                              lane, nx, emit);
                        mc = wave_max(mc);
                    } else {
                        fj /= (T)j;
                        auto emit = [&](int r, T (&y)[PX]) {
#pragma unroll
                            for (int q = 0; q < PX; ++q) {
                                F[r][q] = fma(y[q], fj, F[r][q]);
                                mc = max_abs(mc, y[q]);
                                mf = max_abs(mf, F[r][q]);
                            }
                        };
                        apply_inplace<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T>(d, top, bot, coef,
                                                                              lane, nx, emit);
                        mc = wave_max(mc) * fj;
                    }
                    mf = wave_max(mf);
                    pr0 = (double)mc;
                    pr1 = (double)mf;
                    ++terms;
                }
#pragma unroll
                for (int r = 0; r < RJ; ++r)
#pragma unroll
                    for (int q = 0; q < PX; ++q) {
                        if constexpr (F32C) {
                            const double u = es * ((double)F[r][q] + (double)L[r][q]);
                            F[r][q] = (float)u;
                            L[r][q] = (float)(u - (double)F[r][q]);
                        } else {
                            F[r][q] *= es;
                        }
                    }
            }
            if (a.stats && g == 0 && threadIdx.x == 0) {
                a.stats[((size_t)p * a.K + k) * 2] = terms;
                a.stats[((size_t)p * a.K + k) * 2 + 1] = s;
            }
        }
        // write this slab, combine the non-finite flags of the group
        bool bad = false;
        double* dst = a.uT + (size_t)p * N;
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const int i = lane * PX + q;
                if (r < nrows && i < nx) {
                    const double u = F32C ? (double)F[r][q] + (double)L[r][q] : (double)F[r][q];
                    dst[(size_t)(row0 + r) * nx + i] = u;
                    bad |= !isfinite(u);
                }
            }
        const int any_bad = __syncthreads_or(bad ? 1 : 0);
        double got[2] = {0.0, 0.0};
        if (!aborted) {
            publish_pair(any_bad ? 1.0 : 0.0, 0.0);
            wait_stores();
            __syncthreads();
            group_sync();
            if (!aborted) read_pairs(got);
        }
        if (a.flags && g == 0 && threadIdx.x == 0) {
            int f = pflag | (got[0] != 0.0 ? MG_FLAG_NONFINITE : 0);
            if (aborted) f |= MG_FLAG_ABORT;
            a.flags[p] = f;
        }
    }
    if (aborted && a.flags && threadIdx.x == 0) {
        // mark every path this group had not finished
        for (int64_t p = grp; p < a.P; p += a.ngroups) atomicOr(&a.flags[p], MG_FLAG_ABORT);
    }
}

__global__ void coop_reset_kernel(int* fl, int n, int* abort_word) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) fl[i] = 0;
    if (i == 0) *abort_word = 0;
}

// ---- planning and dispatch ---------------------------------------------------
struct CoopShape {
    int PX, RJ, NW;
};

bool pick_coop_shape(int nx, CoopShape& sh) {
    sh.NW = 8;
    if (nx <= 128) return false;
    if (nx <= 256) { sh.PX = 4; sh.RJ = 8; return true; }
    if (nx <= 512) { sh.PX = 8; sh.RJ = 4; return true; }
    if (nx <= 1024) { sh.PX = 16; sh.RJ = 2; return true; }
    return false;
}

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, bool F32C>
hipError_t coop_kernel_info(const void** fn, size_t* lds) {
    using T = typename std::conditional<F32C, float, double>::type;
    constexpr int RH = Bands<R0, R1, R2>::RH > 0 ? Bands<R0, R1, R2>::RH : 1;
    *fn = (const void*)expmv_coop_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX, F32C>;
    *lds = coop_lds_bytes<PX, NW, RH, T>();
    return hipSuccess;
}

#define MG_COOP_SHAPES(PX, RJ, FULLX, F32C, CALL)                                              \
    if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, 8, 1, 0, 0, 1, FULLX, F32C); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, 8, 2, 1, 0, 1, FULLX, F32C); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 1 && qmax == 2) return CALL(PX, RJ, 8, 2, 1, 1, 2, FULLX, F32C); \
    return hipErrorInvalidValue;

#define MG_COOP_DISPATCH(CALL)                                                                 \
    {                                                                                          \
        const bool full = (ops->grid.nx == 64 * sh.PX);                                        \
        const bool f32 = precision == MG_FP32C;                                                \
        if (sh.PX == 4) {                                                                      \
            if (full) { if (f32) { MG_COOP_SHAPES(4, 8, true, true, CALL) } else { MG_COOP_SHAPES(4, 8, true, false, CALL) } } \
            else { if (f32) { MG_COOP_SHAPES(4, 8, false, true, CALL) } else { MG_COOP_SHAPES(4, 8, false, false, CALL) } } \
        }                                                                                      \
        if (sh.PX == 8) {                                                                      \
            if (full) { if (f32) { MG_COOP_SHAPES(8, 4, true, true, CALL) } else { MG_COOP_SHAPES(8, 4, true, false, CALL) } } \
            else { if (f32) { MG_COOP_SHAPES(8, 4, false, true, CALL) } else { MG_COOP_SHAPES(8, 4, false, false, CALL) } } \
        }                                                                                      \
        if (sh.PX == 16 && f32) {                                                              \
            if (full) { MG_COOP_SHAPES(16, 2, true, true, CALL) } else { MG_COOP_SHAPES(16, 2, false, true, CALL) } \
        }                                                                                      \
        return hipErrorInvalidValue;                                                           \
    }

hipError_t coop_info(const mg_ops* ops, int precision, const void** fn, size_t* lds) {
    CoopShape sh;
    if (!pick_coop_shape(ops->grid.nx, sh)) return hipErrorInvalidValue;
    const int* R = ops->R;
    const int qmax = ops->qmax;
#define MG_CALL_INFO(PX, RJ, NW, R0, R1, R2, QM, FX, F32) \
    coop_kernel_info<PX, RJ, NW, R0, R1, R2, QM, FX, F32>(fn, lds)
    MG_COOP_DISPATCH(MG_CALL_INFO)
#undef MG_CALL_INFO
}

}  // namespace

int coop_rows_per_group_member(int nx) {
    CoopShape sh;
    return pick_coop_shape(nx, sh) ? sh.NW * sh.RJ : 0;
}

// Plan: members per path (G), number of resident groups, exchange-area bytes.
hipError_t coop_plan(const mg_ops* ops, int precision, int64_t P, CoopPlan* plan) {
    CoopShape sh;
    plan->stage = 1;
    if (!pick_coop_shape(ops->grid.nx, sh)) return hipErrorInvalidValue;
    const int RW = sh.NW * sh.RJ;
    const int G = (ops->grid.nv + RW - 1) / RW;
    plan->G = G;
    plan->stage = 2;
    if (G < 1 || G > 64) return hipErrorInvalidValue;
    const void* fn = nullptr;
    size_t lds = 0;
    plan->stage = 3;
    hipError_t e = coop_info(ops, precision, &fn, &lds);
    if (e != hipSuccess) return e;
    plan->lds = lds;
    int dev = 0, cus = 0, per_cu = 0;
    plan->stage = 4;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    plan->cus = cus;
    plan->stage = 5;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * sh.NW, lds)) != hipSuccess)
        return e;
    plan->per_cu = per_cu;
    plan->stage = 6;
    const int resident = per_cu * cus;
    int ngroups = resident / G;
    if (ngroups < 1) return hipErrorInvalidValue;
    int xcd_map = 0;
    if (ngroups >= 8) {
        ngroups = (ngroups / 8) * 8;
        xcd_map = 1;
    }
    if ((int64_t)ngroups > P) {
        ngroups = (int)std::max<int64_t>(P, 1);
        xcd_map = 0;
        if (ngroups >= 8 && ngroups % 8 == 0) xcd_map = 1;
    }
    const size_t elem = precision == MG_FP32C ? 4 : 8;
    plan->G = G;
    plan->ngroups = ngroups;
    plan->xcd_map = xcd_map;
    plan->lds = lds;
    plan->threads = 64 * sh.NW;
    plan->xh_bytes = ((size_t)ngroups * G * 2 * 2 * kRHX * ops->grid.nx * elem + 255) & ~(size_t)255;
    plan->xn_bytes = ((size_t)ngroups * G * 2 * sh.NW * 2 * sizeof(double) + 255) & ~(size_t)255;
    plan->fl_bytes = ((size_t)ngroups * G * sizeof(int) + 256 + 255) & ~(size_t)255;
    plan->bytes = plan->xh_bytes + plan->xn_bytes + plan->fl_bytes;
    return hipSuccess;
}

hipError_t launch_expmv_coop(const mg_ops* ops, const char* tables, size_t tbytes, int64_t P,
                             int K, const double* u0, int u0_broadcast, double* uT, double tol,
                             int precision, int32_t* stats, int32_t* flags, char* xarea,
                             const CoopPlan& plan, hipStream_t s) {
    const void* fn = nullptr;
    size_t lds = 0;
    // this kernel reads tables without x-dependent factors
    if (ops->ND != 0) return hipErrorInvalidValue;
    hipError_t e = coop_info(ops, precision, &fn, &lds);
    if (e != hipSuccess) return e;
    CoopArgs a;
    a.tables = tables;
    a.tbytes = tbytes;
    a.K = K;
    a.nx = ops->grid.nx;
    a.nv = ops->grid.nv;
    a.P = P;
    a.u0 = u0;
    a.u0_bcast = u0_broadcast;
    a.uT = uT;
    a.tol = tol;
    a.stats = stats;
    a.flags = flags;
    a.xh = xarea;
    a.xn = reinterpret_cast<double*>(xarea + plan.xh_bytes);
    a.fl = reinterpret_cast<int*>(xarea + plan.xh_bytes + plan.xn_bytes);
    a.abort_word = a.fl + (size_t)plan.ngroups * plan.G;
    a.G = plan.G;
    a.ngroups = plan.ngroups;
    a.xcd_map = plan.xcd_map;
    const int nfl = plan.ngroups * plan.G;
    hipLaunchKernelGGL(coop_reset_kernel, dim3((nfl + 255) / 256), dim3(256), 0, s, a.fl, nfl,
                       a.abort_word);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(fn, dim3((unsigned)(plan.ngroups * plan.G)),
                                   dim3(plan.threads), args, (unsigned)lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}
