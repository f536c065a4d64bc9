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
// The overlapped form (template flag OVL) synchronises per wave instead: each
// wave has its own counter, bumps it once its stores of the term have
// completed, polls all counters of its group and loads the halo rows and
// norms while it computes the rows that read none of them (rows in the
// segmented order of apply_inplace), and takes the stop decision after the
// term; one workgroup barrier per term guards the LDS halo.  The arithmetic
// per point and the decisions are those of the two-barrier form.
//
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

// The per-(path, step) tables are written by the assembly launch and only
// read here: reading them through the constant address space lets the
// compiler use scalar loads (through the scalar cache) for these wave-uniform
// addresses, although the kernel stores to other global memory.
template <class T>
using ConstMem = __attribute__((address_space(4))) const T;
template <class T>
__device__ inline ConstMem<T>* as_const_mem(const T* p) {
    return (ConstMem<T>*)p;
}

// Exchange area of a cooperative launch (in the caller's workspace, zeroed
// before the launch) and the group layout.
struct XArea {
    char* xh;          // halo rows   [ngroups][G][2 parity][2 side][RHX][64*PX] of T
                       // (point q of lane l at q*64 + l: each store or load
                       // instruction of a wave covers 64 consecutive values)
    double* xn;        // norms       [ngroups][G][2 parity][NW waves][2]
    int* fl;           // counters    [ngroups][G]
    int* abort_word;
    int G;             // workgroups per path
    int ngroups;
    int xcd_map;       // members of a group on one XCD (blockIdx mod 8)
};

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
    const double* xdiag;   // x vectors of the x-dependent factors [ND][nx]
    const double* xchain;  // x-term vectors [nxv][nx]
    const int4* xdesc;     // x-term descriptors [nxt] {depth, outer, middle, inner}
    int nxt, nxv;          // x-terms and their vectors (0: none)
    int nv_pad;            // table rows before the x-term section
    XArea x;
};

struct EulerCoopArgs {
    const double* basis;   // operator tables (B is basis matrix 0, A matrix 1)
    int nx, nv, nv_pad;
    int64_t P;
    double* u;             // [P][nv][nx], updated in place
    const double* dWE;     // [P][NE]
    int NE;
    double dt;
    int32_t* flags;
    const double* xdiag;
    const double* xchain;  // x-term vectors [nxv][nx] (B or A with x-terms)
    const int4* xdesc;     // x-term descriptors [nxt]
    int nxt, nxv;          // x-terms and their vectors (0: none)
    XArea x;
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

// LDS halo between the waves of a cooperative workgroup, double buffered by
// term parity: wave w writes its first RH rows to [par][w][0..RH) and its last
// RH rows to [par][w][RH..2RH).
template <int PX, int RJ, int NW, int RH, class T>
struct HaloX {
    T* base;
    __device__ T* slot(int par, int w, int s) const {
        return base + (((size_t)par * NW + w) * (2 * RH) + s) * (64 * PX);
    }
    __device__ void publish(int par, int w, int lane, const T (&d)[RJ][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                slot(par, w, s)[lane * PX + q] = d[s][q];
                slot(par, w, RH + s)[lane * PX + q] = d[RJ - RH + s][q];
            }
    }
    // rows -RH..-1 from wave w-1 (w > 0)
    __device__ void fetch_top(int par, int w, int lane, T (&top)[RH][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) top[s][q] = slot(par, w - 1, RH + s)[lane * PX + q];
    }
    // rows RJ..RJ+RH-1 from wave w+1 (w < NW-1)
    __device__ void fetch_bot(int par, int w, int lane, T (&bot)[RH][PX]) const {
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) bot[s][q] = slot(par, w + 1, s)[lane * PX + q];
    }
};

// One workgroup's view of its group: slab index g, group index grp, the
// exchange through the workspace and the count of group synchronisations.
// Per synchronisation: every wave publishes (publish_edges, publish_pair) and
// waits for its stores, the workgroup passes a barrier, then sync() bumps this
// member's counter and waits for the others; load_edges and read_pairs read
// what the neighbours published, and next() closes the synchronisation.
template <int PX, int RJ, int NW, int RH, class T>
struct CoopGroup {
    XArea x;
    int lane, w, nx, g, grp;
    int* sh;              // LDS word: abort seen by wave 0
    int counter = 0;      // group syncs done by this launch
    bool aborted = false;

    __device__ __forceinline__ CoopGroup(const XArea& xa, int nx_, int* sh_) : x(xa), nx(nx_), sh(sh_) {
        lane = threadIdx.x & 63;
        w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int b = blockIdx.x;
        if (x.xcd_map) {
            const int xcd = b & 7, k = b >> 3;
            g = k % x.G;
            grp = (k / x.G) * 8 + xcd;
        } else {
            g = b % x.G;
            grp = b / x.G;
        }
        // this group's slices of the exchange area (offsets within them fit
        // 32 bits: G <= 128 members)
        xh_g = reinterpret_cast<T*>(x.xh) + (size_t)grp * x.G * 2 * 2 * kRHX * (64 * PX);
        xn_g = x.xn + (size_t)grp * x.G * 2 * NW * 2;
    }
    T* xh_g;
    double* xn_g;
    __device__ __forceinline__ T* xh_row(int member, int par, int side, int s) const {
        return xh_g + (size_t)(unsigned)((((member * 2 + par) * 2 + side) * kRHX + s) * (64 * PX));
    }
    // this lane's first point in that row (its point q is q*64 further)
    __device__ __forceinline__ T* xh_lane(int member, int par, int side, int s) const {
        return xh_row(member, par, side, s) + (unsigned)lane;
    }
    // per member and parity: NW pairs (one per wave) of norms
    __device__ __forceinline__ double* xn_at(int member, int par, int wave) const {
        return xn_g + ((member * 2 + par) * NW + wave) * 2;
    }
    // edge rows of d for the neighbouring slabs (parity of the coming sync)
    __device__ __forceinline__ void publish_edges(const T (&d)[RJ][PX]) const {
        const int par = counter & 1;
        if (w == 0 && g > 0) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    if (i < nx) xstore(xh_lane(g, par, 0, s) + q * 64, d[s][q]);
                }
        }
        if (w == NW - 1 && g + 1 < x.G) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    if (i < nx) xstore(xh_lane(g, par, 1, s) + q * 64, d[RJ - RH + s][q]);
                }
        }
    }
    // this wave's pair of norms for the coming sync
    __device__ __forceinline__ void publish_pair(double v0, double v1) const {
        if (lane == 0) {
            double* p = xn_at(g, counter & 1, w);
            xstore(p, v0);
            xstore(p + 1, v1);
        }
    }
    // wave 0 bumps the counter and waits (bounded) for every member
    __device__ __forceinline__ void sync() {
        if (w == 0) {
            if (lane == 0) xstore(x.fl + (size_t)grp * x.G + g, counter + 1);
            const int* cnt = x.fl + (size_t)grp * x.G;
            int spins = 0;
            bool ab = false;
            for (;;) {
                bool ready = true;
                for (int mm = lane; mm < x.G; mm += 64)
                    if (xload(cnt + mm) < counter + 1) ready = false;
                if (__all(ready)) break;
                if (++spins > kSpinLimit || xload(x.abort_word)) {
                    ab = true;
                    if (lane == 0) xstore(x.abort_word, 1);
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
    }
    // the neighbours' edge rows into the outer halo rows of the edge waves
    // (the bottom rows are written through selects: two alike branches would
    // be merged into stores through a pointer, which moves the arrays to
    // scratch memory)
    __device__ __forceinline__ void load_edges(T (&top)[RH][PX], T (&bot)[RH][PX]) const {
        const int par = counter & 1;
        if (w == 0) {
#pragma unroll
            for (int s = 0; s < RH; ++s)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    T v = T(0);
                    if (g > 0 && i < nx) v = xload(xh_lane(g - 1, par, 1, s) + q * 64);
                    top[s][q] = v;
                }
        }
        const bool last = w == NW - 1;
#pragma unroll
        for (int s = 0; s < RH; ++s)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const int i = lane * PX + q;
                T v = T(0);
                if (last && g + 1 < x.G && i < nx) v = xload(xh_lane(g + 1, par, 0, s) + q * 64);
                bot[s][q] = last ? v : bot[s][q];
            }
    }
    // maxima over every wave of every member of the pairs of this sync
    __device__ __forceinline__ void read_pairs(double (&out)[2]) const {
        const int par = counter & 1;
        double o0 = 0.0, o1 = 0.0;
        for (int idx = lane; idx < x.G * NW; idx += 64) {
            const double* p = xn_at(idx / NW, par, idx % NW);
            o0 = fmax(o0, xload(p));
            o1 = fmax(o1, xload(p + 1));
        }
        for (int o = 32; o > 0; o >>= 1) {
            o0 = fmax(o0, __shfl_xor(o0, o, 64));
            o1 = fmax(o1, __shfl_xor(o1, o, 64));
        }
        out[0] = uniform(o0);
        out[1] = uniform(o1);
    }
    __device__ __forceinline__ void next() { ++counter; }

    // Overlapped exchange (expmv_coop_kernel with OVL): one counter per wave,
    // [ngroups][G][NW] after the group's member counters are unused.  A wave
    // bumps its counter once its own stores of the sync have completed, and
    // every wave polls all counters of its group itself, so neither needs a
    // workgroup barrier.
    __device__ __forceinline__ void bump_wave() const {
        if (lane == 0) xstore(x.fl + ((size_t)grp * x.G + g) * NW + w, counter + 1);
    }
    // false: the launch was aborted (spin limit here or elsewhere)
    __device__ __forceinline__ bool poll_waves() const {
        const int* cnt = x.fl + (size_t)grp * x.G * NW;
        const int n = x.G * NW;
        for (int spins = 0;; ++spins) {
            bool ready = true;
            for (int mm = lane; mm < n; mm += 64)
                if (xload(cnt + mm) < counter + 1) ready = false;
            if (__all(ready)) return true;
            if (spins > kSpinLimit || xload(x.abort_word)) {
                if (lane == 0) xstore(x.abort_word, 1);
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    // end of a path, overlapped form: every wave publishes its flag with its
    // pair, no workgroup barrier
    __device__ __forceinline__ bool any_member_waves(bool mine) {
        if (aborted) return false;
        publish_pair(__any(mine) ? 1.0 : 0.0, 0.0);
        wait_stores();
        bump_wave();
        if (!poll_waves()) {
            if (lane == 0) sh[0] = 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            aborted = true;
            return false;
        }
        double got[2];
        read_pairs(got);
        next();
        return got[0] != 0.0;
    }
    // end of a path: combine a per-workgroup flag over the group (nonzero if
    // any member set it)
    __device__ __forceinline__ bool any_member(bool mine) {
        const int any = __syncthreads_or(mine ? 1 : 0);
        if (aborted) return false;
        publish_pair(any ? 1.0 : 0.0, 0.0);
        wait_stores();
        __syncthreads();
        sync();
        if (aborted) return false;
        double got[2];
        read_pairs(got);
        next();
        return got[0] != 0.0;
    }
};

// x vectors of the x-dependent factors: registers in FP32, LDS in FP64 (the
// FP64 state, halo and factors together exceed the register file)
template <int ND, class T>
constexpr bool xa_in_lds() {
    return ND > 0 && sizeof(T) == 8;
}

// LDS: halo | abort word (16 bytes) | x vectors [ND][64*PX] (when in LDS) |
// x-term vectors [nxv][64*PX] (their count is known at launch only: the
// launch adds them)
// (the overlapped form keeps two halo buffers, alternating per term)
template <int PX, int NW, int RH, int ND, class T, bool OVL = false>
constexpr size_t coop_halo_elems() {
    return (size_t)(OVL ? 2 : 1) * NW * 2 * RH * 64 * PX;
}
template <int PX, int NW, int RH, int ND, class T, bool OVL = false>
constexpr size_t coop_lds_bytes() {
    return coop_halo_elems<PX, NW, RH, ND, T, OVL>() * sizeof(T) + 16 +
           (xa_in_lds<ND, T>() ? (size_t)ND * 64 * PX * sizeof(T) : 0);
}

// The x vectors at this lane's points (zero beyond nx), in registers or in LDS
// (written by wave 0; the caller passes a barrier before the first use).
template <int PX, int ND, bool LDS, class T>
struct XVec;
template <int PX, int ND, class T>
struct XVec<PX, ND, false, T> {
    static constexpr int NDX = ND > 0 ? ND : 1;
    T v[NDX][PX];
    __device__ __forceinline__ XVec(const double* xdiag, T*, int lane, int nx) {
#pragma unroll
        for (int t = 0; t < NDX; ++t)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const int i = lane * PX + q;
                v[t][q] = (ND > 0 && i < nx) ? (T)xdiag[(size_t)t * nx + i] : T(0);
            }
    }
    __device__ __forceinline__ T operator()(int t, int q) const { return v[t][q]; }
};
template <int PX, int ND, class T>
struct XVec<PX, ND, true, T> {
    const T* xs;
    int lane;
    __device__ __forceinline__ XVec(const double* xdiag, T* lds, int lane_, int nx)
        : xs(lds), lane(lane_) {
        if (threadIdx.x < 64) {
            for (int t = 0; t < ND; ++t)
#pragma unroll
                for (int q = 0; q < PX; ++q) {
                    const int i = lane * PX + q;
                    lds[t * 64 * PX + lane * PX + q] = i < nx ? (T)xdiag[(size_t)t * nx + i] : T(0);
                }
        }
    }
    __device__ __forceinline__ T operator()(int t, int q) const {
        return xs[t * 64 * PX + lane * PX + q];
    }
};

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, bool F32C, int ND,
          int NC, bool OVL>
__global__ __launch_bounds__(64 * NW) void expmv_coop_kernel(CoopArgs a) {
    using T = typename std::conditional<F32C, float, double>::type;
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, ND>();
    // x-term coefficients per row (NC > 0: the operator has x-terms)
    const int ncb = NC > 0 ? a.nxt * (2 * MG_XDIAG_RADIUS + 1) : 0;
    constexpr int RW = NW * RJ;
    constexpr size_t HE = coop_halo_elems<PX, NW, RH, ND, T, OVL>();
    extern __shared__ double lds_d[];
    T* lds = reinterpret_cast<T*>(lds_d);
    HaloC<PX, RJ, NW, RH, T> halo{lds};
    HaloX<PX, RJ, NW, RH, T> halo2{lds};
    int* sh = reinterpret_cast<int*>(lds + HE);
    CoopGroup<PX, RJ, NW, RH, T> cg(a.x, a.nx, sh);
    const int lane = cg.lane, w = cg.w, g = cg.g, grp = cg.grp;
    const int nx = a.nx, nv = a.nv;
    const size_t N = (size_t)nx * nv;
    const int row0 = g * RW + w * RJ;                 // first global row of this wave
    const int nrows = min(RJ, max(0, nv - row0));
    if (threadIdx.x == 0) sh[0] = 0;
    // the x vectors of the x-dependent factors at this lane's points
    T* xl = lds + HE + 16 / sizeof(T);
    const XVec<PX, ND, xa_in_lds<ND, T>(), T> xa(a.xdiag, xl, lane, nx);
    // x-term vectors [nxv][64*PX] in LDS after the x vectors
    T* cvl = xl + (xa_in_lds<ND, T>() ? (size_t)ND * 64 * PX : 0);
    if constexpr (NC > 0) {
        for (int idx = threadIdx.x; idx < a.nxv * 64 * PX; idx += 64 * NW) {
            const int v = idx / (64 * PX), i = idx % (64 * PX);
            cvl[idx] = i < nx ? (T)a.xchain[(size_t)v * nx + i] : T(0);
        }
    }
    const XTerms<PX, T> cvec{a.nxt, a.xdesc, cvl, lane};
    __syncthreads();

    // one application of the operator to this wave's rows, in place (for
    // the overlapped exchange in the segmented order, with a hook)
    auto apply_dir = [&](auto seg, T (&d)[RJ][PX], const T (&top)[RH][PX],
                         const T (&bot)[RH][PX], auto coef, auto ccoef, auto emit, auto hook) {
        constexpr bool SEG = decltype(seg)::value;
        if constexpr (ND == 0)
            apply_inplace<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T, decltype(coef), decltype(emit),
                          SEG, decltype(hook)>(d, top, bot, coef, lane, nx, emit, hook);
        else if constexpr (NC == 0)
            apply_inplace_x<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, MG_XDIAG_RADIUS, T,
                            decltype(coef), decltype(xa), decltype(emit), 0, NoChains, NoChains,
                            SEG, decltype(hook)>(d, top, bot, coef, xa, lane, nx, emit,
                                                 NoChains{}, NoChains{}, hook);
        else
            apply_inplace_x<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, MG_XDIAG_RADIUS, T,
                            decltype(coef), decltype(xa), decltype(emit), NC, decltype(ccoef),
                            decltype(cvec), SEG, decltype(hook)>(d, top, bot, coef, xa, lane, nx,
                                                                 emit, ccoef, cvec, hook);
    };
    auto apply_term = [&](T (&d)[RJ][PX], const T (&top)[RH][PX], const T (&bot)[RH][PX],
                          auto coef, auto ccoef, auto emit) {
        apply_dir(std::false_type{}, d, top, bot, coef, ccoef, emit, NoHook{});
    };
    // overlapped exchange: in the segmented order no halo row is read before
    // step RJ - 2RH; the wave bumps its counter before step IB and polls the
    // group before step IP = RJ - 2RH, then loads the halo rows (LDS and the
    // neighbours') and the norms.  Polling as late as that keeps the loaded
    // rows out of the registers while the other rows are computed (an earlier
    // poll made the 8-row waves spill: 1527 against 1426 ms on the 256^2
    // workload); bumping early, after one row (a quarter of the rows before
    // the poll for the 16-row waves), gives the group's bumps the most time
    // to arrive while leaving the publishing stores a row to complete (8-row
    // waves: 1351 / 1309 / 1432 / 1584 ms with the bump before row 0 / 1 / 2 / 3).
    constexpr int IP = RJ - 2 * RH;
    constexpr int IB = IP >= 8 ? IP / 4 : (IP > 1 ? 1 : 0);
    static_assert(!OVL || (RJ > 2 * RH && IP <= RJ - 2 * RH), "overlapped exchange needs RJ > 2 RH");
    int hb = 0;   // LDS halo buffer of the overlapped form (alternates per term)

    for (int64_t p = grp; p < a.P && !cg.aborted; p += a.x.ngroups) {
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
        for (int k = 0; k < a.K && !cg.aborted; ++k) {
            const TableView tv{a.tables + ((size_t)p * a.K + k) * a.tbytes};
            const int s = tv.s();
            const int m = tv.m();
            const double es = tv.es();
            pflag |= tv.flag();
            const ConstMem<T>* rows = as_const_mem(tv.rows<T>() + (size_t)row0 * NBP);
            auto coef = [&](int r, int e) -> T { return rows[r * NBP + e]; };
            // x-term section of the table (after the nv_pad main rows)
            const ConstMem<T>* crows =
                as_const_mem(tv.rows<T>() + (size_t)a.nv_pad * NBP + (size_t)row0 * ncb);
            auto ccoef = [&](int r, int e) -> T { return crows[r * ncb + e]; };
            int terms = 0;
            for (int sub = 0; sub < s && !cg.aborted; ++sub) {
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
                if constexpr (OVL) {
                    for (int j = 1; j <= m; ++j) {
                        // publish c_{j-1} (LDS halo, edge rows, norms)
                        halo2.publish(hb, w, lane, d);
                        cg.publish_edges(d);
                        cg.publish_pair(pr0, pr1);
                        __syncthreads();
                        if (sh[0]) {
                            cg.aborted = true;
                            break;
                        }
                        T top[RH][PX], bot[RH][PX];
                        const int buf = hb;
                        hb ^= 1;
                        double got[2] = {0.0, 0.0};
                        auto hook = [&](int i) {
                            if (i == IB) {
                                wait_stores();
                                cg.bump_wave();
                            }
                            if (i == IP) {
                                if (w > 0) halo2.fetch_top(buf, w, lane, top);
                                if (w + 1 < NW) halo2.fetch_bot(buf, w, lane, bot);
                                if (cg.poll_waves()) {
                                    cg.load_edges(top, bot);
                                    cg.read_pairs(got);
                                } else {
#pragma unroll
                                    for (int s2 = 0; s2 < RH; ++s2)
#pragma unroll
                                        for (int q = 0; q < PX; ++q) top[s2][q] = bot[s2][q] = T(0);
                                    if (lane == 0) sh[0] = 1;
                                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                                    cg.aborted = true;
                                }
                                cg.next();
                            }
                        };
                        // c_j = Y c_{j-1} in place (not yet scaled or summed)
                        auto raw = [](int, T (&)[PX]) {};
                        apply_dir(std::true_type{}, d, top, bot, coef, ccoef, raw, hook);
                        if (cg.aborted) break;
                        // the stop rule on the norms of c_{j-1} and F_{j-1}, as
                        // below: a stop discards c_j
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
                            const T invj_lo = uniform((float)(1.0 / (double)j - (double)invj));
#pragma unroll
                            for (int r = 0; r < RJ; ++r)
#pragma unroll
                                for (int q = 0; q < PX; ++q) {
                                    const T x = fma(d[r][q], invj, d[r][q] * invj_lo);
                                    d[r][q] = x;
                                    const T yy = x + L[r][q];
                                    const T t = F[r][q] + yy;
                                    L[r][q] = yy - (t - F[r][q]);
                                    F[r][q] = t;
                                    mc = max_abs(mc, x);
                                    mf = max_abs(mf, t);
                                }
                            mc = wave_max(mc);
                        } else {
                            fj /= (T)j;
#pragma unroll
                            for (int r = 0; r < RJ; ++r)
#pragma unroll
                                for (int q = 0; q < PX; ++q) {
                                    F[r][q] = fma(d[r][q], fj, F[r][q]);
                                    mc = max_abs(mc, d[r][q]);
                                    mf = max_abs(mf, F[r][q]);
                                }
                            mc = wave_max(mc) * fj;
                        }
                        mf = wave_max(mf);
                        pr0 = (double)mc;
                        pr1 = (double)mf;
                        ++terms;
                    }
                } else
                for (int j = 1; j <= m; ++j) {
                    halo.publish(w, lane, d);
                    cg.publish_edges(d);
                    cg.publish_pair(pr0, pr1);
                    wait_stores();
                    __syncthreads();
                    // LDS halo read between the two barriers (the next term
                    // writes it after the second)
                    T top[RH][PX], bot[RH][PX];
                    halo.fetch(w, lane, top, bot);
                    cg.sync();
                    if (cg.aborted) break;
                    // neighbours' halo rows and the pairs, loaded together
                    cg.load_edges(top, bot);
                    double got[2];
                    cg.read_pairs(got);
                    cg.next();
                    if (j == 1) {
                        c1 = got[0];
                    } else {
                        const double c2 = got[0], fn = got[1];
                        if (c1 + c2 <= a.tol * fn) break;
                        c1 = c2;
                    }
                    T mc = 0, mf = 0;
                    if constexpr (F32C) {
                        // 1/j as a float and its residual (unbiased scaling
                        // of the term, as in the register-resident kernel)
                        const T invj = uniform((float)(1.0 / (double)j));
                        const T invj_lo = uniform((float)(1.0 / (double)j - (double)invj));
                        auto emit = [&](int r, T (&y)[PX]) {
#pragma unroll
                            for (int q = 0; q < PX; ++q) {
                                const T x = fma(y[q], invj, y[q] * invj_lo);
                                y[q] = x;
                                const T yy = x + L[r][q];
                                const T t = F[r][q] + yy;
                                L[r][q] = yy - (t - F[r][q]);
                                F[r][q] = t;
                                mc = max_abs(mc, x);
                                mf = max_abs(mf, t);
                            }
                        };
                        apply_term(d, top, bot, coef, ccoef, emit);
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
                        apply_term(d, top, bot, coef, ccoef, emit);
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
        const bool any_bad = OVL ? cg.any_member_waves(bad) : cg.any_member(bad);
        if (a.flags && g == 0 && threadIdx.x == 0) {
            int f = pflag | (any_bad ? MG_FLAG_NONFINITE : 0);
            if (cg.aborted) f |= MG_FLAG_ABORT;
            a.flags[p] = f;
        }
    }
    if constexpr (OVL) {
        // a wave that gave up marks the word; the others learn of it here
        __syncthreads();
        if (sh[0]) cg.aborted = true;
    }
    if (cg.aborted && a.flags && threadIdx.x == 0) {
        // mark every path this group had not finished
        for (int64_t p = grp; p < a.P; p += a.x.ngroups) atomicOr(&a.flags[p], MG_FLAG_ABORT);
    }
}

// ---- difference-first form (FP32) ---------------------------------------------
//
// The kernel above applies the operator in place, requests a row's band
// coefficients one row ahead and reads the halo rows before the first row it
// computes.  The form below runs the term loop of the register-resident
// kernel inside the cooperative group: the term alternates between two
// register arrays, each row's x differences are formed once and every output
// point is one FMA chain over the bands (apply_split), rows are produced
// interior first so that the halo rows arrive while interior rows are
// computed, and the workgroup's coefficient rows of a Magnus step are staged
// in LDS once and read one row ahead.  Per term the group synchronises as
// above: the edge waves' outer halo rows come from the neighbouring members,
// the inner ones from LDS.  Built for the compensated FP32 form on grids up
// to 256 points wide (13 % faster than the in-place kernel on the 256^2,
// 4096-path order-3 workload): in FP64 the two term arrays, the partial sum
// and the difference windows of four points per lane need more than the 256
// registers of a wave in an 8-wave workgroup.

// LDS of the difference-first kernel: halo [2][NW][2RH] rows | abort word (16
// bytes) | FP32 form: the workgroup's coefficient rows of the current step
template <int PX, int NW, int RH, class T>
constexpr size_t split_halo_bytes() {
    return (size_t)2 * NW * 2 * RH * 64 * PX * sizeof(T);
}
template <int PX, int RJ, int NW, int RH, int NBP, class T>
constexpr size_t split_lds_bytes() {
    return split_halo_bytes<PX, NW, RH, T>() + 16 +
           (sizeof(T) == 4 ? (size_t)NW * RJ * NBP * sizeof(T) : 0);
}

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX>
__global__ __launch_bounds__(64 * NW) void expmv_coop_split_kernel(CoopArgs a) {
    using T = float;
    constexpr int RH = halo_rows<R0, R1, R2, 0>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, 0>();
    constexpr int RW = NW * RJ;
    extern __shared__ double lds_d[];
    HaloX<PX, RJ, NW, RH, T> halo{reinterpret_cast<T*>(lds_d)};
    char* tail = reinterpret_cast<char*>(lds_d) + split_halo_bytes<PX, NW, RH, T>();
    CoopGroup<PX, RJ, NW, RH, T> cg(a.x, a.nx, reinterpret_cast<int*>(tail));
    T* ctab = reinterpret_cast<T*>(tail + 16);     // this step's coefficient rows
    const int lane = cg.lane, w = cg.w, g = cg.g, grp = cg.grp;
    const int nx = a.nx, nv = a.nv;
    const size_t N = (size_t)nx * nv;
    const int row0 = g * RW + w * RJ;                 // first global row of this wave
    const int nrows = min(RJ, max(0, nv - row0));

    for (int64_t p = grp; p < a.P && !cg.aborted; p += a.x.ngroups) {
        // state F = hi + lo
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
                    L[r][q] = (T)(u - (double)F[r][q]);
                }
        }
        int pflag = 0;
        int tpar = 0;
        for (int k = 0; k < a.K && !cg.aborted; ++k) {
            const TableView tv{a.tables + ((size_t)p * a.K + k) * a.tbytes};
            const int s = tv.s();
            const int m = tv.m();
            const double es = tv.es();
            pflag |= tv.flag();
            {
                // the workgroup's rows of this step into LDS (every term reads them)
                constexpr int n16 = RW * NBP * (int)sizeof(T) / 16;
                static_assert(RW * NBP * sizeof(T) % 16 == 0, "row block not in 16-byte units");
                const uint4* src = reinterpret_cast<const uint4*>(tv.rows<T>() + (size_t)g * RW * NBP);
                uint4* dst = reinterpret_cast<uint4*>(ctab);
                __syncthreads();   // the previous step's reads are done
                for (int i = threadIdx.x; i < n16; i += 64 * NW) dst[i] = src[i];
                __syncthreads();
            }
            const LdsRows<T, NBP> coef{(const T*)ctab + (size_t)w * RJ * NBP};
            int terms = 0;
            for (int sub = 0; sub < s && !cg.aborted; ++sub) {
                T A[RJ][PX], B[RJ][PX];
                T sm = 0;
#pragma unroll
                for (int r = 0; r < RJ; ++r)
#pragma unroll
                    for (int q = 0; q < PX; ++q) {
                        A[r][q] = F[r][q];
                        sm = max_abs(sm, F[r][q]);
                    }
                // this wave's pair for the next exchange: the state norm (first
                // term), then the norms of the previous term and partial sum
                double pr0 = (double)wave_max_dpp(sm), pr1 = 0.0;
                double c1 = 0.0;
                // term j from `in` into `out`; false when the series stopped before it
                auto step = [&](T (&in)[RJ][PX], T (&out)[RJ][PX], int j) -> bool {
                    halo.publish(tpar, w, lane, in);
                    cg.publish_edges(in);
                    cg.publish_pair(pr0, pr1);
                    wait_stores();
                    __syncthreads();
                    cg.sync();
                    if (cg.aborted) return false;
                    T top[RH][PX], bot[RH][PX];
                    // the outer halo rows of the edge waves from the neighbours
                    cg.load_edges(top, bot);
                    double got[2];
                    cg.read_pairs(got);
                    cg.next();
                    if (j == 1) {
                        c1 = got[0];
                    } else {
                        const double c2 = got[0], fn = got[1];
                        if (c1 + c2 <= a.tol * fn) return false;
                        c1 = c2;
                    }
                    const int hp = tpar;
                    auto fb = [&] {
                        if (w + 1 < NW) halo.fetch_bot(hp, w, lane, bot);
                    };
                    auto ft = [&] {
                        if (w > 0) halo.fetch_top(hp, w, lane, top);
                    };
                    T mc = 0, mf = 0;
                    // c_j = Y' c_{j-1} / j goes to `out`; F = hi + lo gains c_j (Kahan)
                    // 1/j as a float and its residual: unbiased scaling of the term
                    const T invj = (float)(1.0 / (double)j);
                    const T invj_lo = (float)(1.0 / (double)j - (double)invj);
                    apply_split<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T>(
                        in, out, top, bot, fb, ft, coef, lane, nx, [&](int r, T (&y)[PX]) {
#pragma unroll
                            for (int q = 0; q < PX; ++q) {
                                const T xv = fma(y[q], invj, y[q] * invj_lo);
                                y[q] = xv;
                                const T yy = xv + L[r][q];
                                const T tt = F[r][q] + yy;
                                L[r][q] = yy - (tt - F[r][q]);
                                F[r][q] = tt;
                                mc = max_abs(mc, xv);
                                mf = max_abs(mf, tt);
                            }
                        });
                    mc = wave_max_dpp(mc);
                    pr0 = (double)mc;
                    pr1 = (double)wave_max_dpp(mf);
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
                    for (int q = 0; q < PX; ++q) {
                        const double u = es * ((double)F[r][q] + (double)L[r][q]);
                        F[r][q] = (float)u;
                        L[r][q] = (float)(u - (double)F[r][q]);
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
                    const double u = (double)F[r][q] + (double)L[r][q];
                    dst[(size_t)(row0 + r) * nx + i] = u;
                    bad |= !isfinite(u);
                }
            }
        const bool any_bad = cg.any_member(bad);
        if (a.flags && g == 0 && threadIdx.x == 0) {
            int f = pflag | (any_bad ? MG_FLAG_NONFINITE : 0);
            if (cg.aborted) f |= MG_FLAG_ABORT;
            a.flags[p] = f;
        }
    }
    if (cg.aborted && a.flags && threadIdx.x == 0) {
        for (int64_t p = grp; p < a.P; p += a.x.ngroups) atomicOr(&a.flags[p], MG_FLAG_ABORT);
    }
}

// Euler-Maruyama on the cooperative layout: u <- u + (dt B + dW_n A) u for
// n = 0..NE-1 (FP64), one group synchronisation per step for the halo rows.
template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, int ND, int NC>
__global__ __launch_bounds__(64 * NW) void euler_coop_kernel(EulerCoopArgs a) {
    using T = double;
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, ND>();
    constexpr int RW = NW * RJ;
    extern __shared__ double lds_d[];
    T* lds = lds_d;
    HaloC<PX, RJ, NW, RH, T> halo{lds};
    CoopGroup<PX, RJ, NW, RH, T> cg(a.x, a.nx, reinterpret_cast<int*>(lds + (size_t)NW * 2 * RH * 64 * PX));
    const int lane = cg.lane, w = cg.w, g = cg.g, grp = cg.grp;
    const int nx = a.nx, nv = a.nv;
    const size_t N = (size_t)nx * nv;
    const int row0 = g * RW + w * RJ;
    const int nrows = min(RJ, max(0, nv - row0));
    T* xl = lds + (size_t)NW * 2 * RH * 64 * PX + 16 / sizeof(T);
    const XVec<PX, ND, xa_in_lds<ND, T>(), T> xa(a.xdiag, xl, lane, nx);
    // x-terms of B and A (NC > 0): vectors [nxv][64*PX] after the x vectors,
    // coefficients in the x-term section of basis matrices 0 and 1
    T* cvl = xl + (xa_in_lds<ND, T>() ? (size_t)ND * 64 * PX : 0);
    const int ncb = NC > 0 ? a.nxt * (2 * MG_XDIAG_RADIUS + 1) : 0;
    if constexpr (NC > 0) {
        for (int idx = threadIdx.x; idx < a.nxv * 64 * PX; idx += 64 * NW) {
            const int v = idx / (64 * PX), i = idx % (64 * PX);
            cvl[idx] = i < nx ? a.xchain[(size_t)v * nx + i] : 0.0;
        }
    }
    const XTerms<PX, T> cvec{a.nxt, a.xdesc, cvl, lane};
    __syncthreads();
    // basis matrices 0 (B) and 1 (A), read through the constant address space
    const ConstMem<double>* Brows = as_const_mem(a.basis + (size_t)row0 * NBP);
    const ConstMem<double>* Arows = as_const_mem(a.basis + ((size_t)a.nv_pad + row0) * NBP);
    const ConstMem<double>* Bc =
        as_const_mem(a.basis + (size_t)MG_NBASIS * a.nv_pad * NBP + (size_t)row0 * ncb);
    const ConstMem<double>* Ac = Bc + (size_t)a.nv_pad * ncb;

    for (int64_t p = grp; p < a.P && !cg.aborted; p += a.x.ngroups) {
        double* src = a.u + (size_t)p * N;
        T d[RJ][PX];
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const int i = lane * PX + q;
                d[r][q] = (r < nrows && i < nx) ? src[(size_t)(row0 + r) * nx + i] : 0.0;
            }
        const double* dw = a.dWE + (size_t)p * a.NE;
        for (int n = 0; n < a.NE; ++n) {
            const double wn = dw[n];
            auto coef = [&](int r, int e) -> T {
                // uniform: the combined coefficient lives in scalar registers
                return uniform(fma(a.dt, Brows[r * NBP + e], wn * Arows[r * NBP + e]));
            };
            halo.publish(w, lane, d);
            cg.publish_edges(d);
            wait_stores();
            __syncthreads();
            T top[RH][PX], bot[RH][PX];
            halo.fetch(w, lane, top, bot);
            cg.sync();
            if (cg.aborted) break;
            cg.load_edges(top, bot);
            cg.next();
            // the new row is the old row plus the operator's row (the old row
            // is still in d when it is emitted)
            auto emit = [&](int r, T (&y)[PX]) {
#pragma unroll
                for (int q = 0; q < PX; ++q) y[q] += d[r][q];
            };
            if constexpr (ND == 0) {
                apply_inplace<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, T>(d, top, bot, coef, lane, nx,
                                                                      emit);
            } else if constexpr (NC == 0) {
                apply_inplace_x<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, MG_XDIAG_RADIUS, T>(
                    d, top, bot, coef, xa, lane, nx, emit);
            } else {
                auto ccoef = [&](int r, int e) -> T {
                    return uniform(fma(a.dt, Bc[r * ncb + e], wn * Ac[r * ncb + e]));
                };
                apply_inplace_x<PX, RJ, R0, R1, R2, QMAX, FULLX, RH, ND, MG_XDIAG_RADIUS, T,
                                decltype(coef), decltype(xa), decltype(emit), NC,
                                decltype(ccoef), decltype(cvec)>(d, top, bot, coef, xa, lane, nx,
                                                                 emit, ccoef, cvec);
            }
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
        const bool any_bad = cg.any_member(bad);
        if (a.flags && g == 0 && threadIdx.x == 0) {
            int f = any_bad ? MG_FLAG_NONFINITE : 0;
            if (cg.aborted) f |= MG_FLAG_ABORT;
            a.flags[p] = f;
        }
    }
    if (cg.aborted && a.flags && threadIdx.x == 0) {
        for (int64_t p = grp; p < a.P; p += a.x.ngroups) atomicOr(&a.flags[p], MG_FLAG_ABORT);
    }
}

__global__ void coop_reset_kernel(int* fl, int n, int* abort_word) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) fl[i] = 0;
    if (i == 0) *abort_word = 0;
}

// ---- planning and dispatch ---------------------------------------------------
struct CoopShape {
    int PX;
};

// x points per lane
bool pick_coop_shape(int nx, CoopShape& sh, int precision = MG_FP64) {
    if (nx <= 128) return false;
    if (nx <= 256) { sh.PX = 4; return true; }
    // FP64 between 256 and 384 points: 5 or 6 points per lane instead of 8
    // (less padding, and fewer registers for the x-term form)
    if (precision == MG_FP64 && nx <= 320) { sh.PX = 5; return true; }
    if (precision == MG_FP64 && nx <= 384) { sh.PX = 6; return true; }
    if (nx <= 512) { sh.PX = 8; return true; }
    if (nx <= 1024) { sh.PX = 16; return true; }
    return false;
}

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, bool F32C, int ND,
          int NC = 0, bool OVL = false>
hipError_t coop_kernel_info(const void** fn, size_t* lds, int* nw, int* rows) {
    using T = typename std::conditional<F32C, float, double>::type;
    constexpr int RH = halo_rows<R0, R1, R2, ND>();
    if constexpr ((OVL && RJ <= 2 * RH) || RJ < RH) {
        // the overlapped exchange needs rows that read no halo row; a wave
        // publishes RH of its rows as halo
        return hipErrorInvalidValue;
    } else {
        *nw = NW;
        *rows = NW * RJ;
        *fn = (const void*)expmv_coop_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX, F32C, ND, NC, OVL>;
        *lds = coop_lds_bytes<PX, NW, RH, ND, T, OVL>();
        return hipSuccess;
    }
}

// A cooperative Taylor kernel: entry, LDS, waves and rows per workgroup.
struct KInfo {
    const void* fn = nullptr;
    size_t lds = 0;
    int nw = 0, rows = 0;
};

template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX>
hipError_t split_kernel_info(KInfo* ki) {
    using T = float;
    constexpr int RH = halo_rows<R0, R1, R2, 0>();
    constexpr int NBP = table_stride<R0, R1, R2, QMAX, 0>();
    ki->fn = (const void*)expmv_coop_split_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX>;
    ki->lds = split_lds_bytes<PX, RJ, NW, RH, NBP, T>();
    ki->nw = NW;
    ki->rows = NW * RJ;
    return hipSuccess;
}

#define MG_SPLIT_SHAPES(PX, RJ, NW, FULLX)                                                      \
    if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1)                                      \
        return split_kernel_info<PX, RJ, NW, 1, 0, 0, 1, FULLX>(ki);                           \
    if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1)                                      \
        return split_kernel_info<PX, RJ, NW, 2, 1, 0, 1, FULLX>(ki);                           \
    if (R[0] == 2 && R[1] == 1 && R[2] == 1 && qmax == 2)                                      \
        return split_kernel_info<PX, RJ, NW, 2, 1, 1, 2, FULLX>(ki);                           \
    return hipErrorInvalidValue;

// The difference-first kernel for this operator, if built: the FP32 form on
// grids up to 256 points wide with coefficients that depend on v only.
hipError_t split_info(const mg_ops* ops, int precision, KInfo* ki) {
    CoopShape sh;
    if (precision != MG_FP32C || ops->ND != 0 || !pick_coop_shape(ops->grid.nx, sh, precision) ||
        sh.PX != 4)
        return hipErrorInvalidValue;
    const bool full = ops->grid.nx == 64 * sh.PX;
    const int* R = ops->R;
    const int qmax = ops->qmax;
    if (full) { MG_SPLIT_SHAPES(4, 8, 8, true) }
    else { MG_SPLIT_SHAPES(4, 8, 8, false) }
}
#undef MG_SPLIT_SHAPES

// Kernel shapes without (MG_COOP_SHAPES) and with (MG_COOP_SHAPES_ND)
// x-dependent factors; the latter exist for the order-1 and order-2 bands.
#define MG_COOP_SHAPES(PX, RJ, NW, FULLX, F32C, CALL)                                          \
    if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 1, 0, 0, 1, FULLX, F32C, 0); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, F32C, 0); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 1 && qmax == 2) return CALL(PX, RJ, NW, 2, 1, 1, 2, FULLX, F32C, 0); \
    if (R[0] == 3 && R[1] == 3 && R[2] == 3 && qmax == 2) return CALL(PX, RJ, NW, 3, 3, 3, 2, FULLX, F32C, 0); \
    return hipErrorInvalidValue;
#define MG_COOP_SHAPES_ND(PX, RJ, NW, FULLX, F32C, CALL)                                       \
    if (ops->ND == 3) {                                                                        \
        if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 1, 0, 0, 1, FULLX, F32C, 3); \
        if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, F32C, 3); \
        return hipErrorInvalidValue;                                                           \
    }                                                                                          \
    if (ops->ND != MG_MAX_XDIAG) return hipErrorInvalidValue;                                  \
    if (R[0] == 1 && R[1] == 0 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 1, 0, 0, 1, FULLX, F32C, MG_MAX_XDIAG); \
    if (R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1) return CALL(PX, RJ, NW, 2, 1, 0, 1, FULLX, F32C, MG_MAX_XDIAG); \
    return hipErrorInvalidValue;
#define MG_COOP_FULLX(SHAPES, PX, RJ, NW, F32C, CALL)                                          \
    if (full) { SHAPES(PX, RJ, NW, true, F32C, CALL) } else { SHAPES(PX, RJ, NW, false, F32C, CALL) }

// Workgroup shape per x-width and precision: 8 waves of RJ rows, or, where
// the FP64 state, halo and factors do not fit 256 registers, 4 waves of twice
// the rows (one wave per SIMD, which may use 512 registers; at nx <= 256 the
// FP64 kernel without x-factors also runs 4 waves of 16 rows: it spills none
// of its registers there, against 60 bytes per lane with 8 waves of 8 rows,
// and its 4096-path 256^2 order-3 launch takes 1955 ms against 2000).  At nx > 512
// FP32C runs 4 waves of 6 rows: 24 rows per workgroup, so 43 members hold a
// 1024-row path where 16-row workgroups need 64, and the exchange, which grows
// with the member count, costs less.  FP64 at nx > 512 runs 4 waves of 2 rows
// (8 rows per workgroup, up to 128 members for 1024 rows): sixteen FP64
// points per lane for the state, the term, the pending rows and the halo fit
// 512 registers only with two rows per wave (three rows spill).  The table
// rows are padded to the most rows per workgroup of any shape of the x width
// (coop_rows_max), which every shape's row count divides.  x-dependent factors
// up to nx = 512.
#define MG_COOP_DISPATCH(CALL)                                                                 \
    {                                                                                          \
        const bool full = (ops->grid.nx == 64 * sh.PX);                                        \
        const bool f32 = precision == MG_FP32C;                                                \
        const bool nd = ops->ND > 0;                                                           \
        if (sh.PX == 4) {                                                                      \
            if (f32) {                                                                         \
                if (nd) { MG_COOP_FULLX(MG_COOP_SHAPES_ND, 4, 8, 8, true, CALL) }               \
                else { MG_COOP_FULLX(MG_COOP_SHAPES, 4, 8, 8, true, CALL) }                     \
            } else {                                                                           \
                if (nd) { MG_COOP_FULLX(MG_COOP_SHAPES_ND, 4, 16, 4, false, CALL) }             \
                else if (variant & 1) { MG_COOP_FULLX(MG_COOP_SHAPES, 4, 8, 8, false, CALL) }   \
                else { MG_COOP_FULLX(MG_COOP_SHAPES, 4, 16, 4, false, CALL) }                   \
            }                                                                                  \
        }                                                                                      \
        if (sh.PX == 5 && !f32) {                                                              \
            if (nd) { MG_COOP_SHAPES_ND(5, 8, 4, false, false, CALL) }                         \
            else { MG_COOP_SHAPES(5, 8, 4, false, false, CALL) }                               \
        }                                                                                      \
        if (sh.PX == 6 && !f32) {                                                              \
            if (nd) { MG_COOP_SHAPES_ND(6, 8, 4, false, false, CALL) }                         \
            else { MG_COOP_SHAPES(6, 8, 4, false, false, CALL) }                               \
        }                                                                                      \
        if (sh.PX == 8) {                                                                      \
            if (f32) {                                                                         \
                if (nd) { MG_COOP_FULLX(MG_COOP_SHAPES_ND, 8, 4, 8, true, CALL) }               \
                else if (variant & 1) { MG_COOP_FULLX(MG_COOP_SHAPES, 8, 8, 4, true, CALL) }    \
                else { MG_COOP_FULLX(MG_COOP_SHAPES, 8, 4, 8, true, CALL) }                     \
            } else {                                                                           \
                if (nd) { MG_COOP_FULLX(MG_COOP_SHAPES_ND, 8, 8, 4, false, CALL) }              \
                else { MG_COOP_FULLX(MG_COOP_SHAPES, 8, 8, 4, false, CALL) }                    \
            }                                                                                  \
        }                                                                                      \
        if (sh.PX == 16 && f32 && !nd) { MG_COOP_FULLX(MG_COOP_SHAPES, 16, 6, 4, true, CALL) }  \
        if (sh.PX == 16 && !f32 && !nd) { MG_COOP_FULLX(MG_COOP_SHAPES, 16, 2, 4, false, CALL) } \
        return hipErrorInvalidValue;                                                           \
    }

// the Euler kernel exists in FP64 for nx <= 512
template <int PX, int RJ, int NW, int R0, int R1, int R2, int QMAX, bool FULLX, bool F32C, int ND,
          int NC = 0>
hipError_t euler_kernel_info(const void** fn, size_t* lds, int* nw, int* rows) {
    if constexpr (F32C || PX > 8) {
        return hipErrorInvalidValue;
    } else {
        constexpr int RH = halo_rows<R0, R1, R2, ND>();
        *nw = NW;
        *rows = NW * RJ;
        *fn = (const void*)euler_coop_kernel<PX, RJ, NW, R0, R1, R2, QMAX, FULLX, ND, NC>;
        *lds = coop_lds_bytes<PX, NW, RH, ND, double>();
        return hipSuccess;
    }
}

hipError_t coop_info_classic(const mg_ops* ops, int precision, CoopKind kind, int variant,
                             const void** fn, size_t* lds, int* nw, int* rows) {
    CoopShape sh;
    if (!pick_coop_shape(ops->grid.nx, sh, precision)) return hipErrorInvalidValue;
    const int* R = ops->R;
    const int qmax = ops->qmax;
    // alternative shapes (bit 0) exist for the Taylor kernel without
    // x-dependent factors, FP64 at 4 points per lane and FP32C at 8; the
    // overlapped exchange (bit 1) for every Taylor kernel whose waves hold
    // more than 2 RH rows
    if (variant < 0 || variant >= MG_COOP_VARIANTS) return hipErrorInvalidValue;
    const bool ovl = (variant & 2) != 0;
    if ((variant & 1) &&
        !(kind == CoopKind::Expmv && ops->ND == 0 && ops->NC == 0 &&
          ((precision == MG_FP64 && sh.PX == 4) || (precision == MG_FP32C && sh.PX == 8))))
        return hipErrorInvalidValue;
    if (ovl && kind != CoopKind::Expmv) return hipErrorInvalidValue;
    if (kind == CoopKind::Expmv && ops->NC > 0) {
        // x-terms: FP64, four x-factors, the order-2 band shape, the FP64
        // x-factor workgroup shapes; the x-term vectors add to the LDS
        if (precision != MG_FP64 || ops->ND != MG_MAX_XDIAG ||
            !(R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1))
            return hipErrorInvalidValue;
        const bool full = ops->grid.nx == 64 * sh.PX;
        const size_t xv = (size_t)ops->NXV * 64 * sh.PX * sizeof(double);
#define MG_CHAIN_INFO(PX, RJ, NW, FX)                                                            \
    {                                                                                            \
        const hipError_t e =                                                                     \
            ovl ? coop_kernel_info<PX, RJ, NW, 2, 1, 0, 1, FX, false, MG_MAX_XDIAG, 1, true>(     \
                      fn, lds, nw, rows)                                                         \
                : coop_kernel_info<PX, RJ, NW, 2, 1, 0, 1, FX, false, MG_MAX_XDIAG, 1, false>(    \
                      fn, lds, nw, rows);                                                        \
        *lds += xv;                                                                              \
        return e;                                                                                \
    }
        if (sh.PX == 4) { if (full) { MG_CHAIN_INFO(4, 16, 4, true) } else { MG_CHAIN_INFO(4, 16, 4, false) } }
        if (sh.PX == 5) { MG_CHAIN_INFO(5, 8, 4, false) }
        if (sh.PX == 6) { MG_CHAIN_INFO(6, 8, 4, false) }
        if (sh.PX == 8) { if (full) { MG_CHAIN_INFO(8, 8, 4, true) } else { MG_CHAIN_INFO(8, 8, 4, false) } }
#undef MG_CHAIN_INFO
        return hipErrorInvalidValue;
    }
    if (kind == CoopKind::Euler && ops->xt_in_ba) {
        // B or A with x-terms: the x-term Euler kernels (FP64, four x-factors,
        // the order-2 band shape)
        if (precision != MG_FP64 || ops->ND != MG_MAX_XDIAG ||
            !(R[0] == 2 && R[1] == 1 && R[2] == 0 && qmax == 1))
            return hipErrorInvalidValue;
        const bool full = ops->grid.nx == 64 * sh.PX;
        const size_t xv = (size_t)ops->NXV * 64 * sh.PX * sizeof(double);
#define MG_EULER_XT_INFO(PX, RJ, NW, FX)                                                         \
    {                                                                                            \
        const hipError_t e = euler_kernel_info<PX, RJ, NW, 2, 1, 0, 1, FX, false, MG_MAX_XDIAG, 1>( \
            fn, lds, nw, rows);                                                                  \
        *lds += xv;                                                                              \
        return e;                                                                                \
    }
        if (sh.PX == 4) { if (full) { MG_EULER_XT_INFO(4, 16, 4, true) } else { MG_EULER_XT_INFO(4, 16, 4, false) } }
        if (sh.PX == 5) { MG_EULER_XT_INFO(5, 8, 4, false) }
        if (sh.PX == 6) { MG_EULER_XT_INFO(6, 8, 4, false) }
        if (sh.PX == 8) { if (full) { MG_EULER_XT_INFO(8, 8, 4, true) } else { MG_EULER_XT_INFO(8, 8, 4, false) } }
#undef MG_EULER_XT_INFO
        return hipErrorInvalidValue;
    }
    if (kind == CoopKind::Euler) {
        if (precision != MG_FP64) return hipErrorInvalidValue;
#define MG_CALL_INFO(PX, RJ, NW, R0, R1, R2, QM, FX, F32, ND) \
    euler_kernel_info<PX, RJ, NW, R0, R1, R2, QM, FX, F32, ND>(fn, lds, nw, rows)
        MG_COOP_DISPATCH(MG_CALL_INFO)
#undef MG_CALL_INFO
    }
#define MG_CALL_INFO(PX, RJ, NW, R0, R1, R2, QM, FX, F32, ND)                                   \
    (ovl ? coop_kernel_info<PX, RJ, NW, R0, R1, R2, QM, FX, F32, ND, 0, true>(fn, lds, nw, rows)  \
         : coop_kernel_info<PX, RJ, NW, R0, R1, R2, QM, FX, F32, ND, 0, false>(fn, lds, nw, rows))
    MG_COOP_DISPATCH(MG_CALL_INFO)
#undef MG_CALL_INFO
}

// The kernel a call of this kind runs: the difference-first Taylor kernel
// where one is built for the operator, else the in-place one; `variant`
// selects a variant with the same rows per workgroup and the same arithmetic
// (coop_variant_valid), -1 the one recorded in the operator by the autotuner.
hipError_t coop_info(const mg_ops* ops, int precision, CoopKind kind, KInfo* ki, int variant = -1) {
    if (kind != CoopKind::Expmv) variant = 0;
    else if (variant < 0) variant = ops->tuned_coop[precision == MG_FP32C ? 1 : 0];
    if (kind == CoopKind::Expmv && split_info(ops, precision, ki) == hipSuccess)
        // the difference-first kernel has no alternative of the same arithmetic
        return variant == 0 ? hipSuccess : hipErrorInvalidValue;
    return coop_info_classic(ops, precision, kind, variant, &ki->fn, &ki->lds, &ki->nw, &ki->rows);
}

}  // namespace

int coop_rows_max(int nx) {
    CoopShape sh;
    if (!pick_coop_shape(nx, sh)) return 0;
    // the most rows per workgroup of any shape instantiated for this x width
    // (5, 6 and 8 points per lane: 32 rows, the FP32C shapes of these widths
    // included)
    return sh.PX == 4 ? 64 : sh.PX == 16 ? 24 : 32;
}

int coop_table_rows(int nx, int nv) {
    const int rw = coop_rows_max(nx);
    return rw == 0 ? 0 : (nv + rw - 1) / rw * rw;
}

bool coop_supported(const mg_ops* ops, int precision, CoopKind kind) {
    KInfo ki;
    return coop_info(ops, precision, kind, &ki) == hipSuccess;
}

bool coop_variant_shape(const mg_ops* ops, int precision, int variant, int* nw, int* rows) {
    KInfo ki;
    if (coop_info(ops, precision, CoopKind::Expmv, &ki, variant) != hipSuccess) return false;
    *nw = ki.nw;
    *rows = ki.rows;
    return true;
}

int coop_variant_scratch(const mg_ops* ops, int precision, int variant) {
    KInfo ki;
    if (coop_info(ops, precision, CoopKind::Expmv, &ki, variant) != hipSuccess) return -1;
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, ki.fn) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return (int)at.localSizeBytes;
}

bool coop_variant_valid(const mg_ops* ops, int precision, int variant) {
    KInfo ki;
    return variant >= 0 && variant < MG_COOP_VARIANTS &&
           coop_info(ops, precision, CoopKind::Expmv, &ki, variant) == hipSuccess;
}

// Plan: members per path (G), number of resident groups, exchange-area bytes.
hipError_t coop_plan(const mg_ops* ops, int precision, int64_t P, CoopPlan* plan, CoopKind kind,
                     int variant) {
    KInfo ki;
    plan->stage = 1;
    hipError_t e = coop_info(ops, precision, kind, &ki, variant);
    if (e != hipSuccess) return e;
    const void* fn = ki.fn;
    const size_t lds = ki.lds;
    const int nw = ki.nw, rows = ki.rows;
    // G workgroups of `rows` rows hold a path
    const int G = (ops->grid.nv + rows - 1) / rows;
    if (G * rows > ops->nv_pad) return hipErrorInvalidValue;   // tables shorter than the slabs
    plan->G = G;
    plan->stage = 2;
    if (G < 1 || G > 128) return hipErrorInvalidValue;
    plan->stage = 3;
    plan->lds = lds;
    int dev = 0, cus = 0, per_cu = 0;
    plan->stage = 4;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    plan->cus = cus;
    plan->stage = 5;
    // a shape whose LDS exceeds a compute unit's is not planned (checked
    // before the attribute call, which would leave a pending HIP error)
    int lds_cu = 0;
    if ((e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                   dev)) != hipSuccess)
        return e;
    if (lds > (size_t)lds_cu) return hipErrorInvalidValue;
    if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
            hipSuccess ||
        (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * nw, lds)) != hipSuccess) {
        (void)hipGetLastError();   // the caller may go on with another shape
        return e;
    }
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
    plan->threads = 64 * nw;
    CoopShape sh;
    pick_coop_shape(ops->grid.nx, sh, precision);
    plan->xh_bytes = ((size_t)ngroups * G * 2 * 2 * kRHX * (64 * sh.PX) * elem + 255) & ~(size_t)255;
    plan->xn_bytes = ((size_t)ngroups * G * 2 * nw * 2 * sizeof(double) + 255) & ~(size_t)255;
    // counters: one per wave (the overlapped exchange; the other kernels use
    // the first ngroups * G), then the abort word
    plan->fl_bytes = ((size_t)ngroups * G * nw * sizeof(int) + 256 + 255) & ~(size_t)255;
    plan->bytes = plan->xh_bytes + plan->xn_bytes + plan->fl_bytes;
    return hipSuccess;
}

namespace {
XArea xarea_of(char* xarea, const CoopPlan& plan) {
    XArea x;
    x.xh = xarea;
    x.xn = reinterpret_cast<double*>(xarea + plan.xh_bytes);
    x.fl = reinterpret_cast<int*>(xarea + plan.xh_bytes + plan.xn_bytes);
    x.abort_word = x.fl + (size_t)plan.ngroups * plan.G * (plan.threads / 64);
    x.G = plan.G;
    x.ngroups = plan.ngroups;
    x.xcd_map = plan.xcd_map;
    return x;
}
}  // namespace

hipError_t launch_expmv_coop(const mg_ops* ops, const char* tables, size_t tbytes, int64_t P,
                             int K, const double* u0, int u0_broadcast, double* uT, double tol,
                             int precision, int32_t* stats, int32_t* flags, char* xarea,
                             const CoopPlan& plan, hipStream_t s) {
    KInfo ki;
    hipError_t e = coop_info(ops, precision, CoopKind::Expmv, &ki);
    if (e != hipSuccess) return e;
    const void* fn = ki.fn;
    const size_t lds = ki.lds;
    if (64 * ki.nw != plan.threads || lds != plan.lds) return hipErrorInvalidValue;   // other plan
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
    a.xdiag = ops->xdiag_dev;
    a.xchain = ops->NC > 0 ? mg_xchain_dev(ops) : nullptr;
    a.xdesc = ops->NC > 0 ? mg_xdesc_dev(ops) : nullptr;
    a.nxt = ops->NC;
    a.nxv = ops->NXV;
    a.nv_pad = ops->nv_pad;
    a.x = xarea_of(xarea, plan);
    const int nfl = plan.ngroups * plan.G * (plan.threads / 64);
    hipLaunchKernelGGL(coop_reset_kernel, dim3((nfl + 255) / 256), dim3(256), 0, s, a.x.fl, nfl,
                       a.x.abort_word);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(fn, dim3((unsigned)(plan.ngroups * plan.G)),
                                   dim3(plan.threads), args, (unsigned)lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_euler_coop(const mg_ops* ops, double* u, int64_t P, const double* dWE, int NE,
                             double dt, int32_t* flags, char* xarea, const CoopPlan& plan,
                             hipStream_t s) {
    KInfo ki;
    hipError_t e = coop_info(ops, MG_FP64, CoopKind::Euler, &ki);
    if (e != hipSuccess) return e;
    const void* fn = ki.fn;
    const size_t lds = ki.lds;
    if (64 * ki.nw != plan.threads || lds != plan.lds) return hipErrorInvalidValue;   // other plan
    EulerCoopArgs a;
    a.basis = ops->basis_dev;
    a.nx = ops->grid.nx;
    a.nv = ops->grid.nv;
    a.nv_pad = ops->nv_pad;
    a.P = P;
    a.u = u;
    a.dWE = dWE;
    a.NE = NE;
    a.dt = dt;
    a.flags = flags;
    a.xdiag = ops->xdiag_dev;
    a.xchain = ops->xt_in_ba ? mg_xchain_dev(ops) : nullptr;
    a.xdesc = ops->xt_in_ba ? mg_xdesc_dev(ops) : nullptr;
    a.nxt = ops->xt_in_ba ? ops->NC : 0;
    a.nxv = ops->xt_in_ba ? ops->NXV : 0;
    a.x = xarea_of(xarea, plan);
    const int nfl = plan.ngroups * plan.G * (plan.threads / 64);
    hipLaunchKernelGGL(coop_reset_kernel, dim3((nfl + 255) / 256), dim3(256), 0, s, a.x.fl, nfl,
                       a.x.abort_word);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(fn, dim3((unsigned)(plan.ngroups * plan.G)),
                                   dim3(plan.threads), args, (unsigned)lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}
