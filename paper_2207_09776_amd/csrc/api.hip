// C ABI of the library: argument checking, workspace layout, kernel launches.
// Every check happens on the host before anything is enqueued.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "mg_internal.h"

namespace {

thread_local std::string g_last_error;

// ---- kernel timing (instrumentation) ---------------------------------------
struct TimedLaunch {
    std::string name;
    hipEvent_t start, stop;
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<TimedLaunch> g_timed;

struct TimingScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    const char* name;
    bool on;
    // n == nullptr: never timed (no events are created)
    TimingScope(const char* n, hipStream_t st) : s(st), name(n) {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        on = g_timing_on && n != nullptr;
        if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
        else
            on = false;
    }
    void done() {
        if (!on) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_timing_mu);
        g_timed.push_back({name, a, b});
        on = false;
    }
};

bool is_finite(double x) { return std::isfinite(x); }

mg_status hip_fail(hipError_t e, const char* where) {
    return mg_fail(MG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

mg_status mg_fail(mg_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

extern "C" {

const char* mg_last_error(void) { return g_last_error.c_str(); }

const char* mg_version(void) { return "magnus-mi355x 0.1 (gfx950)"; }

namespace {
// Kernel family for a grid: resident (one workgroup per path) or cooperative.
enum class Family { None, Resident, Coop };
Family family_of(const mg_ops* ops, int precision) {
    if (launch_expmv_resident(ops, nullptr, 0, 1, 1, nullptr, 0, nullptr, 0.0, precision, nullptr,
                              nullptr, nullptr, true) == hipSuccess)
        return Family::Resident;
    if (coop_supported(ops, precision)) return Family::Coop;
    return Family::None;
}
}  // namespace

namespace {
// ---- autotune cache ---------------------------------------------------------
// Kernel shapes picked by mg_autotune_expmv, keyed by the device architecture
// and everything about an operator that decides which kernels and shapes
// exist and how fast they run: grid, precision, order and the form of the
// factored operator (band radii, x-factors, x-terms).  New operators with a
// cached key start with the cached shape; the cache is saved to and loaded
// from a text file by the caller.
struct TuneKey {
    std::string arch;
    int v[13];
    bool operator<(const TuneKey& o) const {
        if (arch != o.arch) return arch < o.arch;
        return std::lexicographical_compare(v, v + 13, o.v, o.v + 13);
    }
};
struct TuneVal {
    int fam, a, b, c;   // fam 0: resident shape (PX, RJ, NW); 1: cooperative variant a
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

// the architecture name of a device without its feature suffixes
void device_arch(int dev, std::string& out) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        out = "unknown";
        return;
    }
    out = prop.gcnArchName;
    const size_t colon = out.find(':');
    if (colon != std::string::npos) out.resize(colon);
}

void tune_key(const mg_ops* ops, int precision, TuneKey& k) {
    device_arch(ops->device, k.arch);
    const int v[13] = {ops->grid.nx, ops->grid.nv, precision, ops->order, ops->ND, ops->NC,
                       ops->NXV,     ops->R[0],   ops->R[1], ops->R[2],  ops->qmax, ops->NBP,
                       ops->nv_pad};
    std::copy(v, v + 13, k.v);
}

// record the operator's tuned shape for `precision`
void tune_cache_store(const mg_ops* ops, int precision) {
    const int pi = precision == MG_FP32C ? 1 : 0;
    TuneVal val{0, 0, 0, 0};
    if (family_of(ops, precision) == Family::Coop) {
        val = {1, ops->tuned_coop[pi], 0, 0};
    } else {
        const int* t = ops->tuned[pi];
        if (t[0] == 0) return;
        val = {0, t[0], t[1], t[2]};
    }
    TuneKey k;
    tune_key(ops, precision, k);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[k] = val;
}

// start a new operator with the cached shapes of its key
void tune_cache_apply(mg_ops* ops) {
    for (int precision : {MG_FP64, MG_FP32C}) {
        TuneVal val;
        TuneKey k;
        tune_key(ops, precision, k);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(k);
            if (it == g_tune.end()) continue;
            val = it->second;
        }
        const int pi = precision == MG_FP32C ? 1 : 0;
        if (val.fam == 1) {
            if (coop_variant_valid(ops, precision, val.a)) ops->tuned_coop[pi] = val.a;
        } else {
            int cand[4][3];
            const int n = resident_candidates(ops->grid.nx, ops->grid.nv, cand, 4);
            for (int i = 0; i < n; ++i)
                if (cand[i][0] == val.a && cand[i][1] == val.b && cand[i][2] == val.c) {
                    ops->tuned[pi][0] = val.a;
                    ops->tuned[pi][1] = val.b;
                    ops->tuned[pi][2] = val.c;
                }
        }
    }
}
}  // namespace

mg_status mg_autotune_cache_save(const char* path, int32_t* entries) {
    g_last_error.clear();
    if (!path) return mg_fail(MG_EINVAL, "mg_autotune_cache_save: NULL path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return mg_fail(MG_EINVAL, std::string("mg_autotune_cache_save: cannot write ") + path);
    std::fprintf(f, "mg-autotune-cache 1\n");
    for (const auto& kv : g_tune) {
        std::fprintf(f, "%s", kv.first.arch.c_str());
        for (int x : kv.first.v) std::fprintf(f, " %d", x);
        std::fprintf(f, " %d %d %d %d\n", kv.second.fam, kv.second.a, kv.second.b, kv.second.c);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) return mg_fail(MG_EINVAL, std::string("mg_autotune_cache_save: cannot write ") + path);
    if (entries) *entries = (int32_t)g_tune.size();
    return MG_OK;
}

mg_status mg_autotune_cache_load(const char* path, int32_t* entries) {
    g_last_error.clear();
    if (!path) return mg_fail(MG_EINVAL, "mg_autotune_cache_load: NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return mg_fail(MG_EINVAL, std::string("mg_autotune_cache_load: cannot read ") + path);
    char line[512];
    std::map<TuneKey, TuneVal> got;
    bool ok = std::fgets(line, sizeof line, f) && std::strncmp(line, "mg-autotune-cache 1", 19) == 0;
    while (ok && std::fgets(line, sizeof line, f)) {
        if (line[0] == '\n' || line[0] == '#') continue;
        char arch[64];
        TuneKey k;
        TuneVal val;
        const int n = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d",
                                  arch, &k.v[0], &k.v[1], &k.v[2], &k.v[3], &k.v[4], &k.v[5],
                                  &k.v[6], &k.v[7], &k.v[8], &k.v[9], &k.v[10], &k.v[11],
                                  &k.v[12], &val.fam, &val.a, &val.b, &val.c);
        if (n != 18 || (val.fam != 0 && val.fam != 1)) {
            ok = false;
            break;
        }
        k.arch = arch;
        got[k] = val;
    }
    std::fclose(f);
    if (!ok) return mg_fail(MG_EINVAL, std::string("mg_autotune_cache_load: malformed file ") + path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : got) g_tune[kv.first] = kv.second;
    if (entries) *entries = (int32_t)got.size();
    return MG_OK;
}

mg_status mg_build_operators(const mg_grid* grid, const mg_coeffs* coeffs, int32_t order,
                             mg_ops** out) {
    g_last_error.clear();
    if (!grid || !coeffs || !out) return mg_fail(MG_EINVAL, "mg_build_operators: NULL argument");
    *out = nullptr;
    if (order < 1 || order > 3) return mg_fail(MG_EINVAL, "mg_build_operators: order must be 1..3");
    if (grid->nx < 1 || grid->nv < 1 || grid->nx > 8192 || grid->nv > 8192)
        return mg_fail(MG_EINVAL, "mg_build_operators: nx and nv must be in 1..8192");
    if (!is_finite(grid->ax) || !is_finite(grid->bx) || !is_finite(grid->av) || !is_finite(grid->bv) ||
        !(grid->bx > grid->ax) || !(grid->bv > grid->av))
        return mg_fail(MG_EINVAL, "mg_build_operators: empty or non-finite domain");
    mg_ops* ops = new (std::nothrow) mg_ops();
    if (!ops) return mg_fail(MG_ENOMEM, "mg_build_operators: out of host memory");
    mg_status st;
    try {
        st = mg_build_host(grid, coeffs, order, ops);
    } catch (const std::bad_alloc&) {
        st = mg_fail(MG_ENOMEM, "mg_build_operators: out of host memory");
    }
    if (st != MG_OK) {
        delete ops;
        return st;
    }
    hipError_t e = hipGetDevice(&ops->device);
    const size_t bytes = ops->basis_host.size() * sizeof(double);
    if (e == hipSuccess) e = hipMalloc((void**)&ops->basis_dev, bytes);
    if (e == hipSuccess)
        e = hipMemcpy(ops->basis_dev, ops->basis_host.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && ops->ND > 0) {
        // x vectors, their statistics, x-term vectors and statistics, then the
        // x-term descriptors (int32, at a 16-byte aligned offset)
        std::vector<double> all(ops->xdiag_host);
        all.insert(all.end(), ops->xstat_host.begin(), ops->xstat_host.end());
        all.insert(all.end(), ops->xchain_host.begin(), ops->xchain_host.end());
        all.insert(all.end(), ops->cstat_host.begin(), ops->cstat_host.end());
        if (all.size() % 2) all.push_back(0.0);
        ops->xdesc_off = all.size();
        all.resize(all.size() + (ops->xdesc_host.size() + 1) / 2, 0.0);
        if (!ops->xdesc_host.empty())
            std::memcpy(all.data() + ops->xdesc_off, ops->xdesc_host.data(),
                        ops->xdesc_host.size() * sizeof(int32_t));
        e = hipMalloc((void**)&ops->xdiag_dev, all.size() * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpy(ops->xdiag_dev, all.data(), all.size() * sizeof(double),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        if (ops->basis_dev) (void)hipFree(ops->basis_dev);
        if (ops->xdiag_dev) (void)hipFree(ops->xdiag_dev);
        delete ops;
        return hip_fail(e, "mg_build_operators");
    }
    // cooperative default: the overlapped exchange where it is built for an
    // operator without x-terms and spills no more than the two-barrier kernel
    // (it was faster on every such shape measured; where it spills, and with
    // x-terms, the autotuner decides); the cache may override
    for (int precision : {MG_FP64, MG_FP32C})
        if (ops->NC == 0 && coop_variant_valid(ops, precision, 2)) {
            const int s2 = coop_variant_scratch(ops, precision, 2);
            const int s0 = coop_variant_scratch(ops, precision, 0);
            if (s2 >= 0 && s0 >= 0 && s2 <= s0) ops->tuned_coop[precision == MG_FP32C ? 1 : 0] = 2;
        }
    tune_cache_apply(ops);
    *out = ops;
    return MG_OK;
}

mg_status mg_free_operators(mg_ops* ops) {
    if (!ops) return MG_OK;
    hipError_t e = hipSuccess;
    if (ops->basis_dev) e = hipFree(ops->basis_dev);
    if (ops->xdiag_dev) {
        hipError_t e2 = hipFree(ops->xdiag_dev);
        if (e == hipSuccess) e = e2;
    }
    delete ops;
    return e == hipSuccess ? MG_OK : hip_fail(e, "mg_free_operators");
}

mg_status mg_iterated_integrals(const double* dW, int64_t P, int64_t Nf, double T, int32_t K,
                                int32_t order, double* coef, double* pathstat, void* stream) {
    g_last_error.clear();
    if (P < 0 || K < 1 || Nf < 1) return mg_fail(MG_ESHAPE, "mg_iterated_integrals: need P >= 0, K >= 1, Nf >= 1");
    if (Nf % K != 0) return mg_fail(MG_ESHAPE, "mg_iterated_integrals: Nf must be a multiple of K");
    if (P > 0x7fffffff) return mg_fail(MG_ESHAPE, "mg_iterated_integrals: P too large");
    if (!(T > 0.0) || !is_finite(T)) return mg_fail(MG_EINVAL, "mg_iterated_integrals: T must be positive");
    if (order < 1 || order > 3) return mg_fail(MG_EINVAL, "mg_iterated_integrals: order must be 1..3");
    if (P == 0) return MG_OK;
    if (!dW || !coef) return mg_fail(MG_EINVAL, "mg_iterated_integrals: NULL pointer");
    hipError_t e = launch_iterated_integrals(dW, P, Nf, T, K, order, coef, pathstat,
                                             (hipStream_t)stream);
    return e == hipSuccess ? MG_OK : hip_fail(e, "mg_iterated_integrals");
}

mg_status mg_iterated_integrals_steps(const double* dW, int64_t P, int64_t Nf, double T,
                                      const int32_t* K, int32_t Kmax, int32_t order, double* coef,
                                      double* pathstat, void* stream) {
    g_last_error.clear();
    const char* where = "mg_iterated_integrals_steps";
    if (P < 0 || Kmax < 1 || Nf < 1)
        return mg_fail(MG_ESHAPE, std::string(where) + ": need P >= 0, Kmax >= 1, Nf >= 1");
    if (P > 0x7fffffff) return mg_fail(MG_ESHAPE, std::string(where) + ": P too large");
    if (!(T > 0.0) || !is_finite(T)) return mg_fail(MG_EINVAL, std::string(where) + ": T must be positive");
    if (order < 1 || order > 3) return mg_fail(MG_EINVAL, std::string(where) + ": order must be 1..3");
    if (P == 0) return MG_OK;
    if (!dW || !K || !coef) return mg_fail(MG_EINVAL, std::string(where) + ": NULL pointer");
    hipError_t e = launch_iterated_integrals_steps(dW, P, Nf, T, K, Kmax, order, coef, pathstat,
                                                   (hipStream_t)stream);
    return e == hipSuccess ? MG_OK : hip_fail(e, where);
}

mg_status mg_euler_increments(const double* dW, int64_t P, int64_t Nf, int32_t NE, double* dWE,
                              void* stream) {
    g_last_error.clear();
    if (P < 0 || NE < 1 || Nf < 1) return mg_fail(MG_ESHAPE, "mg_euler_increments: need P >= 0, NE >= 1, Nf >= 1");
    if (Nf % NE != 0) return mg_fail(MG_ESHAPE, "mg_euler_increments: Nf must be a multiple of NE");
    if (P > ((int64_t)1 << 40) / NE) return mg_fail(MG_ESHAPE, "mg_euler_increments: P*NE too large");
    if (P == 0) return MG_OK;
    if (!dW || !dWE) return mg_fail(MG_EINVAL, "mg_euler_increments: NULL pointer");
    hipError_t e = launch_euler_increments(dW, P, Nf, NE, dWE, (hipStream_t)stream);
    return e == hipSuccess ? MG_OK : hip_fail(e, "mg_euler_increments");
}

size_t mg_workspace_bytes(const mg_ops* ops, int64_t P, int32_t K, int32_t precision) {
    if (!ops || P <= 0 || K <= 0 || (precision != MG_FP64 && precision != MG_FP32C)) return 0;
    size_t bytes = (size_t)P * (size_t)K * mg_table_bytes(ops, precision);
    if (family_of(ops, precision) == Family::Coop) {
        // the largest exchange area of the workgroup shapes the autotuner may
        // pick, so that a workspace sized before tuning still fits after it
        CoopPlan plan;
        if (coop_plan(ops, precision, P, &plan) != hipSuccess) return 0;
        size_t xa = plan.bytes;
        for (int v = 0; v < MG_COOP_VARIANTS; ++v)
            if (coop_variant_valid(ops, precision, v) &&
                coop_plan(ops, precision, P, &plan, CoopKind::Expmv, v) == hipSuccess)
                xa = std::max(xa, plan.bytes);
        bytes += xa;
    }
    return bytes;
}

namespace {

// A validated mg_magnus_expmv call: everything checked, nothing launched.
struct ExpmvCall {
    const mg_ops* ops;
    const double* coef;
    int64_t P;
    int K;
    const double* u0;
    int bcast;
    double* uT;
    int precision;
    double tol;
    int32_t* stats;
    int32_t* flags;
    Family fam = Family::None;
    CoopPlan plan;
    size_t tbytes = 0, need = 0;
};

// Checks one call (everything but the workspace, which the callers check);
// `where` prefixes the error message.
mg_status expmv_prepare(ExpmvCall& c, const std::string& where) {
    if (!c.ops) return mg_fail(MG_EINVAL, where + ": NULL ops");
    if (c.P < 0 || c.K < 1) return mg_fail(MG_ESHAPE, where + ": need P >= 0 and K >= 1");
    if (c.P > 0x7fffffff / (int64_t)c.K) return mg_fail(MG_ESHAPE, where + ": P*K too large");
    if (c.precision != MG_FP64 && c.precision != MG_FP32C)
        return mg_fail(MG_EINVAL, where + ": unknown precision");
    if (!(c.tol == c.tol) || c.tol >= 1.0) return mg_fail(MG_EINVAL, where + ": tol must be < 1");
    if (c.tol <= 0.0) c.tol = c.precision == MG_FP64 ? 0x1p-53 : 0x1p-24;
    if (c.ops->NC > 0 && c.precision != MG_FP64)
        return mg_fail(MG_EUNSUPPORTED,
                       where + ": operators with x-derivative chains (x-dependent noise meeting "
                               "d/dx) are built for MG_FP64 only");
    c.fam = family_of(c.ops, c.precision);
    if (c.fam == Family::None)
        return mg_fail(MG_EUNSUPPORTED,
                       where + (c.ops->ND > 0
                                    ? ": x-dependent coefficients need nx <= 512 (orders 1, 2)"
                                    : ": no kernel for this grid size and precision"));
    if (c.P == 0) return MG_OK;
    if (!c.coef || !c.u0 || !c.uT) return mg_fail(MG_EINVAL, where + ": NULL pointer");
    if (c.fam == Family::Coop) {
        hipError_t e = coop_plan(c.ops, c.precision, c.P, &c.plan);
        if (e != hipSuccess)
            return mg_fail(MG_EUNSUPPORTED,
                           where + ": no cooperative plan: " + hipGetErrorString(e) + " (stage " +
                               std::to_string(c.plan.stage) + ", G " + std::to_string(c.plan.G) +
                               ", per_cu " + std::to_string(c.plan.per_cu) + ", cus " +
                               std::to_string(c.plan.cus) + ", lds " +
                               std::to_string(c.plan.lds) + ")");
    }
    c.tbytes = mg_table_bytes(c.ops, c.precision);
    c.need = (size_t)c.P * c.K * c.tbytes + (c.fam == Family::Coop ? c.plan.bytes : 0);
    return MG_OK;
}

// Positivity check of a batch (after the Taylor kernel): a path whose initial
// state is non-negative solves a forward Kolmogorov equation, so its exact
// solution stays a non-negative density; a final state with a negative part
// beyond kNegativeTol of its maximum marks a Magnus step beyond the
// convergence region of the expansion and sets MG_FLAG_NEGATIVE.  The space
// discretisation alone (central differences, not monotone) also leaves small
// negative values where a grid resolves the density poorly: about 0.04 of the
// maximum for the N(0, 0.25 I) density on 24^2 cells over [-5, 5]^2, below
// 3e-4 on 256^2, against 0.45 for a diverged step of the 256^2 order-3
// workload; the threshold sits between the two.  One workgroup per path: min
// of u0, min and max of uT.
constexpr double kNegativeTol = 0.1;
__global__ __launch_bounds__(256) void negativity_kernel(const double* __restrict__ u0,
                                                         int u0_bcast,
                                                         const double* __restrict__ uT,
                                                         size_t N, int32_t* __restrict__ flags) {
    const int64_t p = blockIdx.x;
    const double* a = u0 + (u0_bcast ? 0 : (size_t)p * N);
    const double* b = uT + (size_t)p * N;
    double amin = 0.0, bmin = 0.0, bmax = 0.0;
    for (size_t i = threadIdx.x; i < N; i += 256) {
        amin = fmin(amin, a[i]);
        bmin = fmin(bmin, b[i]);
        bmax = fmax(bmax, b[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        amin = fmin(amin, __shfl_xor(amin, o, 64));
        bmin = fmin(bmin, __shfl_xor(bmin, o, 64));
        bmax = fmax(bmax, __shfl_xor(bmax, o, 64));
    }
    __shared__ double red[4][3];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = amin;
        red[w][1] = bmin;
        red[w][2] = bmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            amin = fmin(amin, red[k][0]);
            bmin = fmin(bmin, red[k][1]);
            bmax = fmax(bmax, red[k][2]);
        }
        if (amin >= 0.0 && bmin < -kNegativeTol * bmax) atomicOr(&flags[p], MG_FLAG_NEGATIVE);
    }
}

// Launches a prepared call with its workspace.  `timed`: bracket the Taylor
// kernel with the timing instrumentation when it is on (creates HIP events).
mg_status expmv_launch(const ExpmvCall& c, char* ws, hipStream_t s, const std::string& where,
                       bool timed = true) {
    if (c.P == 0) return MG_OK;
    char* tables = ws;
    hipError_t e = launch_assemble(c.ops, c.coef, c.P, c.K, c.tol, c.precision, tables, s);
    if (e != hipSuccess) return hip_fail(e, (where + " (assemble)").c_str());
    TimingScope ts(timed ? "expmv" : nullptr, s);
    if (c.fam == Family::Resident)
        e = launch_expmv_resident(c.ops, tables, c.tbytes, c.P, c.K, c.u0, c.bcast, c.uT, c.tol,
                                  c.precision, c.stats, c.flags, s, false);
    else
        e = launch_expmv_coop(c.ops, tables, c.tbytes, c.P, c.K, c.u0, c.bcast, c.uT, c.tol,
                              c.precision, c.stats, c.flags, tables + (size_t)c.P * c.K * c.tbytes,
                              c.plan, s);
    ts.done();
    if (e == hipSuccess && c.flags) {
        hipLaunchKernelGGL(negativity_kernel, dim3((unsigned)c.P), dim3(256), 0, s, c.u0, c.bcast,
                           c.uT, (size_t)c.ops->grid.nx * c.ops->grid.nv, c.flags);
        e = hipGetLastError();
    }
    return e == hipSuccess ? MG_OK : hip_fail(e, where.c_str());
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace {
// Workspaces hold FP64 tables read in 16-byte units and the 32/64-bit words
// of the cooperative exchange: they must start on a 16-byte boundary (device
// allocations start on much larger ones).
bool ws_aligned(const void* ws) { return ((uintptr_t)ws & 15) == 0; }
}  // namespace

mg_status mg_magnus_expmv(const mg_ops* ops, const double* coef, int64_t P, int32_t K,
                          const double* u0, int32_t u0_broadcast, double* uT, int32_t precision,
                          double tol, void* ws, size_t ws_bytes, int32_t* stats, int32_t* flags,
                          void* stream) {
    g_last_error.clear();
    ExpmvCall c{ops, coef, P, K, u0, u0_broadcast, uT, precision, tol, stats, flags};
    const std::string where = "mg_magnus_expmv";
    mg_status st = expmv_prepare(c, where);
    if (st != MG_OK || P == 0) return st;
    if (!ws) return mg_fail(MG_EINVAL, where + ": NULL pointer");
    if (!ws_aligned(ws)) return mg_fail(MG_EINVAL, where + ": workspace not 16-byte aligned");
    if (ws_bytes < c.need)
        return mg_fail(MG_ENOMEM, where + ": workspace smaller than mg_workspace_bytes()");
    return expmv_launch(c, (char*)ws, (hipStream_t)stream, where);
}

namespace {
// Scratch memory of mg_magnus_expmv_noalloc: its workspace (the per-(path,
// step) tables and the cooperative exchange area) in a device array that the
// runtime places on every device the library runs on when the code object
// is loaded there, held until the process ends.  Host code never names the
// array in device work: on the host `scratch` is only a stand-in; its device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = MG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up on
// the first call on that device, with that device current).
mg_status scratch_on_current_device(char** out, const std::string& where) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, (where + " (hipGetDevice)").c_str());
    if (dev < 0 || dev >= kMaxDevices)
        return mg_fail(MG_EUNSUPPORTED, where + ": device index beyond " + std::to_string(kMaxDevices));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, (where + " (hipGetSymbolAddress)").c_str());
        if (!ptr) return mg_fail(MG_EHIP, where + ": no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}
}  // namespace

mg_status mg_magnus_expmv_noalloc(const mg_ops* ops, const double* coef, int64_t P, int32_t K,
                                  const double* u0, int32_t u0_broadcast, double* uT,
                                  int32_t precision, double tol, int32_t* stats, int32_t* flags,
                                  void* stream) {
    g_last_error.clear();
    ExpmvCall c{ops, coef, P, K, u0, u0_broadcast, uT, precision, tol, stats, flags};
    const std::string where = "mg_magnus_expmv_noalloc";
    mg_status st = expmv_prepare(c, where);
    if (st != MG_OK || P == 0) return st;
    if (c.need > kScratchBytes)
        return mg_fail(MG_ENOMEM, where + ": the call needs " + std::to_string(c.need) +
                                      " bytes of scratch memory, above the fixed " +
                                      std::to_string(kScratchBytes) +
                                      " (use mg_magnus_expmv with a workspace)");
    char* ws = nullptr;
    if ((st = scratch_on_current_device(&ws, where)) != MG_OK) return st;
    // same kernels as mg_magnus_expmv; the timing instrumentation (which
    // creates HIP events) stays off here
    return expmv_launch(c, ws, (hipStream_t)stream, where, false);
}

namespace {
// number of 64-bit words that differ between a and b (bitwise)
__global__ void count_differences(const unsigned long long* a, const unsigned long long* b,
                                  size_t n, unsigned long long* count) {
    unsigned long long c = 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        c += a[i] != b[i];
    if (c) atomicAdd(count, c);
}
}  // namespace

mg_status mg_autotune_expmv(mg_ops* ops, const double* coef, int64_t P, int32_t K,
                            const double* u0, int32_t u0_broadcast, double* uT, int32_t precision,
                            double tol, void* ws, size_t ws_bytes, int32_t reps, char* report,
                            size_t report_bytes, void* stream) {
    g_last_error.clear();
    const std::string where = "mg_autotune_expmv";
    if (report && report_bytes) report[0] = 0;
    ExpmvCall c{ops, coef, P, K, u0, u0_broadcast, uT, precision, tol, nullptr, nullptr};
    mg_status st = expmv_prepare(c, where);
    if (st != MG_OK) return st;
    if (P == 0) return mg_fail(MG_ESHAPE, where + ": need P >= 1");
    if (reps < 1 || reps > 100) return mg_fail(MG_EINVAL, where + ": reps must be in 1..100");
    if (!ws) return mg_fail(MG_EINVAL, where + ": NULL pointer");
    if (!ws_aligned(ws)) return mg_fail(MG_EINVAL, where + ": workspace not 16-byte aligned");
    if (ws_bytes < c.need)
        return mg_fail(MG_ENOMEM, where + ": workspace smaller than mg_workspace_bytes()");
    const int pi = precision == MG_FP32C ? 1 : 0;
    const bool coop = c.fam == Family::Coop;
    // candidates: workgroup shapes of the register-resident kernel, or shape
    // variants of the cooperative kernel; all apply the same operations per
    // point in the same order
    int cand[4][3];
    int cv[MG_COOP_VARIANTS];   // cooperative variants that plan on this device
    int ncand = 0;
    if (!coop && ops->NC == 0) ncand = resident_candidates(ops->grid.nx, ops->grid.nv, cand, 4);
    if (coop) {
        CoopPlan vp;
        for (int v = 0; v < MG_COOP_VARIANTS; ++v)
            if (coop_variant_valid(ops, precision, v) &&
                coop_plan(ops, precision, P, &vp, CoopKind::Expmv, v) == hipSuccess)
                cv[ncand++] = v;
        if (ncand > 0 && cv[0] != 0) ncand = 0;   // the default is the reference
    }
    if (ncand < 2) {
        if (report && report_bytes)
            snprintf(report, report_bytes, "no alternative shapes for this operator and grid");
        return MG_OK;
    }
    std::string rep;
    hipStream_t s = (hipStream_t)stream;
    char* tables = (char*)ws;
    const size_t tab_bytes = (size_t)P * K * c.tbytes;
    hipError_t e = launch_assemble(ops, coef, P, K, c.tol, precision, tables, s);
    if (e != hipSuccess) return hip_fail(e, (where + " (assemble)").c_str());
    const size_t N = (size_t)ops->grid.nx * ops->grid.nv;
    const int tuned_before = ops->tuned_coop[pi];
    double* ref = nullptr;
    unsigned long long* cnt = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int best = -1;
    float best_ms = 0.0f;
    auto cleanup = [&] {
        if (ref) (void)hipFree(ref);
        if (cnt) (void)hipFree(cnt);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    };
    // one launch of candidate i (false: it does not fit the workspace)
    CoopPlan plan;
    auto launch = [&](int i, bool& fits) -> hipError_t {
        fits = true;
        if (!coop)
            return launch_expmv_resident(ops, tables, c.tbytes, P, K, u0, u0_broadcast, uT, c.tol,
                                         precision, nullptr, nullptr, s, false, cand[i]);
        ops->tuned_coop[pi] = cv[i];
        hipError_t le = coop_plan(ops, precision, P, &plan);
        if (le != hipSuccess) return le;
        if (tab_bytes + plan.bytes > ws_bytes) {
            fits = false;
            return hipSuccess;
        }
        return launch_expmv_coop(ops, tables, c.tbytes, P, K, u0, u0_broadcast, uT, c.tol,
                                 precision, nullptr, nullptr, tables + tab_bytes, plan, s);
    };
    // the tuning call is not on a hot path: it allocates a reference copy of
    // uT and synchronises the stream
    if ((e = hipMalloc((void**)&ref, (size_t)P * N * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&cnt, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        cleanup();
        return hip_fail(e, where.c_str());
    }
    for (int i = 0; i < ncand && e == hipSuccess; ++i) {
        // one launch to warm up (and, for the first shape, the reference result)
        bool fits = true;
        e = launch(i, fits);
        if (e != hipSuccess) break;
        char name[96];
        if (coop) {
            int nw = 0, rows = 0;
            (void)coop_variant_shape(ops, precision, cv[i], &nw, &rows);
            snprintf(name, sizeof name, "variant %d (%d waves of %d rows%s)", cv[i], nw,
                     nw ? rows / nw : 0, (cv[i] & 2) ? ", overlapped exchange" : "");
        } else {
            snprintf(name, sizeof name, "PX=%d RJ=%d NW=%d", cand[i][0], cand[i][1], cand[i][2]);
        }
        if (!fits) {
            rep += std::string(i ? "; " : "") + name + ": workspace too small, skipped";
            if (i == 0) break;
            continue;
        }
        unsigned long long diff = 0;
        if (i == 0) {
            e = hipMemcpyAsync(ref, uT, (size_t)P * N * sizeof(double), hipMemcpyDeviceToDevice, s);
        } else {
            e = hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(count_differences, dim3(1024), dim3(256), 0, s,
                                   reinterpret_cast<const unsigned long long*>(uT),
                                   reinterpret_cast<const unsigned long long*>(ref),
                                   (size_t)P * N, cnt);
                e = hipGetLastError();
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(&diff, cnt, sizeof(diff), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (e != hipSuccess) break;
        (void)hipEventRecord(a, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(i, fits);
        (void)hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) break;
        ms /= (float)reps;
        char line[200];
        snprintf(line, sizeof line, "%s%s: %.3f ms%s", i ? "; " : "", name, ms,
                 diff ? " (result differs: excluded)" : "");
        rep += line;
        // every candidate computes the same operations per point in the same
        // order, so the results must agree bit for bit
        if (diff == 0 && (best < 0 || ms < best_ms)) {
            best = i;
            best_ms = ms;
        }
    }
    cleanup();
    if (coop) ops->tuned_coop[pi] = tuned_before;
    if (e != hipSuccess) return hip_fail(e, where.c_str());
    if (best < 0) {
        if (report && report_bytes) snprintf(report, report_bytes, "%s", rep.c_str());
        return MG_OK;
    }
    if (coop) {
        ops->tuned_coop[pi] = cv[best];
        rep += "; chosen variant " + std::to_string(cv[best]);
    } else {
        int* t = ops->tuned[pi];
        t[0] = cand[best][0];
        t[1] = cand[best][1];
        t[2] = cand[best][2];
        rep += "; chosen PX=" + std::to_string(t[0]) + " RJ=" + std::to_string(t[1]) +
               " NW=" + std::to_string(t[2]);
    }
    tune_cache_store(ops, precision);
    if (report && report_bytes) snprintf(report, report_bytes, "%s", rep.c_str());
    return MG_OK;
}

namespace {

// The ladder shared by the two step-size selections: argument checks, the
// device buffers of a set-up call, and one rung (both orders over the paths
// at K steps, their relative distances and flags copied to the host).
struct StepLadder {
    const mg_ops *ops2, *ops3;
    const double *dW, *u0;
    int64_t P, Nf;
    double T;
    int32_t precision;
    void* stream;
    size_t N = 0, wsb = 0;
    double *coef = nullptr, *u2 = nullptr, *u3 = nullptr, *err = nullptr;
    int32_t* fl = nullptr;
    void* ws = nullptr;
    std::vector<double> herr;
    std::vector<int32_t> hfl;

    ~StepLadder() {
        for (void* q : {(void*)coef, (void*)u2, (void*)u3, (void*)err, (void*)fl, ws})
            if (q) (void)hipFree(q);
    }
    StepLadder(const StepLadder&) = delete;              // owns its device buffers
    StepLadder& operator=(const StepLadder&) = delete;

    mg_status check(const std::string& where, int32_t K0, int32_t factor, int32_t Kmax,
                    double tol) const {
        if (!ops2 || !ops3 || !dW || !u0) return mg_fail(MG_EINVAL, where + ": NULL pointer");
        if (ops2->order != 2 || ops3->order != 3)
            return mg_fail(MG_EINVAL, where + ": need operators of orders 2 and 3");
        const mg_grid& g2 = ops2->grid;
        const mg_grid& g3 = ops3->grid;
        if (g2.nx != g3.nx || g2.nv != g3.nv || g2.ax != g3.ax || g2.bx != g3.bx ||
            g2.av != g3.av || g2.bv != g3.bv)
            return mg_fail(MG_EINVAL, where + ": the two operators are on different grids");
        if (P < 1 || P > 0x7fffffff || Nf < 1) return mg_fail(MG_ESHAPE, where + ": bad sizes");
        if (K0 < 1 || factor < 2 || Kmax < K0 || Nf % K0 != 0)
            return mg_fail(MG_EINVAL,
                           where + ": need K0 >= 1 dividing Nf, factor >= 2, Kmax >= K0");
        if (!(tol > 0.0) || !is_finite(T) || !(T > 0.0))
            return mg_fail(MG_EINVAL, where + ": need tol > 0 and T > 0");
        return MG_OK;
    }

    // buffers sized for the largest K the ladder may reach
    mg_status allocate(const std::string& where, int32_t K0, int32_t factor, int32_t Kmax) {
        N = (size_t)ops2->grid.nx * ops2->grid.nv;
        int64_t Kcap = K0;
        while (Kcap * factor <= Kmax && Nf % (Kcap * factor) == 0) Kcap *= factor;
        const size_t ws2 = mg_workspace_bytes(ops2, P, (int32_t)Kcap, precision);
        const size_t ws3 = mg_workspace_bytes(ops3, P, (int32_t)Kcap, precision);
        if (ws2 == 0 || ws3 == 0)
            return mg_fail(MG_EUNSUPPORTED, where + ": no kernel for this grid and precision");
        wsb = std::max(ws2, ws3);
        hipError_t e = hipSuccess;
        if ((e = hipMalloc((void**)&coef, (size_t)P * Kcap * 6 * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&u2, (size_t)P * N * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&u3, (size_t)P * N * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&err, (size_t)P * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&fl, (size_t)P * 2 * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc(&ws, wsb)) != hipSuccess)
            return hip_fail(e, where.c_str());
        herr.assign((size_t)P, 0.0);
        hfl.assign((size_t)P * 2, 0);
        return MG_OK;
    }

    // one rung: gap(p) = ||u3_p - u2_p||_F / ||u3_p||_F at K steps, +inf for a
    // flagged or non-finite path
    mg_status rung(const std::string& where, int32_t K, std::vector<double>& gap) {
        mg_status st;
        if ((st = mg_iterated_integrals(dW, P, Nf, T, K, 3, coef, nullptr, stream)) != MG_OK)
            return st;
        // the order-3 weights: their first four are the order-2 ones
        if ((st = mg_magnus_expmv(ops2, coef, P, K, u0, 1, u2, precision, 0.0, ws, wsb, nullptr,
                                  fl, stream)) != MG_OK)
            return st;
        if ((st = mg_magnus_expmv(ops3, coef, P, K, u0, 1, u3, precision, 0.0, ws, wsb, nullptr,
                                  fl + P, stream)) != MG_OK)
            return st;
        if ((st = mg_error_vs_exact(&ops2->grid, nullptr, nullptr, u2, u3, P, 0, err, stream)) !=
            MG_OK)
            return st;
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = hipSuccess;
        if ((e = hipMemcpyAsync(herr.data(), err, (size_t)P * sizeof(double),
                                hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(hfl.data(), fl, (size_t)P * 2 * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, where.c_str());
        gap.resize((size_t)P);
        for (int64_t p = 0; p < P; ++p)
            gap[p] = (hfl[p] || hfl[P + p] || !std::isfinite(herr[p]))
                         ? std::numeric_limits<double>::infinity()
                         : herr[p];
        return MG_OK;
    }
};

}  // namespace

mg_status mg_select_magnus_steps(const mg_ops* ops2, const mg_ops* ops3, const double* dW,
                                 int64_t Ps, int64_t Nf, double T, const double* u0, int32_t K0,
                                 int32_t factor, int32_t Kmax, double tol, int32_t precision,
                                 int32_t* K_out, double* gap_out, int32_t* accepted,
                                 void* stream) {
    g_last_error.clear();
    const std::string where = "mg_select_magnus_steps";
    if (!K_out || !gap_out || !accepted) return mg_fail(MG_EINVAL, where + ": NULL pointer");
    StepLadder L{ops2, ops3, dW, u0, Ps, Nf, T, precision, stream};
    mg_status st = L.check(where, K0, factor, Kmax, tol);
    if (st != MG_OK || (st = L.allocate(where, K0, factor, Kmax)) != MG_OK) return st;
    std::vector<double> gaps;
    int32_t K = K0, lastK = 0;
    double lastgap = 0.0;
    bool ok = false;
    while (K <= Kmax && Nf % K == 0) {
        if ((st = L.rung(where, K, gaps)) != MG_OK) return st;
        // the largest distance over the sample decides
        double gap = 0.0;
        for (double g : gaps) gap = std::max(gap, g);
        lastK = K;
        lastgap = gap;
        if (gap <= tol) {
            ok = true;
            break;
        }
        if ((int64_t)K * factor > 0x7fffffff) break;
        K *= factor;
    }
    *K_out = lastK;
    *gap_out = lastgap;
    *accepted = ok ? 1 : 0;
    return MG_OK;
}

mg_status mg_select_magnus_steps_per_path(const mg_ops* ops2, const mg_ops* ops3,
                                          const double* dW, int64_t P, int64_t Nf, double T,
                                          const double* u0, int32_t K0, int32_t factor,
                                          int32_t Kmax, double tol, int32_t precision,
                                          int32_t* K_out, double* gap_out, int64_t* n_accepted,
                                          void* stream) {
    g_last_error.clear();
    const std::string where = "mg_select_magnus_steps_per_path";
    if (!K_out || !gap_out || !n_accepted) return mg_fail(MG_EINVAL, where + ": NULL pointer");
    StepLadder L{ops2, ops3, dW, u0, P, Nf, T, precision, stream};
    mg_status st = L.check(where, K0, factor, Kmax, tol);
    if (st != MG_OK || (st = L.allocate(where, K0, factor, Kmax)) != MG_OK) return st;
    std::vector<double> gaps;
    std::vector<char> done((size_t)P, 0);
    int64_t nacc = 0;
    int32_t K = K0;
    // every rung runs as one batch over the paths until all are accepted; a
    // path keeps the first step count whose distance is within tol
    while (K <= Kmax && Nf % K == 0 && nacc < P) {
        if ((st = L.rung(where, K, gaps)) != MG_OK) return st;
        for (int64_t p = 0; p < P; ++p) {
            if (done[p]) continue;
            K_out[p] = K;
            gap_out[p] = gaps[p];
            if (gaps[p] <= tol) {
                done[p] = 1;
                ++nacc;
            }
        }
        if ((int64_t)K * factor > 0x7fffffff) break;
        K *= factor;
    }
    *n_accepted = nacc;
    return MG_OK;
}

namespace {
// dst row (dst_idx ? dst_idx[i] : i) = columns [off, off + len) of src row
// (src_idx ? src_idx[i] : i), for i < n (a src_stride of 0 repeats one row)
__global__ void copy_rows(const double* __restrict__ src, size_t src_stride, size_t off,
                          const int32_t* __restrict__ src_idx, double* __restrict__ dst,
                          size_t dst_stride, const int32_t* __restrict__ dst_idx, int64_t n,
                          size_t len) {
    const size_t total = (size_t)n * len;
    for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (size_t)gridDim.x * 256) {
        const size_t i = t / len, c = t % len;
        const size_t sr = src_idx ? (size_t)src_idx[i] : i;
        const size_t dr = dst_idx ? (size_t)dst_idx[i] : i;
        dst[dr * dst_stride + c] = src[sr * src_stride + off + c];
    }
}

hipError_t launch_copy_rows(const double* src, size_t src_stride, size_t off,
                            const int32_t* src_idx, double* dst, size_t dst_stride,
                            const int32_t* dst_idx, int64_t n, size_t len, hipStream_t s) {
    const size_t total = (size_t)n * len;
    if (total == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_rows, dim3(blocks), dim3(256), 0, s, src, src_stride, off, src_idx,
                       dst, dst_stride, dst_idx, n, len);
    return hipGetLastError();
}
}  // namespace

mg_status mg_magnus_adaptive(const mg_ops* ops2, const mg_ops* ops3, const double* dW, int64_t P,
                             int64_t Nf, double T, const double* u0, int32_t u0_broadcast,
                             double* uT, int32_t K0, int32_t factor, int32_t max_level,
                             double tol, int32_t precision, int32_t* levels, double* gaps,
                             void* stream) {
    g_last_error.clear();
    const std::string where = "mg_magnus_adaptive";
    if (!levels || !gaps || !uT) return mg_fail(MG_EINVAL, where + ": NULL pointer");
    StepLadder L{ops2, ops3, dW, u0, P, Nf, T, precision, stream};
    // the ladder's checks (orders, grids, sizes, K0 | Nf, factor, tol, T)
    mg_status st = L.check(where, K0, factor, K0, tol);
    if (st != MG_OK) return st;
    if (max_level < 0 || max_level > 20) return mg_fail(MG_EINVAL, where + ": max_level in 0..20");
    int64_t mmax = 1;
    for (int i = 0; i < max_level; ++i) mmax *= factor;
    const int64_t n = Nf / K0;
    if (mmax > (1 << 20) || n % mmax != 0)
        return mg_fail(MG_EINVAL,
                       where + ": factor^max_level must divide the fine increments of a step");
    // buffers: the ladder's (coefficients for mmax sub-steps, u2, u3, distances,
    // flags, expmv workspace) plus a slice of dW, the states of the active
    // paths and three index lists
    if ((st = L.allocate(where, (int32_t)mmax, 2, (int32_t)mmax)) != MG_OK) return st;
    const size_t N = L.N;
    double *dws = nullptr, *ucur = nullptr;
    int32_t* idx = nullptr;
    struct Free {
        double** a;
        double** b;
        int32_t** c;
        ~Free() {
            if (*a) (void)hipFree(*a);
            if (*b) (void)hipFree(*b);
            if (*c) (void)hipFree(*c);
        }
    } release{&dws, &ucur, &idx};
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if ((e = hipMalloc((void**)&dws, (size_t)P * n * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&ucur, (size_t)P * N * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&idx, (size_t)P * 3 * sizeof(int32_t))) != hipSuccess)
        return hip_fail(e, where.c_str());
    // the state of every path starts as u0
    if ((e = launch_copy_rows(u0, u0_broadcast ? 0 : N, 0, nullptr, uT, N, nullptr, P, N, s)) !=
        hipSuccess)
        return hip_fail(e, where.c_str());
    const double h = T / K0;
    std::vector<int32_t> active, acc_pos, acc_row, next;
    for (int32_t k = 0; k < K0; ++k) {
        active.resize((size_t)P);
        for (int64_t p = 0; p < P; ++p) active[p] = (int32_t)p;
        int64_t m = 1;
        for (int32_t lev = 0; lev <= max_level && !active.empty(); ++lev, m *= factor) {
            const int64_t A = (int64_t)active.size();
            // the active paths' increments of this coarse step and their states
            if ((e = hipMemcpyAsync(idx, active.data(), A * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = launch_copy_rows(dW, Nf, (size_t)k * n, idx, dws, n, nullptr, A, n, s)) !=
                    hipSuccess ||
                (e = launch_copy_rows(uT, N, 0, idx, ucur, N, nullptr, A, N, s)) != hipSuccess)
                return hip_fail(e, where.c_str());
            // orders 2 and 3 over m sub-steps (the order-3 weights; their
            // first four are the order-2 ones), and their distances
            if ((st = mg_iterated_integrals(dws, A, n, h, (int32_t)m, 3, L.coef, nullptr,
                                            stream)) != MG_OK ||
                (st = mg_magnus_expmv(ops2, L.coef, A, (int32_t)m, ucur, 0, L.u2, precision, 0.0,
                                      L.ws, L.wsb, nullptr, L.fl, stream)) != MG_OK ||
                (st = mg_magnus_expmv(ops3, L.coef, A, (int32_t)m, ucur, 0, L.u3, precision, 0.0,
                                      L.ws, L.wsb, nullptr, L.fl + P, stream)) != MG_OK ||
                (st = mg_error_vs_exact(&ops2->grid, nullptr, nullptr, L.u2, L.u3, A, 0, L.err,
                                        stream)) != MG_OK)
                return st;
            if ((e = hipMemcpyAsync(L.herr.data(), L.err, A * sizeof(double),
                                    hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipMemcpyAsync(L.hfl.data(), L.fl, A * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipMemcpyAsync(L.hfl.data() + P, L.fl + P, A * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(e, where.c_str());
            // accept within tol (or at the last level): the order-3 state
            // replaces the path's; the others are redone at the next level
            acc_pos.clear();
            acc_row.clear();
            next.clear();
            for (int64_t i = 0; i < A; ++i) {
                const int32_t p = active[i];
                double g = L.herr[i];
                if (L.hfl[i] || L.hfl[P + i] || !std::isfinite(g))
                    g = std::numeric_limits<double>::infinity();
                if (g <= tol || lev == max_level) {
                    levels[(size_t)p * K0 + k] = lev;
                    gaps[(size_t)p * K0 + k] = g;
                    acc_pos.push_back((int32_t)i);
                    acc_row.push_back(p);
                } else {
                    next.push_back(p);
                }
            }
            const int64_t nacc = (int64_t)acc_pos.size();
            if (nacc > 0) {
                if ((e = hipMemcpyAsync(idx + P, acc_pos.data(), nacc * sizeof(int32_t),
                                        hipMemcpyHostToDevice, s)) != hipSuccess ||
                    (e = hipMemcpyAsync(idx + 2 * P, acc_row.data(), nacc * sizeof(int32_t),
                                        hipMemcpyHostToDevice, s)) != hipSuccess ||
                    (e = launch_copy_rows(L.u3, N, 0, idx + P, uT, N, idx + 2 * P, nacc, N,
                                          s)) != hipSuccess ||
                    (e = hipStreamSynchronize(s)) != hipSuccess)
                    return hip_fail(e, where.c_str());
            }
            active.swap(next);
        }
    }
    return MG_OK;
}

size_t mg_workspace_bytes_multi(const mg_job* jobs, int32_t njobs) {
    if (!jobs || njobs <= 0) return 0;
    size_t total = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        const mg_job& j = jobs[i];
        if (j.P <= 0) continue;
        const size_t b = mg_workspace_bytes(j.ops, j.P, j.K, j.precision);
        if (b == 0) return 0;
        total += round256(b);
    }
    return total;
}

mg_status mg_magnus_expmv_multi(const mg_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                                void* stream) {
    g_last_error.clear();
    if (njobs < 0) return mg_fail(MG_EINVAL, "mg_magnus_expmv_multi: njobs < 0");
    if (njobs == 0) return MG_OK;
    if (!jobs) return mg_fail(MG_EINVAL, "mg_magnus_expmv_multi: NULL jobs");
    std::vector<ExpmvCall> calls;
    calls.reserve(njobs);
    size_t total = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        const mg_job& j = jobs[i];
        ExpmvCall c{j.ops, j.coef, j.P, j.K, j.u0, j.u0_broadcast, j.uT, j.precision, j.tol,
                    j.stats, j.flags};
        mg_status st = expmv_prepare(c, "mg_magnus_expmv_multi: job " + std::to_string(i));
        if (st != MG_OK) return st;
        if (c.P > 0) total += round256(c.need);
        calls.push_back(c);
    }
    if (total > 0 && !ws) return mg_fail(MG_EINVAL, "mg_magnus_expmv_multi: NULL workspace");
    if (total > 0 && !ws_aligned(ws))
        return mg_fail(MG_EINVAL, "mg_magnus_expmv_multi: workspace not 16-byte aligned");
    if (ws_bytes < total)
        return mg_fail(MG_ENOMEM,
                       "mg_magnus_expmv_multi: workspace smaller than mg_workspace_bytes_multi()");
    char* base = (char*)ws;
    size_t off = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        if (calls[i].P == 0) continue;
        mg_status st = expmv_launch(calls[i], base + off, (hipStream_t)stream,
                                    "mg_magnus_expmv_multi: job " + std::to_string(i));
        if (st != MG_OK) return st;
        off += round256(calls[i].need);
    }
    return MG_OK;
}

namespace {
// Euler kernel family: resident (nx, nv <= 128) or cooperative (nx <= 512)
Family euler_family(const mg_ops* ops) {
    if (launch_euler_resident(ops, nullptr, 1, nullptr, 1, 0.0, nullptr, nullptr, true) ==
        hipSuccess)
        return Family::Resident;
    if (coop_supported(ops, MG_FP64, CoopKind::Euler)) return Family::Coop;
    return Family::None;
}
}  // namespace

size_t mg_euler_workspace_bytes(const mg_ops* ops, int64_t P) {
    if (!ops || P < 0) return (size_t)-1;
    const Family f = euler_family(ops);
    if (f == Family::None) return (size_t)-1;
    if (f == Family::Resident || P == 0) return 0;
    CoopPlan plan;
    if (coop_plan(ops, MG_FP64, P, &plan, CoopKind::Euler) != hipSuccess) return (size_t)-1;
    return plan.bytes;
}

mg_status mg_euler_step(const mg_ops* ops, double* u, int64_t P, const double* dWE, int32_t NE,
                        double dt, int32_t precision, void* ws, size_t ws_bytes, int32_t* flags,
                        void* stream) {
    g_last_error.clear();
    if (!ops) return mg_fail(MG_EINVAL, "mg_euler_step: NULL ops");
    if (P < 0 || NE < 0) return mg_fail(MG_ESHAPE, "mg_euler_step: need P >= 0 and NE >= 0");
    if (P > 0x7fffffff) return mg_fail(MG_ESHAPE, "mg_euler_step: P too large");
    if (precision != MG_FP64) return mg_fail(MG_EUNSUPPORTED, "mg_euler_step: only MG_FP64");
    if (!is_finite(dt)) return mg_fail(MG_EINVAL, "mg_euler_step: dt must be finite");
    hipStream_t s = (hipStream_t)stream;
    const Family fam = euler_family(ops);
    if (fam == Family::None)
        return mg_fail(MG_EUNSUPPORTED, "mg_euler_step: no kernel for this grid size");
    if (P == 0 || NE == 0) return MG_OK;
    if (!u || !dWE) return mg_fail(MG_EINVAL, "mg_euler_step: NULL pointer");
    CoopPlan plan;
    if (fam == Family::Coop) {
        hipError_t e = coop_plan(ops, MG_FP64, P, &plan, CoopKind::Euler);
        if (e != hipSuccess) return hip_fail(e, "mg_euler_step: cooperative plan");
        if (!ws || ws_bytes < plan.bytes)
            return mg_fail(MG_ENOMEM, "mg_euler_step: workspace too small (need " +
                                          std::to_string(plan.bytes) + " bytes)");
        if (!ws_aligned(ws)) return mg_fail(MG_EINVAL, "mg_euler_step: workspace not 16-byte aligned");
    }
    TimingScope ts("euler", s);
    hipError_t e = fam == Family::Resident
                       ? launch_euler_resident(ops, u, P, dWE, NE, dt, flags, s, false)
                       : launch_euler_coop(ops, u, P, dWE, NE, dt, flags,
                                           static_cast<char*>(ws), plan, s);
    ts.done();
    return e == hipSuccess ? MG_OK : hip_fail(e, "mg_euler_step");
}

mg_status mg_error_vs_exact(const mg_grid* grid, const mg_exact* ex, const double* pathstat,
                            const double* u, const double* uref, int64_t P, int32_t kappa,
                            double* err, void* stream) {
    g_last_error.clear();
    if (!grid) return mg_fail(MG_EINVAL, "mg_error_vs_exact: NULL grid");
    if (P < 0 || P > 0x7fffffff) return mg_fail(MG_ESHAPE, "mg_error_vs_exact: bad P");
    if (grid->nx < 1 || grid->nv < 1 || !(grid->bx > grid->ax) || !(grid->bv > grid->av))
        return mg_fail(MG_EINVAL, "mg_error_vs_exact: bad grid");
    if (kappa < 0 || kappa > 30 || (grid->nx >> kappa) < 1 || (grid->nv >> kappa) < 1)
        return mg_fail(MG_EINVAL, "mg_error_vs_exact: kappa window is empty");
    if (!uref) {
        if (!ex) return mg_fail(MG_EINVAL, "mg_error_vs_exact: NULL exact parameters");
        if (!(ex->sigma * ex->sigma < ex->a) || !(ex->s0sq > 0.0) || !(ex->T > 0.0))
            return mg_fail(MG_EINVAL, "mg_error_vs_exact: need sigma^2 < a, s0sq > 0, T > 0");
    }
    if (P == 0) return MG_OK;
    if (!u || !err || (!uref && !pathstat))
        return mg_fail(MG_EINVAL, "mg_error_vs_exact: NULL pointer");
    hipError_t e = launch_error_vs_exact(grid, ex, pathstat, u, uref, P, kappa, err,
                                         (hipStream_t)stream);
    return e == hipSuccess ? MG_OK : hip_fail(e, "mg_error_vs_exact");
}

mg_status mg_check_flags(const int32_t* flags, int64_t P, int32_t* bits_out, int64_t* first_out,
                         void* stream) {
    g_last_error.clear();
    if (bits_out) *bits_out = 0;
    if (first_out) *first_out = -1;
    if (P < 0) return mg_fail(MG_ESHAPE, "mg_check_flags: P < 0");
    if (P == 0) return MG_OK;
    if (!flags) return mg_fail(MG_EINVAL, "mg_check_flags: NULL flags");
    std::vector<int32_t> h;
    try {
        h.resize((size_t)P);
    } catch (const std::bad_alloc&) {
        return mg_fail(MG_ENOMEM, "mg_check_flags: out of host memory");
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h.data(), flags, (size_t)P * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "mg_check_flags");
    int32_t bits = 0;
    int64_t first = -1, count = 0;
    for (int64_t p = 0; p < P; ++p)
        if (h[(size_t)p]) {
            bits |= h[(size_t)p];
            if (first < 0) first = p;
            ++count;
        }
    if (bits_out) *bits_out = bits;
    if (first_out) *first_out = first;
    if (count == 0) return MG_OK;
    return mg_fail(MG_ENONFINITE, "mg_check_flags: " + std::to_string(count) + " of " +
                                      std::to_string(P) + " paths flagged (first: path " +
                                      std::to_string(first) + ", bits " + std::to_string(bits) +
                                      ")");
}

mg_status mg_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_on = on != 0;
    return MG_OK;
}

mg_status mg_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    for (auto& t : g_timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    g_timed.clear();
    return MG_OK;
}

mg_status mg_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
    g_last_error.clear();
    if (!kernel || !total_ms || !launches) return mg_fail(MG_EINVAL, "mg_timing_read: NULL");
    std::lock_guard<std::mutex> lk(g_timing_mu);
    double tot = 0.0;
    int64_t n = 0;
    for (auto& t : g_timed) {
        if (t.name != kernel) continue;
        hipError_t e = hipEventSynchronize(t.stop);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess) return hip_fail(e, "mg_timing_read");
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return MG_OK;
}

}  // extern "C"
