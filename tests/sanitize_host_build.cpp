// Host-only driver of the operator build (the Kronecker-factored Magnus
// basis of Section 2) for the address and undefined-behaviour sanitizers:
// tests/test_host_sanitizers.py compiles this file together with
// paper_2207_09776_amd/csrc/ops_build.cpp by g++ (no device code, no HIP
// calls) and runs it.  Each case builds the basis for one coefficient set
// and order and checks the status and the shape of the result; any
// out-of-bounds access, leak or undefined operation in the build aborts the
// run with a sanitizer report.

#include "ops_build.cpp"

#include <cmath>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

mg_status mg_fail(mg_status code, const std::string& msg) {
    std::printf("  status %d: %s\n", (int)code, msg.c_str());
    return code;
}
// the table padding of the kernel shapes is irrelevant here
int resident_rows(int, int) { return 0; }
int coop_table_rows(int, int nv) { return nv; }

namespace {

using Fn = std::function<double(double, double)>;

struct Set {
    const char* name;
    Fn h, fx, fv, gxx, gxv, gvv, sig, sx, sv;
};

int failures = 0;

// Interior nodes x_i = a + i (b - a)/(n + 1), i = 1..n; grids [nv][nx], x fastest.
std::vector<double> sample(const Fn& f, int nx, int nv, double lo, double hi) {
    std::vector<double> z((size_t)nx * nv);
    for (int j = 0; j < nv; ++j)
        for (int i = 0; i < nx; ++i) {
            const double x = lo + (i + 1) * (hi - lo) / (nx + 1);
            const double v = lo + (j + 1) * (hi - lo) / (nv + 1);
            z[(size_t)j * nx + i] = f(x, v);
        }
    return z;
}

void run(const Set& s, int nx, int nv, int order, bool expect_ok) {
    const double lo = -4.0, hi = 4.0;
    std::vector<double> arr[9];
    const Fn* fns[9] = {&s.h, &s.fx, &s.fv, &s.gxx, &s.gxv, &s.gvv, &s.sig, &s.sx, &s.sv};
    const double* ptr[9];
    for (int k = 0; k < 9; ++k) {
        ptr[k] = nullptr;
        if (*fns[k]) {
            arr[k] = sample(*fns[k], nx, nv, lo, hi);
            ptr[k] = arr[k].data();
        }
    }
    mg_grid g{nx, nv, lo, hi, lo, hi};
    mg_coeffs c{};
    c.h = ptr[0];
    c.fx = ptr[1];
    c.fv = ptr[2];
    c.gxx = ptr[3];
    c.gxv = ptr[4];
    c.gvv = ptr[5];
    c.sig = ptr[6];
    c.sx = ptr[7];
    c.sv = ptr[8];
    mg_ops* ops = new mg_ops();
    const mg_status st = mg_build_host(&g, &c, order, ops);
    const bool ok = st == MG_OK;
    std::printf("%-28s %4dx%-4d order %d: %s (ND %d, x-terms %d, x vectors %d, NBP %d)\n", s.name,
                nx, nv, order, ok ? "built" : "rejected", ops->ND, ops->NC, ops->NXV, ops->NBP);
    if (ok != expect_ok) {
        std::printf("  UNEXPECTED: expected %s\n", expect_ok ? "a build" : "a rejection");
        ++failures;
    }
    if (ok) {
        const size_t rows = (size_t)MG_NBASIS * ops->nv_pad;
        if (ops->basis_host.size() != rows * (ops->NBP + ops->NCB) ||
            ops->xdesc_host.size() != (size_t)ops->NC * 4 ||
            ops->xchain_host.size() != (size_t)ops->NXV * nx) {
            std::printf("  UNEXPECTED: table sizes\n");
            ++failures;
        }
        for (double v : ops->basis_host)
            if (!std::isfinite(v)) {
                std::printf("  UNEXPECTED: non-finite table entry\n");
                ++failures;
                break;
            }
    }
    delete ops;
}

}  // namespace

int main() {
    const double a = 1.1, sigma = 1.0 / std::sqrt(10.0);
    const Fn none;
    // eq. (coeffsLangevinConst): constant diffusion and noise, transport -v d/dx
    Set constant{"constant Langevin", none, [](double, double v) { return -v; }, none, none, none,
                 [=](double, double) { return a; }, none, none,
                 [=](double, double) { return sigma; }};
    // eq. (coeffsLangevinVar): x-dependent diffusion and noise through d/dv
    Set paper_var{"variable Langevin", none, [](double, double v) { return -v; }, none, none, none,
                  [=](double x, double) { return a * (1.0 + 1.0 / (x * x + 1.0)); }, none, none,
                  [=](double x, double) { return sigma * std::sqrt(1.0 + 1.0 / (x * x + 1.0)); }};
    // x,v-dependent diffusion (a short sum of products), v-dependent noise
    Set xv{"x,v-dependent diffusion", none, [](double, double v) { return -v; }, none, none, none,
           [](double x, double v) {
               const double s = 1.0 + 0.3 * std::exp(-0.5 * (x * x + v * v));
               return s * s;
           },
           none, none, [](double, double v) { return 0.5 / (1.0 + 0.1 * v * v); }};
    // every v-dependent term of eq. (generalSPDE) that the build takes
    Set general_v{"v-dependent general set", [](double, double v) { return -0.1 * v * v; },
                  [](double, double v) { return -v; }, [](double, double v) { return 0.2 * v; },
                  none, [](double, double v) { return 0.05 + 0.01 * v; },
                  [](double, double v) { return 1.0 + 0.1 * v * v; },
                  [](double, double v) { return 0.1 * v; }, none,
                  [](double, double) { return 0.5; }};
    Set with_gxx{"g^xx", none, [](double, double v) { return -v; }, none,
                 [](double x, double) { return 0.5 + 0.2 / (1.0 + x * x); }, none,
                 [](double, double) { return 1.0; }, none, none, [](double, double) { return 0.5; }};
    // x-dependent coefficients of the D^x terms and noise through D^x
    Set x_deriv{"x-dependent D^x terms", none,
                [](double x, double v) { return -v * (1.0 + 0.2 / (1.0 + x * x)); }, none, none,
                [](double x, double) { return 0.1 / (1.0 + x * x); },
                [](double, double) { return 1.0; }, none,
                [](double x, double) { return 0.3 * std::sqrt(1.0 + 1.0 / (1.0 + x * x)); }, none};
    Set full_rank{"full-rank diffusion (rejected)", none, [](double, double v) { return -v; }, none,
                  none, none,
                  [](double x, double v) { return 1.0 + 0.1 * std::sin(7.3 * x * v + 3.1 * x * x); },
                  none, none, [](double, double) { return 0.5; }};
    Set nonfinite{"non-finite diffusion (rejected)", none, [](double, double v) { return -v; }, none,
                  none, none, [](double x, double) { return x > 0 ? NAN : 1.0; }, none, none,
                  [](double, double) { return 0.5; }};

    for (int order = 1; order <= 3; ++order) {
        run(constant, 24, 20, order, true);
        run(constant, 17, 33, order, true);
        run(paper_var, 24, 20, order, true);
        run(paper_var, 41, 9, order, true);
        run(general_v, 24, 20, order, true);
    }
    run(xv, 24, 20, 1, true);
    run(xv, 24, 20, 2, true);
    run(xv, 24, 20, 3, false);
    for (int order = 1; order <= 3; ++order) run(with_gxx, 24, 20, order, true);
    run(x_deriv, 24, 20, 1, true);
    run(x_deriv, 24, 20, 2, true);
    run(x_deriv, 24, 20, 3, false);   // three x derivatives in [[B,A],A]
    run(full_rank, 24, 20, 2, false);
    run(nonfinite, 24, 20, 2, false);
    // degenerate grids
    run(constant, 1, 1, 3, true);
    run(paper_var, 2, 3, 3, true);
    std::printf(failures ? "FAILED %d\n" : "ok\n", failures);
    return failures ? 1 : 0;
}
