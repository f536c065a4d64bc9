// Host construction of the Magnus basis in factored (Kronecker) form.
//
// Section 2 ("Computation of A and B") builds, for coefficients sampled on the
// grid, B = diag(vec H) + diag(vec F^x)(I (x) D^x) + diag(vec F^v)(D^v (x) I)
//         + 1/2 diag(vec G^xx)(I (x) D^xx) + diag(vec G^xv)(D^v (x) D^x)
//         + 1/2 diag(vec G^vv)(D^vv (x) I)
//       A = diag(vec Sigma) + diag(vec Sigma^x)(I (x) D^x) + diag(vec Sigma^v)(D^v (x) I).
// When every coefficient depends on v only, diag(vec Z) = diag(z(v)) (x) I, so
// with G^xx = Sigma^x = 0 both are sums V_0 (x) I + V_1 (x) D^x with banded
// nv x nv factors V_q.  Products of such sums are again sums over powers of
// D^x ((V (x) D^p)(W (x) D^q) = VW (x) D^{p+q}), so A^2 and the commutators of
// eq. (MagnusFormulas) are formed exactly, as products of the truncated
// matrices, by 1-D banded products.  Powers of D^x up to 2 occur.
//
// Coefficients of the terms without an x derivative (H, F^v, G^vv in B;
// Sigma, Sigma^v in A) may also depend on x.  Such a coefficient grid z(x, v)
// is written exactly (to rounding) as a short sum sum_t b_t(v) a_t(x) by a
// cross decomposition with complete pivoting, so diag(vec Z) = sum_t
// diag(b_t) (x) diag(a_t): the operators gain terms W (x) diag(a) next to the
// V_q (x) D^q terms.  Where D^x meets such a factor once in a product (the
// commutators of eq. (MagnusFormulas) with x-dependent noise through d/dv,
// as in eq. (coeffsLangevinVar)), the x part is a chain
// diag(alpha) D^x diag(beta) (one of alpha, beta may be the unit vector):
// the operators gain terms C (x) diag(alpha) D^x diag(beta).  Products that
// would need a second D^x on a chain, or a chain times a chain, are reported
// as unsupported.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mg_internal.h"

namespace {

// Square band matrix: entry (i, j) for |i - j| <= r stored at a[i*(2r+1) + (j-i+r)].
struct Band {
    int n = 0, r = 0;
    std::vector<double> a;
    Band() = default;
    Band(int n_, int r_) : n(n_), r(r_), a((size_t)n_ * (2 * r_ + 1), 0.0) {}
    double get(int i, int j) const {
        int o = j - i;
        if (o < -r || o > r || j < 0 || j >= n) return 0.0;
        return a[(size_t)i * (2 * r + 1) + (o + r)];
    }
    void set(int i, int j, double v) { a[(size_t)i * (2 * r + 1) + (j - i + r)] = v; }
};

Band band_zero(int n) { return Band(n, 0); }

Band band_mul(const Band& A, const Band& B) {
    Band C(A.n, A.r + B.r);
    for (int i = 0; i < A.n; ++i)
        for (int k = std::max(0, i - A.r); k <= std::min(A.n - 1, i + A.r); ++k) {
            double aik = A.get(i, k);
            if (aik == 0.0) continue;
            for (int j = std::max(0, k - B.r); j <= std::min(B.n - 1, k + B.r); ++j) {
                double bkj = B.get(k, j);
                if (bkj != 0.0) C.set(i, j, C.get(i, j) + aik * bkj);
            }
        }
    return C;
}

Band band_axpby(double alpha, const Band& A, double beta, const Band& B) {
    Band C(A.n, std::max(A.r, B.r));
    for (int i = 0; i < A.n; ++i)
        for (int j = std::max(0, i - C.r); j <= std::min(A.n - 1, i + C.r); ++j)
            C.set(i, j, alpha * A.get(i, j) + beta * B.get(i, j));
    return C;
}

Band band_diag(const std::vector<double>& d) {
    Band D((int)d.size(), 0);
    for (int i = 0; i < (int)d.size(); ++i) D.set(i, i, d[i]);
    return D;
}

// (1/(2 d)) tridiag(-1, 0, 1) and (1/d^2) tridiag(1, -2, 1), zero boundary values.
Band first_difference(int n, double d) {
    Band D(n, 1);
    for (int i = 0; i < n; ++i) {
        if (i > 0) D.set(i, i - 1, -1.0 / (2.0 * d));
        if (i + 1 < n) D.set(i, i + 1, 1.0 / (2.0 * d));
    }
    return D;
}
Band second_difference(int n, double d) {
    Band D(n, 1);
    for (int i = 0; i < n; ++i) {
        if (i > 0) D.set(i, i - 1, 1.0 / (d * d));
        D.set(i, i, -2.0 / (d * d));
        if (i + 1 < n) D.set(i, i + 1, 1.0 / (d * d));
    }
    return D;
}

bool band_is_zero(const Band& B) {
    return std::all_of(B.a.begin(), B.a.end(), [](double v) { return v == 0.0; });
}

// Registry of the x vectors of diagonal x-factors diag(a); equal vectors share
// one entry, so products of factors can be matched exactly.
struct XReg {
    std::vector<std::vector<double>> vecs;
    int find_or_add(const std::vector<double>& a) {
        for (size_t k = 0; k < vecs.size(); ++k)
            if (vecs[k] == a) return (int)k;
        vecs.push_back(a);
        return (int)vecs.size() - 1;
    }
};

// sum_{q=0..2} V[q] (x) (D^x)^q + sum_k W[k] (x) diag(xreg.vecs[id[k]])
//   + sum_k C[k] (x) diag(a_k) D^x diag(b_k)   (a_k = vecs[ca[k]], b_k =
//   vecs[cb[k]], index -1: the unit vector)
struct KOp {
    Band V[3];
    std::vector<Band> W;
    std::vector<int> id;
    std::vector<Band> C;
    std::vector<int> ca, cb;
    explicit KOp(int nv) { for (auto& b : V) b = band_zero(nv); }
    void add_w(int xid, const Band& B) {
        for (size_t k = 0; k < id.size(); ++k)
            if (id[k] == xid) {
                W[k] = band_axpby(1.0, W[k], 1.0, B);
                return;
            }
        id.push_back(xid);
        W.push_back(B);
    }
    void add_c(int ia, int ib, const Band& B) {
        for (size_t k = 0; k < ca.size(); ++k)
            if (ca[k] == ia && cb[k] == ib) {
                C[k] = band_axpby(1.0, C[k], 1.0, B);
                return;
            }
        ca.push_back(ia);
        cb.push_back(ib);
        C.push_back(B);
    }
};

// registry id of the pointwise product of two x vectors (-1: unit)
int xmul(XReg& xr, int ia, int ib) {
    if (ia < 0) return ib;
    if (ib < 0) return ia;
    const std::vector<double>& a = xr.vecs[ia];
    const std::vector<double>& b = xr.vecs[ib];
    std::vector<double> ab(a.size());
    for (size_t i = 0; i < a.size(); ++i) ab[i] = a[i] * b[i];
    return xr.find_or_add(ab);
}

// Product of two factored operators; false (with a reason) when a power of
// D^x meets a non-constant diagonal x-factor, which this form cannot hold.
bool kop_mul(const KOp& X, const KOp& Y, XReg& xr, KOp& out, std::string& why) {
    int nv = X.V[0].n;
    KOp Z(nv);
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            if (band_is_zero(X.V[p]) || band_is_zero(Y.V[q])) continue;
            Band P = band_mul(X.V[p], Y.V[q]);
            if (band_is_zero(P)) continue;
            if (p + q > 2) { why = "x-derivative power above 2 in the Magnus basis"; return false; }
            Z.V[p + q] = band_axpby(1.0, Z.V[p + q], 1.0, P);
        }
    const char* deep = "an x derivative meets an x-dependent coefficient more than once in the "
                       "Magnus basis (order 3 with x-dependent noise)";
    // (V (x) D^p)(W (x) diag(a)): diag for p = 0, the chain D diag(a) for p = 1
    for (size_t k = 0; k < Y.W.size(); ++k)
        for (int p = 0; p < 3; ++p) {
            if (band_is_zero(X.V[p]) || band_is_zero(Y.W[k])) continue;
            Band P = band_mul(X.V[p], Y.W[k]);
            if (band_is_zero(P)) continue;
            if (p > 1) { why = deep; return false; }
            if (p == 0) Z.add_w(Y.id[k], P);
            else Z.add_c(-1, Y.id[k], P);
        }
    // (V (x) D^p) chain: only p = 0
    for (size_t k = 0; k < Y.C.size(); ++k)
        for (int p = 0; p < 3; ++p) {
            if (band_is_zero(X.V[p]) || band_is_zero(Y.C[k])) continue;
            Band P = band_mul(X.V[p], Y.C[k]);
            if (band_is_zero(P)) continue;
            if (p > 0) { why = deep; return false; }
            Z.add_c(Y.ca[k], Y.cb[k], P);
        }
    // chain (V (x) D^q): only q = 0; chain (W (x) diag(b)) = chain with beta b
    for (size_t k = 0; k < X.C.size(); ++k) {
        for (int q = 0; q < 3; ++q) {
            if (band_is_zero(X.C[k]) || band_is_zero(Y.V[q])) continue;
            Band P = band_mul(X.C[k], Y.V[q]);
            if (band_is_zero(P)) continue;
            if (q > 0) { why = deep; return false; }
            Z.add_c(X.ca[k], X.cb[k], P);
        }
        for (size_t m = 0; m < Y.W.size(); ++m) {
            if (band_is_zero(X.C[k]) || band_is_zero(Y.W[m])) continue;
            Band P = band_mul(X.C[k], Y.W[m]);
            if (band_is_zero(P)) continue;
            Z.add_c(X.ca[k], xmul(xr, X.cb[k], Y.id[m]), P);
        }
        for (size_t m = 0; m < Y.C.size(); ++m) {
            if (band_is_zero(X.C[k]) || band_is_zero(Y.C[m])) continue;
            if (band_is_zero(band_mul(X.C[k], Y.C[m]))) continue;
            why = deep;
            return false;
        }
    }
    for (size_t k = 0; k < X.W.size(); ++k) {
        // (W (x) diag(a))(V (x) D^q): diag for q = 0, the chain diag(a) D for q = 1
        for (int q = 0; q < 3; ++q) {
            if (band_is_zero(X.W[k]) || band_is_zero(Y.V[q])) continue;
            Band P = band_mul(X.W[k], Y.V[q]);
            if (band_is_zero(P)) continue;
            if (q > 1) { why = deep; return false; }
            if (q == 0) Z.add_w(X.id[k], P);
            else Z.add_c(X.id[k], -1, P);
        }
        // (W (x) diag(a)) chain = chain with alpha a * alpha
        for (size_t m = 0; m < Y.C.size(); ++m) {
            if (band_is_zero(X.W[k]) || band_is_zero(Y.C[m])) continue;
            Band P = band_mul(X.W[k], Y.C[m]);
            if (band_is_zero(P)) continue;
            Z.add_c(xmul(xr, X.id[k], Y.ca[m]), Y.cb[m], P);
        }
        for (size_t m = 0; m < Y.W.size(); ++m) {
            if (band_is_zero(X.W[k]) || band_is_zero(Y.W[m])) continue;
            Band P = band_mul(X.W[k], Y.W[m]);
            if (band_is_zero(P)) continue;
            const std::vector<double>& a = xr.vecs[X.id[k]];
            const std::vector<double>& b = xr.vecs[Y.id[m]];
            std::vector<double> ab(a.size());
            for (size_t i = 0; i < a.size(); ++i) ab[i] = a[i] * b[i];
            Z.add_w(xr.find_or_add(ab), P);
        }
    }
    out = Z;
    return true;
}

bool kop_comm(const KOp& X, const KOp& Y, XReg& xr, KOp& out, std::string& why) {
    const int nv = X.V[0].n;
    KOp XY(nv), YX(nv);
    if (!kop_mul(X, Y, xr, XY, why) || !kop_mul(Y, X, xr, YX, why)) return false;
    KOp Z(nv);
    for (int q = 0; q < 3; ++q) Z.V[q] = band_axpby(1.0, XY.V[q], -1.0, YX.V[q]);
    for (size_t k = 0; k < XY.W.size(); ++k) Z.add_w(XY.id[k], XY.W[k]);
    for (size_t k = 0; k < YX.W.size(); ++k) Z.add_w(YX.id[k], band_axpby(-1.0, YX.W[k], 0.0, YX.W[k]));
    for (size_t k = 0; k < XY.C.size(); ++k) Z.add_c(XY.ca[k], XY.cb[k], XY.C[k]);
    for (size_t k = 0; k < YX.C.size(); ++k)
        Z.add_c(YX.ca[k], YX.cb[k], band_axpby(-1.0, YX.C[k], 0.0, YX.C[k]));
    out = Z;
    return true;
}

// Exact low-rank form of a coefficient grid z[j][i] (v row j, x column i):
// z = sum_t b_t(v) a_t(x), by cross approximation with complete pivoting
// (Gaussian elimination on the residual, largest entry first), stopped when
// the residual is below 1e-14 of max|z| (the rounding level of the operator).
// For the smooth coefficients of the workloads the rank is the number of
// separable terms of the formula.  The x vectors are scaled to a largest
// entry of 1.
bool low_rank(const double* z, int nx, int nv, int max_rank, std::vector<std::vector<double>>& bs,
              std::vector<std::vector<double>>& as) {
    std::vector<double> R(z, z + (size_t)nx * nv);
    double zmax = 0.0;
    for (double v : R) zmax = std::max(zmax, std::fabs(v));
    bs.clear();
    as.clear();
    if (zmax == 0.0) return true;
    for (int t = 0; t <= max_rank; ++t) {
        size_t piv = 0;
        double pmax = 0.0;
        for (size_t k = 0; k < R.size(); ++k)
            if (std::fabs(R[k]) > pmax) { pmax = std::fabs(R[k]); piv = k; }
        if (pmax <= 1e-14 * zmax) return true;
        if (t == max_rank) return false;
        const int jp = (int)(piv / nx), ip = (int)(piv % nx);
        std::vector<double> a(nx), b(nv);
        double amax = 0.0;
        for (int i = 0; i < nx; ++i) { a[i] = R[(size_t)jp * nx + i]; amax = std::max(amax, std::fabs(a[i])); }
        const double sa = 1.0 / amax;
        for (int i = 0; i < nx; ++i) a[i] *= sa;
        // b_j = R[j][ip] / a[ip] so that b a^T reproduces row jp and column ip
        for (int j = 0; j < nv; ++j) b[j] = R[(size_t)j * nx + ip] / a[ip];
        for (int j = 0; j < nv; ++j)
            for (int i = 0; i < nx; ++i) R[(size_t)j * nx + i] -= b[j] * a[i];
        bs.push_back(b);
        as.push_back(a);
    }
    return false;
}

// Coefficient that must depend on v only: returns per-row values or fails.
bool v_only(const double* c, int nx, int nv, std::vector<double>& out, bool& nonzero) {
    out.assign(nv, 0.0);
    nonzero = false;
    if (!c) return true;
    for (int j = 0; j < nv; ++j) {
        double v = c[(size_t)j * nx];
        for (int i = 1; i < nx; ++i)
            if (c[(size_t)j * nx + i] != v) return false;
        if (!std::isfinite(v)) return false;
        out[j] = v;
        if (v != 0.0) nonzero = true;
    }
    return true;
}

bool all_zero(const double* c, size_t n) {
    if (!c) return true;
    for (size_t i = 0; i < n; ++i)
        if (c[i] != 0.0) return false;
    return true;
}

}  // namespace

mg_status mg_build_host(const mg_grid* g, const mg_coeffs* cf, int order, mg_ops* ops) {
    const int nx = g->nx, nv = g->nv;
    const size_t N = (size_t)nx * nv;
    if (!all_zero(cf->gxx, N) || !all_zero(cf->sx, N))
        return mg_fail(MG_EUNSUPPORTED, "g^xx and sigma^x must be zero in this build");
    // Coefficients of the D^x terms must depend on v only; the others may
    // depend on x through the low-rank form.
    enum { H, FX, FV, GXV, GVV, SIG, SV, NCOEF };
    const double* fields[NCOEF] = {cf->h, cf->fx, cf->fv, cf->gxv, cf->gvv, cf->sig, cf->sv};
    const char* names[NCOEF] = {"h", "fx", "fv", "gxv", "gvv", "sig", "sv"};
    const bool x_allowed[NCOEF] = {true, false, true, false, true, true, true};
    std::vector<double> c[NCOEF];                 // v-only part of each coefficient
    std::vector<std::vector<double>> xb[NCOEF];  // x-dependent terms: b_t(v) ...
    std::vector<int> xid[NCOEF];                 // ... times diag(a_t), registry ids
    XReg xr;
    for (int t = 0; t < NCOEF; ++t) {
        bool nz;
        if (v_only(fields[t], nx, nv, c[t], nz)) continue;
        if (!x_allowed[t])
            return mg_fail(MG_EUNSUPPORTED, std::string("coefficient ") + names[t] +
                                                " multiplies an x derivative and must be finite "
                                                "and depend on v only in this build");
        for (size_t k = 0; k < N; ++k)
            if (!std::isfinite(fields[t][k]))
                return mg_fail(MG_EINVAL, std::string("coefficient ") + names[t] + " is not finite");
        std::vector<std::vector<double>> bs, as;
        if (!low_rank(fields[t], nx, nv, MG_MAX_XDIAG, bs, as))
            return mg_fail(MG_EUNSUPPORTED, std::string("coefficient ") + names[t] +
                                                " is not a sum of at most 4 products b(v) a(x)");
        c[t].assign(nv, 0.0);
        for (size_t r = 0; r < bs.size(); ++r) {
            const std::vector<double>& a = as[r];
            bool constant = std::all_of(a.begin(), a.end(), [&](double v) { return v == a[0]; });
            if (constant) {
                for (int j = 0; j < nv; ++j) c[t][j] += bs[r][j] * a[0];
            } else {
                xb[t].push_back(bs[r]);
                xid[t].push_back(xr.find_or_add(a));
            }
        }
    }
    const double dx = (g->bx - g->ax) / (nx + 1), dv = (g->bv - g->av) / (nv + 1);
    Band Dv = first_difference(nv, dv), Dvv = second_difference(nv, dv);

    // B = V_0 (x) I + V_1 (x) D^x + sum W (x) diag(a)
    KOp B(nv), A(nv);
    B.V[0] = band_axpby(1.0, band_diag(c[H]), 1.0, band_mul(band_diag(c[FV]), Dv));
    B.V[0] = band_axpby(1.0, B.V[0], 0.5, band_mul(band_diag(c[GVV]), Dvv));
    B.V[1] = band_axpby(1.0, band_diag(c[FX]), 1.0, band_mul(band_diag(c[GXV]), Dv));
    for (size_t r = 0; r < xb[H].size(); ++r) B.add_w(xid[H][r], band_diag(xb[H][r]));
    for (size_t r = 0; r < xb[FV].size(); ++r) B.add_w(xid[FV][r], band_mul(band_diag(xb[FV][r]), Dv));
    for (size_t r = 0; r < xb[GVV].size(); ++r)
        B.add_w(xid[GVV][r], band_axpby(0.5, band_mul(band_diag(xb[GVV][r]), Dvv), 0.0, Dvv));
    // A = V_0 (x) I + sum W (x) diag(a)
    A.V[0] = band_axpby(1.0, band_diag(c[SIG]), 1.0, band_mul(band_diag(c[SV]), Dv));
    for (size_t r = 0; r < xb[SIG].size(); ++r) A.add_w(xid[SIG][r], band_diag(xb[SIG][r]));
    for (size_t r = 0; r < xb[SV].size(); ++r) A.add_w(xid[SV][r], band_mul(band_diag(xb[SV][r]), Dv));

    const int nact = order == 1 ? 2 : (order == 2 ? 4 : 6);
    KOp M[MG_NBASIS] = {B, A, KOp(nv), KOp(nv), KOp(nv), KOp(nv)};
    std::string why;
    bool ok = true;
    // only the matrices the order uses have to exist in this form
    if (nact > 2) ok = ok && kop_mul(A, A, xr, M[2], why) && kop_comm(B, A, xr, M[3], why);
    if (nact > 4) ok = ok && kop_comm(M[3], A, xr, M[4], why) && kop_comm(M[3], B, xr, M[5], why);
    if (!ok) return mg_fail(MG_EUNSUPPORTED, why);

    // Band radii actually used, after dropping cancellation residues.  A
    // factor V_q multiplies (D^x)^q, whose norm is about (1/dx)^q, and a factor
    // W multiplies diag(a), whose norm is max|a|, so entries are compared with
    // the whole matrix through these weights: entries below 1e-14 of the
    // largest weighted entry of the same basis matrix are zero in exact
    // arithmetic and stem from rounding in the products (a factor can consist
    // of residues only, e.g. the D^x part of [[B,A],B] for the
    // constant-coefficient operator).
    int R[3] = {0, 0, 0}, RW = 0;
    const double wq[3] = {1.0, 1.0 / dx, 1.0 / (dx * dx)};
    std::vector<double> wa(xr.vecs.size());
    for (size_t k = 0; k < xr.vecs.size(); ++k) {
        double m = 0.0;
        for (double v : xr.vecs[k]) m = std::max(m, std::fabs(v));
        wa[k] = m;
    }
    std::vector<int> used(xr.vecs.size(), 0);
    // chain terms: weight max|alpha| max|beta| / dx, and the distinct chains
    // the active matrices use
    auto xmax = [&](int id) { return id < 0 ? 1.0 : wa[id]; };
    std::vector<std::pair<int, int>> chains;
    auto chain_slot = [&](int ia, int ib) {
        for (size_t c = 0; c < chains.size(); ++c)
            if (chains[c].first == ia && chains[c].second == ib) return (int)c;
        chains.push_back({ia, ib});
        return (int)chains.size() - 1;
    };
    int RC = 0;
    for (int l = 0; l < MG_NBASIS; ++l) {
        double mx = 0.0;
        for (int q = 0; q < 3; ++q)
            for (double v : M[l].V[q].a) mx = std::max(mx, std::fabs(v) * wq[q]);
        for (size_t k = 0; k < M[l].W.size(); ++k)
            for (double v : M[l].W[k].a) mx = std::max(mx, std::fabs(v) * wa[M[l].id[k]]);
        for (size_t k = 0; k < M[l].C.size(); ++k) {
            const double wc = xmax(M[l].ca[k]) * xmax(M[l].cb[k]) / dx;
            for (double v : M[l].C[k].a) mx = std::max(mx, std::fabs(v) * wc);
        }
        for (size_t k = 0; k < M[l].C.size(); ++k) {
            Band& C = M[l].C[k];
            const double wc = xmax(M[l].ca[k]) * xmax(M[l].cb[k]) / dx;
            for (double& v : C.a)
                if (std::fabs(v) * wc <= 1e-14 * mx) v = 0.0;
            if (l >= nact || band_is_zero(C)) continue;
            for (int i = 0; i < nv; ++i)
                for (int o = -C.r; o <= C.r; ++o)
                    if (C.get(i, i + o) != 0.0) RC = std::max(RC, std::abs(o));
            chain_slot(M[l].ca[k], M[l].cb[k]);
        }
        for (int q = 0; q < 3; ++q) {
            Band& V = M[l].V[q];
            for (double& v : V.a)
                if (std::fabs(v) * wq[q] <= 1e-14 * mx) v = 0.0;
            if (l >= nact) continue;
            for (int i = 0; i < nv; ++i)
                for (int o = -V.r; o <= V.r; ++o)
                    if (V.get(i, i + o) != 0.0) R[q] = std::max(R[q], std::abs(o));
        }
        for (size_t k = 0; k < M[l].W.size(); ++k) {
            Band& W = M[l].W[k];
            for (double& v : W.a)
                if (std::fabs(v) * wa[M[l].id[k]] <= 1e-14 * mx) v = 0.0;
            if (l >= nact) continue;
            for (int i = 0; i < nv; ++i)
                for (int o = -W.r; o <= W.r; ++o)
                    if (W.get(i, i + o) != 0.0) {
                        RW = std::max(RW, std::abs(o));
                        used[M[l].id[k]] = 1;
                    }
        }
    }
    // diagonal x-factors in use, numbered 0 .. nd-1 in registry order
    std::vector<int> slot(xr.vecs.size(), -1);
    int nd = 0;
    for (size_t k = 0; k < xr.vecs.size(); ++k)
        if (used[k]) slot[k] = nd++;
    if (nd > MG_MAX_XDIAG)
        return mg_fail(MG_EUNSUPPORTED, "more than 4 x-dependent factors in the Magnus basis");
    if (RW > MG_XDIAG_RADIUS)
        return mg_fail(MG_EUNSUPPORTED, "band radius of an x-dependent factor above 2");
    if ((int)chains.size() > MG_MAX_XCHAIN)
        return mg_fail(MG_EUNSUPPORTED, "more than 2 chains diag(a) D^x diag(b) in the Magnus basis");
    if (RC > MG_XDIAG_RADIUS)
        return mg_fail(MG_EUNSUPPORTED, "band radius of a chain factor above 2");
    // highest power of D^x with a non-zero factor among the active matrices
    int qmax = 0;
    for (int l = 0; l < nact; ++l)
        for (int q = 1; q < 3; ++q)
            for (double v : M[l].V[q].a)
                if (v != 0.0) qmax = std::max(qmax, q);
    // Round the radii up to one of the band shapes the kernels are built for;
    // the padding entries are zeros.
    static const int kShapes[4][4] = {{1, 0, 0, 1}, {2, 1, 0, 1}, {2, 1, 1, 2}, {3, 3, 3, 2}};
    int shape = -1;
    for (int k = 0; k < 4 && shape < 0; ++k)
        if (R[0] <= kShapes[k][0] && R[1] <= kShapes[k][1] && R[2] <= kShapes[k][2] &&
            qmax <= kShapes[k][3])
            shape = k;
    if (shape < 0) return mg_fail(MG_EUNSUPPORTED, "Magnus basis band radius above 3");
    if (!chains.empty()) shape = std::max(shape, 1);   // built for the order-2 band shape
    if ((nd > 0 || !chains.empty()) && shape > 1)
        return mg_fail(MG_EUNSUPPORTED,
                       "x-dependent coefficients are built for band shapes up to (2,1,0) in this build");
    for (int q = 0; q < 3; ++q) R[q] = kShapes[shape][q];
    ops->qmax = kShapes[shape][3];

    ops->grid = *g;
    ops->order = order;
    ops->nactive = nact;
    for (int q = 0; q < 3; ++q) ops->R[q] = R[q];
    // x-dependent factors: the kernels are built for 3 and for 4 factors
    // (unused ones are zero; the variable-coefficient workloads use 3), and
    // with chains for 4 factors and 2 chains
    ops->NC = chains.empty() ? 0 : MG_MAX_XCHAIN;
    ops->ND = nd > 0 || ops->NC > 0 ? (nd <= 3 && ops->NC == 0 ? 3 : MG_MAX_XDIAG) : 0;
    ops->RW = ops->ND > 0 ? MG_XDIAG_RADIUS : 0;
    // V2 (the Dt^2 factor) has entries in the row only where Dt^2 occurs
    const int nq = ops->qmax >= 2 ? 3 : 2;
    ops->NB = (2 * R[0] + 1) + (2 * R[1] + 1) + (nq == 3 ? 2 * R[2] + 1 : 0) +
              ops->ND * (2 * ops->RW + 1);
    ops->NBP = (ops->NB + 1) & ~1;
    ops->xdiag_host.assign((size_t)ops->ND * nx, 0.0);
    ops->xstat_host.assign((size_t)ops->ND * 4, 0.0);
    for (size_t k = 0; k < xr.vecs.size(); ++k) {
        if (slot[k] < 0) continue;
        const std::vector<double>& a = xr.vecs[k];
        double sum = 0.0, lo = a[0], hi = a[0];
        for (int i = 0; i < nx; ++i) {
            ops->xdiag_host[(size_t)slot[k] * nx + i] = a[i];
            sum += a[i];
            lo = std::min(lo, a[i]);
            hi = std::max(hi, a[i]);
        }
        double* st = ops->xstat_host.data() + (size_t)slot[k] * 4;
        st[0] = sum;                 // for the trace
        st[1] = 0.5 * (hi + lo);     // midpoint and half-width of the values,
        st[2] = 0.5 * (hi - lo);     // for the 1-norm bound
    }
    // chain vectors alpha_c, beta_c [NC][2][nx] and per chain {max|alpha| max|beta|, 0, 0, 0}
    ops->xchain_host.assign((size_t)ops->NC * 2 * nx, 0.0);
    ops->cstat_host.assign((size_t)ops->NC * 4, 0.0);
    for (size_t c = 0; c < chains.size(); ++c) {
        const int ids[2] = {chains[c].first, chains[c].second};
        double mx[2] = {0.0, 0.0};
        for (int h = 0; h < 2; ++h)
            for (int i = 0; i < nx; ++i) {
                const double v = ids[h] < 0 ? 1.0 : xr.vecs[ids[h]][i];
                ops->xchain_host[(c * 2 + h) * nx + i] = v;
                mx[h] = std::max(mx[h], std::fabs(v));
            }
        ops->cstat_host[c * 4] = mx[0] * mx[1];
    }
    // table rows are padded to the rows the kernel shape covers
    int rows = resident_rows(nx, nv);
    if (rows == 0) rows = coop_table_rows(nx, nv);
    ops->nv_pad = std::max(nv, rows);
    // main rows [6][nv_pad][NBP], then the chain section [6][nv_pad][NCB]
    ops->NCB = ops->NC * (2 * MG_XDIAG_RADIUS + 1);
    ops->basis_host.assign((size_t)MG_NBASIS * ops->nv_pad * (ops->NBP + ops->NCB), 0.0);
    const double fold[3] = {1.0, 1.0 / (2.0 * dx), 1.0 / (4.0 * dx * dx)};
    for (int l = 0; l < MG_NBASIS; ++l)
        for (int j = 0; j < nv; ++j) {
            double* row = ops->basis_host.data() + ((size_t)l * ops->nv_pad + j) * ops->NBP;
            int off = 0;
            for (int q = 0; q < nq; ++q) {
                for (int o = -R[q]; o <= R[q]; ++o) row[off + o + R[q]] = M[l].V[q].get(j, j + o) * fold[q];
                off += 2 * R[q] + 1;
            }
            for (size_t k = 0; k < M[l].W.size(); ++k) {
                const int sl = slot[M[l].id[k]];
                if (sl < 0) continue;
                double* w = row + off + sl * (2 * ops->RW + 1);
                for (int o = -ops->RW; o <= ops->RW; ++o) w[o + ops->RW] = M[l].W[k].get(j, j + o);
            }
            // chain bands, with the 1/(2 dx) of D^x folded in
            double* crow = ops->basis_host.data() + (size_t)MG_NBASIS * ops->nv_pad * ops->NBP +
                           ((size_t)l * ops->nv_pad + j) * ops->NCB;
            for (size_t k = 0; k < M[l].C.size(); ++k) {
                if (band_is_zero(M[l].C[k])) continue;
                int sl = -1;
                for (size_t c = 0; c < chains.size(); ++c)
                    if (chains[c].first == M[l].ca[k] && chains[c].second == M[l].cb[k]) sl = (int)c;
                if (sl < 0) continue;   // only in matrices the order does not use
                double* w = crow + sl * (2 * MG_XDIAG_RADIUS + 1);
                for (int o = -MG_XDIAG_RADIUS; o <= MG_XDIAG_RADIUS; ++o)
                    w[o + MG_XDIAG_RADIUS] = M[l].C[k].get(j, j + o) / (2.0 * dx);
            }
        }
    return MG_OK;
}
