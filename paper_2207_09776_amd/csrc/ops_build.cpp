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
// diag(b_t) (x) diag(a_t).  Every operator is then a sum of terms V (x) X
// with X a word diag(x_0) D^x diag(x_1) ... D^x diag(x_d) in the x vectors
// (the unit vector included) and D^x; a product of two terms is the product
// of the V factors times the concatenated word, whose two middle vectors
// merge into their pointwise product: again exact, as products of the
// truncated matrices.  Words of depth up to 2 occur at order 3 of
// eq. (coeffsLangevinVar) (x-dependent noise through d/dv meets -v d/dx twice
// in [[B,A],B]); deeper words are reported as unsupported.  The kernels take
// words with unit vectors only (powers of D^x) as the V_q tables, depth-0
// words as diagonal x-factors, and the others as x-terms.

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

// An x word diag(x_0) L_1 diag(x_1) ... L_d diag(x_d), d <= 2, whose letters
// L_h are Dt = tridiag(-1, 0, 1) (D^x without its 1/(2 dx)) or
// Dxx = tridiag(1, -2, 1) (D^xx without its 1/dx^2); x_h is a registry id,
// -1 for the unit vector.
struct XWord {
    int d = 0;
    int id[3] = {-1, -1, -1};
    int lt[2] = {0, 0};   // letter h+1: 0 Dt, 1 Dxx
    bool unit() const {
        for (int h = 0; h <= d; ++h)
            if (id[h] >= 0) return false;
        return true;
    }
    // a power of Dt (the V_q tables)
    bool plain() const {
        for (int h = 0; h < d; ++h)
            if (lt[h] != 0) return false;
        return unit();
    }
    bool operator==(const XWord& o) const {
        if (d != o.d) return false;
        for (int h = 0; h <= d; ++h)
            if (id[h] != o.id[h]) return false;
        for (int h = 0; h < d; ++h)
            if (lt[h] != o.lt[h]) return false;
        return true;
    }
    // the factor of the raw letters: (1/(2 dx)) per Dt, 1/dx^2 per Dxx
    double fold(double dx) const {
        double f = 1.0;
        for (int h = 0; h < d; ++h) f *= lt[h] ? 1.0 / (dx * dx) : 1.0 / (2.0 * dx);
        return f;
    }
};

// sum_k V[k] (x) X_k over distinct words X_k
struct KOp {
    int nv;
    std::vector<XWord> w;
    std::vector<Band> V;
    explicit KOp(int nv_) : nv(nv_) {}
    void add(const XWord& x, const Band& B) {
        for (size_t k = 0; k < w.size(); ++k)
            if (w[k] == x) {
                V[k] = band_axpby(1.0, V[k], 1.0, B);
                return;
            }
        w.push_back(x);
        V.push_back(B);
    }
    void add_q(int q, const Band& B) {   // B (x) Dt^q
        XWord x;
        x.d = q;
        add(x, B);
    }
    void add_w(int xid, const Band& B) {   // B (x) diag(x vector xid)
        XWord x;
        x.id[0] = xid;
        add(x, B);
    }
    void add_x(int xid, int letter, const Band& B) {   // B (x) diag(x vector xid) L
        XWord x;
        x.d = 1;
        x.id[0] = xid;
        x.lt[0] = letter;
        add(x, B);
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

// Product of two factored operators; false (with a reason) when a word would
// exceed depth 2.
bool kop_mul(const KOp& X, const KOp& Y, XReg& xr, KOp& out, std::string& why) {
    KOp Z(X.nv);
    for (size_t s = 0; s < X.w.size(); ++s)
        for (size_t t = 0; t < Y.w.size(); ++t) {
            if (band_is_zero(X.V[s]) || band_is_zero(Y.V[t])) continue;
            Band P = band_mul(X.V[s], Y.V[t]);
            if (band_is_zero(P)) continue;
            const XWord& a = X.w[s];
            const XWord& b = Y.w[t];
            if (a.d + b.d > 2) {
                why = a.plain() && b.plain()
                          ? "x-derivative power above 2 in the Magnus basis"
                          : "x derivatives and x-dependent coefficients meet more than twice in a "
                            "product of the Magnus basis";
                return false;
            }
            XWord c;
            c.d = a.d + b.d;
            for (int h = 0; h < a.d; ++h) c.id[h] = a.id[h];
            c.id[a.d] = xmul(xr, a.id[a.d], b.id[0]);
            for (int h = 1; h <= b.d; ++h) c.id[a.d + h] = b.id[h];
            for (int h = 0; h < a.d; ++h) c.lt[h] = a.lt[h];
            for (int h = 0; h < b.d; ++h) c.lt[a.d + h] = b.lt[h];
            Z.add(c, P);
        }
    out = Z;
    return true;
}

bool kop_comm(const KOp& X, const KOp& Y, XReg& xr, KOp& out, std::string& why) {
    KOp XY(X.nv), YX(X.nv);
    if (!kop_mul(X, Y, xr, XY, why) || !kop_mul(Y, X, xr, YX, why)) return false;
    KOp Z(X.nv);
    for (size_t k = 0; k < XY.w.size(); ++k) Z.add(XY.w[k], XY.V[k]);
    for (size_t k = 0; k < YX.w.size(); ++k) Z.add(YX.w[k], band_axpby(-1.0, YX.V[k], 0.0, YX.V[k]));
    out = Z;
    return true;
}

// The x word as an nx x nx band matrix (raw letters), for the 1-norm and the
// trace of an x-term.
Band word_matrix(const XWord& x, const XReg& xr, int nx) {
    auto vec = [&](int id) {
        return id < 0 ? std::vector<double>((size_t)nx, 1.0) : xr.vecs[id];
    };
    Band L[2] = {Band(nx, 1), Band(nx, 1)};
    for (int i = 0; i < nx; ++i) {
        if (i > 0) { L[0].set(i, i - 1, -1.0); L[1].set(i, i - 1, 1.0); }
        if (i + 1 < nx) { L[0].set(i, i + 1, 1.0); L[1].set(i, i + 1, 1.0); }
        L[1].set(i, i, -2.0);
    }
    Band M = band_diag(vec(x.id[0]));
    for (int h = 1; h <= x.d; ++h) M = band_mul(band_mul(M, L[x.lt[h - 1]]), band_diag(vec(x.id[h])));
    return M;
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
    // Every coefficient may depend on x through the low-rank form.
    enum { H, FX, FV, GXX, GXV, GVV, SIG, SX, SV, NCOEF };
    const double* fields[NCOEF] = {cf->h,   cf->fx,  cf->fv, cf->gxx, cf->gxv,
                                   cf->gvv, cf->sig, cf->sx, cf->sv};
    const char* names[NCOEF] = {"h", "fx", "fv", "gxx", "gxv", "gvv", "sig", "sx", "sv"};
    (void)N;
    std::vector<double> c[NCOEF];                 // v-only part of each coefficient
    std::vector<std::vector<double>> xb[NCOEF];  // x-dependent terms: b_t(v) ...
    std::vector<int> xid[NCOEF];                 // ... times diag(a_t), registry ids
    XReg xr;
    for (int t = 0; t < NCOEF; ++t) {
        bool nz;
        if (v_only(fields[t], nx, nv, c[t], nz)) continue;
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
    Band b0 = band_axpby(1.0, band_diag(c[H]), 1.0, band_mul(band_diag(c[FV]), Dv));
    b0 = band_axpby(1.0, b0, 0.5, band_mul(band_diag(c[GVV]), Dvv));
    B.add_q(0, b0);
    B.add_q(1, band_axpby(1.0, band_diag(c[FX]), 1.0, band_mul(band_diag(c[GXV]), Dv)));
    for (size_t r = 0; r < xb[H].size(); ++r) B.add_w(xid[H][r], band_diag(xb[H][r]));
    for (size_t r = 0; r < xb[FV].size(); ++r) B.add_w(xid[FV][r], band_mul(band_diag(xb[FV][r]), Dv));
    for (size_t r = 0; r < xb[GVV].size(); ++r)
        B.add_w(xid[GVV][r], band_axpby(0.5, band_mul(band_diag(xb[GVV][r]), Dvv), 0.0, Dvv));
    // terms with an x derivative and x-dependent coefficients: words
    // diag(a) Dt, and the second difference D^xx as the letter Dxx
    for (size_t r = 0; r < xb[FX].size(); ++r) B.add_x(xid[FX][r], 0, band_diag(xb[FX][r]));
    for (size_t r = 0; r < xb[GXV].size(); ++r)
        B.add_x(xid[GXV][r], 0, band_mul(band_diag(xb[GXV][r]), Dv));
    if (!std::all_of(c[GXX].begin(), c[GXX].end(), [](double v) { return v == 0.0; }))
        B.add_x(-1, 1, band_axpby(0.5, band_diag(c[GXX]), 0.0, band_diag(c[GXX])));
    for (size_t r = 0; r < xb[GXX].size(); ++r)
        B.add_x(xid[GXX][r], 1, band_axpby(0.5, band_diag(xb[GXX][r]), 0.0, band_diag(xb[GXX][r])));
    // A = V_0 (x) I + sum W (x) diag(a)
    A.add_q(0, band_axpby(1.0, band_diag(c[SIG]), 1.0, band_mul(band_diag(c[SV]), Dv)));
    for (size_t r = 0; r < xb[SIG].size(); ++r) A.add_w(xid[SIG][r], band_diag(xb[SIG][r]));
    for (size_t r = 0; r < xb[SV].size(); ++r) A.add_w(xid[SV][r], band_mul(band_diag(xb[SV][r]), Dv));
    // noise through D^x
    A.add_q(1, band_diag(c[SX]));
    for (size_t r = 0; r < xb[SX].size(); ++r) A.add_x(xid[SX][r], 0, band_diag(xb[SX][r]));

    const int nact = order == 1 ? 2 : (order == 2 ? 4 : 6);
    KOp M[MG_NBASIS] = {B, A, KOp(nv), KOp(nv), KOp(nv), KOp(nv)};
    std::string why;
    bool ok = true;
    // only the matrices the order uses have to exist in this form
    if (nact > 2) ok = ok && kop_mul(A, A, xr, M[2], why) && kop_comm(B, A, xr, M[3], why);
    if (nact > 4) ok = ok && kop_comm(M[3], A, xr, M[4], why) && kop_comm(M[3], B, xr, M[5], why);
    if (!ok) return mg_fail(MG_EUNSUPPORTED, why);

    // The three kinds of terms: words with unit vectors only (powers of D^x,
    // the V_q tables), depth-0 words (diagonal x-factors W (x) diag(a)) and
    // the other words (x-terms C (x) X).
    struct Split {
        Band V[3];
        std::vector<int> wid;
        std::vector<Band> W;
        std::vector<XWord> xw;
        std::vector<Band> X;
    };
    std::vector<Split> S(MG_NBASIS);
    for (int l = 0; l < MG_NBASIS; ++l) {
        for (auto& b : S[l].V) b = band_zero(nv);
        for (size_t k = 0; k < M[l].w.size(); ++k) {
            const XWord& x = M[l].w[k];
            if (x.plain()) S[l].V[x.d] = band_axpby(1.0, S[l].V[x.d], 1.0, M[l].V[k]);
            else if (x.d == 0) { S[l].wid.push_back(x.id[0]); S[l].W.push_back(M[l].V[k]); }
            else { S[l].xw.push_back(x); S[l].X.push_back(M[l].V[k]); }
        }
    }

    // Band radii actually used, after dropping cancellation residues.  A
    // factor V_q multiplies (D^x)^q, whose norm is about (1/dx)^q, a factor W
    // multiplies diag(a), whose norm is max|a|, and an x-term factor multiplies
    // a word of norm about prod_h max|x_h| (1/dx)^d, so entries are compared
    // with the whole matrix through these weights: entries below 1e-14 of the
    // largest weighted entry of the same basis matrix are zero in exact
    // arithmetic and stem from rounding in the products (a factor can consist
    // of residues only, e.g. the D^x part of [[B,A],B] for the
    // constant-coefficient operator).
    int R[3] = {0, 0, 0}, RW = 0, RC = 0;
    const double wq[3] = {1.0, 1.0 / dx, 1.0 / (dx * dx)};
    std::vector<double> wa(xr.vecs.size());
    for (size_t k = 0; k < xr.vecs.size(); ++k) {
        double m = 0.0;
        for (double v : xr.vecs[k]) m = std::max(m, std::fabs(v));
        wa[k] = m;
    }
    auto xmax = [&](int id) { return id < 0 ? 1.0 : wa[id]; };
    auto wword = [&](const XWord& x) {
        double w = 1.0;
        for (int h = 0; h <= x.d; ++h) w *= xmax(x.id[h]);
        for (int h = 0; h < x.d; ++h) w *= x.lt[h] ? 4.0 / (dx * dx) : 1.0 / dx;
        return w;
    };
    std::vector<int> used(xr.vecs.size(), 0);
    std::vector<XWord> xterms;   // distinct x-terms of the active matrices
    auto xterm_slot = [&](const XWord& x) {
        for (size_t k = 0; k < xterms.size(); ++k)
            if (xterms[k] == x) return (int)k;
        return -1;
    };
    auto radius = [&](const Band& V) {
        int r = 0;
        for (int i = 0; i < nv; ++i)
            for (int o = -V.r; o <= V.r; ++o)
                if (V.get(i, i + o) != 0.0) r = std::max(r, std::abs(o));
        return r;
    };
    for (int l = 0; l < MG_NBASIS; ++l) {
        Split& T = S[l];
        double mx = 0.0;
        for (int q = 0; q < 3; ++q)
            for (double v : T.V[q].a) mx = std::max(mx, std::fabs(v) * wq[q]);
        for (size_t k = 0; k < T.W.size(); ++k)
            for (double v : T.W[k].a) mx = std::max(mx, std::fabs(v) * wa[T.wid[k]]);
        for (size_t k = 0; k < T.X.size(); ++k)
            for (double v : T.X[k].a) mx = std::max(mx, std::fabs(v) * wword(T.xw[k]));
        for (int q = 0; q < 3; ++q) {
            for (double& v : T.V[q].a)
                if (std::fabs(v) * wq[q] <= 1e-14 * mx) v = 0.0;
            if (l < nact) R[q] = std::max(R[q], radius(T.V[q]));
        }
        for (size_t k = 0; k < T.W.size(); ++k) {
            for (double& v : T.W[k].a)
                if (std::fabs(v) * wa[T.wid[k]] <= 1e-14 * mx) v = 0.0;
            if (l >= nact || band_is_zero(T.W[k])) continue;
            RW = std::max(RW, radius(T.W[k]));
            used[T.wid[k]] = 1;
        }
        for (size_t k = 0; k < T.X.size(); ++k) {
            const double ww = wword(T.xw[k]);
            for (double& v : T.X[k].a)
                if (std::fabs(v) * ww <= 1e-14 * mx) v = 0.0;
            if (l >= nact || band_is_zero(T.X[k])) continue;
            RC = std::max(RC, radius(T.X[k]));
            if (xterm_slot(T.xw[k]) < 0) xterms.push_back(T.xw[k]);
        }
    }
    // With x-terms the kernels take the V tables of the order-2 band shape
    // (radii 2 and 1, no Dt^2): a Dt^2 factor, or a Dt factor of radius above
    // 1, becomes an x-term with unit vectors.
    if (!xterms.empty()) {
        for (int q = 1; q < 3; ++q) {
            if (q == 1 && R[1] <= 1) continue;
            XWord x;
            x.d = q;
            for (int l = 0; l < MG_NBASIS; ++l) {
                if (band_is_zero(S[l].V[q])) continue;
                S[l].xw.push_back(x);
                S[l].X.push_back(S[l].V[q]);
                S[l].V[q] = band_zero(nv);
                if (l >= nact) continue;
                RC = std::max(RC, radius(S[l].X.back()));
                if (xterm_slot(x) < 0) xterms.push_back(x);
            }
            R[q] = 0;
        }
    }
    // Euler reads B and A from the V tables and the diagonal factors only
    bool xt_in_ba = false;
    for (int l = 0; l < 2; ++l)
        for (size_t k = 0; k < S[l].X.size(); ++k) xt_in_ba = xt_in_ba || !band_is_zero(S[l].X[k]);
    // diagonal x-factors in use, numbered in registry order; with x-terms
    // the first MG_MAX_XDIAG keep their own slots (those of B and A, which the
    // Euler kernels read, come first: the coefficients are registered before
    // any product) and the others become depth-0 x-terms
    std::vector<int> slot(xr.vecs.size(), -1);
    int nd = 0;
    std::vector<int> overflow;
    for (size_t k = 0; k < xr.vecs.size(); ++k) {
        if (!used[k]) continue;
        if (nd < MG_MAX_XDIAG) slot[k] = nd++;
        else overflow.push_back((int)k);
    }
    if (!overflow.empty() && xterms.empty())
        return mg_fail(MG_EUNSUPPORTED, "more than 4 x-dependent factors in the Magnus basis");
    for (int id : overflow)
        for (int l = 0; l < 2; ++l)
            for (int w : S[l].wid)
                if (w == id)
                    return mg_fail(MG_EUNSUPPORTED,
                                   "more than 4 x-dependent factors in B and A together");
    for (int id : overflow) {
        XWord x;
        x.id[0] = id;
        xterms.push_back(x);
        RC = std::max(RC, RW);
    }
    if (RW > MG_XDIAG_RADIUS)
        return mg_fail(MG_EUNSUPPORTED, "band radius of an x-dependent factor above 2");
    if ((int)xterms.size() > MG_MAX_XTERM)
        return mg_fail(MG_EUNSUPPORTED, "more than 32 x-terms in the Magnus basis");
    if (RC > MG_XDIAG_RADIUS)
        return mg_fail(MG_EUNSUPPORTED, "band radius of an x-term factor above 2");
    // x-term vectors: slot 0 the unit vector, then every other vector the
    // words use, in registry order
    std::vector<int> vslot(xr.vecs.size(), -1);
    int nxv = xterms.empty() ? 0 : 1;
    for (size_t k = 0; k < xr.vecs.size(); ++k) {
        bool in = false;
        for (const XWord& x : xterms)
            for (int h = 0; h <= x.d; ++h) in = in || x.id[h] == (int)k;
        if (in) vslot[k] = nxv++;
    }
    if (nxv > MG_MAX_XVEC)
        return mg_fail(MG_EUNSUPPORTED, "more than 16 distinct x vectors in the x-terms");
    // highest power of D^x with a non-zero factor among the active matrices
    int qmax = 0;
    for (int l = 0; l < nact; ++l)
        for (int q = 1; q < 3; ++q)
            for (double v : S[l].V[q].a)
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
    if (!xterms.empty()) shape = std::max(shape, 1);   // built for the order-2 band shape
    if ((nd > 0 || !xterms.empty()) && shape > 1)
        return mg_fail(MG_EUNSUPPORTED,
                       "x-dependent coefficients are built for band shapes up to (2,1,0) in this library");
    for (int q = 0; q < 3; ++q) R[q] = kShapes[shape][q];
    ops->qmax = kShapes[shape][3];

    ops->grid = *g;
    ops->order = order;
    ops->nactive = nact;
    for (int q = 0; q < 3; ++q) ops->R[q] = R[q];
    // x-dependent factors: the kernels are built for 3 and for 4 factors
    // (unused ones are zero; the variable-coefficient workloads use 3), and
    // with x-terms for 4 factors
    ops->NC = (int)xterms.size();
    ops->xt_in_ba = xt_in_ba;
    ops->NXV = nxv;
    ops->ND = nd > 0 || ops->NC > 0 ? (nd <= 3 && ops->NC == 0 ? 3 : MG_MAX_XDIAG) : 0;
    ops->RW = ops->ND > 0 ? MG_XDIAG_RADIUS : 0;
    // V2 (the Dt^2 factor) has entries in the row only where Dt^2 occurs
    const int nq = ops->qmax >= 2 ? 3 : 2;
    ops->NB = (2 * R[0] + 1) + (2 * R[1] + 1) + (nq == 3 ? 2 * R[2] + 1 : 0) +
              ops->ND * (2 * ops->RW + 1);
    ops->NBP = (ops->NB + 1) & ~1;
    // Diagonal x-factors as midpoint plus deviation: W (x) diag(a) =
    // (m W) (x) I + W (x) diag(a - m) with m the midpoint of a.  The first part
    // joins the V0 band (in FP64, here) wherever every W of that factor fits
    // the V0 radius, so the kernels multiply only the deviation: in the FP32
    // form a point's diagonal is then not the near-cancelling sum of two large
    // rounded parts (the trace-shifted V0 centre and the full x-factor).
    std::vector<double> xmid(ops->ND, 0.0);
    ops->xdiag_host.assign((size_t)ops->ND * nx, 0.0);
    ops->xstat_host.assign((size_t)ops->ND * 4, 0.0);
    for (size_t k = 0; k < xr.vecs.size(); ++k) {
        if (slot[k] < 0) continue;
        const std::vector<double>& a = xr.vecs[k];
        double lo = a[0], hi = a[0];
        for (int i = 0; i < nx; ++i) {
            lo = std::min(lo, a[i]);
            hi = std::max(hi, a[i]);
        }
        bool fits = true;
        for (int l = 0; l < MG_NBASIS; ++l)
            for (size_t t = 0; t < S[l].W.size(); ++t)
                if (S[l].wid[t] == (int)k && radius(S[l].W[t]) > R[0]) fits = false;
        const double m = fits ? 0.5 * (hi + lo) : 0.0;
        xmid[slot[k]] = m;
        double sum = 0.0;
        for (int i = 0; i < nx; ++i) {
            ops->xdiag_host[(size_t)slot[k] * nx + i] = a[i] - m;
            sum += a[i] - m;
        }
        double* st = ops->xstat_host.data() + (size_t)slot[k] * 4;
        st[0] = sum;                 // for the trace
        st[1] = 0.5 * (hi + lo) - m; // midpoint and half-width of the values,
        st[2] = 0.5 * (hi - lo);     // for the 1-norm bound
    }
    // x-term vectors [NXV][nx], descriptors {d, outer, middle, inner} and per
    // x-term {||X||_1, tr X, 0, 0}
    ops->xchain_host.assign((size_t)nxv * nx, 0.0);
    for (int i = 0; i < nx && nxv > 0; ++i) ops->xchain_host[i] = 1.0;
    for (size_t k = 0; k < xr.vecs.size(); ++k)
        if (vslot[k] >= 0)
            for (int i = 0; i < nx; ++i) ops->xchain_host[(size_t)vslot[k] * nx + i] = xr.vecs[k][i];
    ops->xdesc_host.assign((size_t)ops->NC * 4, 0);
    ops->cstat_host.assign((size_t)ops->NC * 4, 0.0);
    auto vs = [&](int id) { return id < 0 ? 0 : vslot[id]; };
    for (int k = 0; k < ops->NC; ++k) {
        const XWord& x = xterms[k];
        int32_t* d = ops->xdesc_host.data() + (size_t)k * 4;
        d[0] = x.d | (x.lt[0] << 2) | (x.lt[1] << 3);   // depth, letters
        d[1] = vs(x.id[0]);
        d[2] = x.d == 2 ? vs(x.id[1]) : 0;
        d[3] = vs(x.id[x.d]);
        if (x.d == 0) d[3] = 0;   // the unit vector: the outer vector is the factor
        const Band X = word_matrix(x, xr, nx);
        double n1 = 0.0, tr = 0.0;
        for (int j = 0; j < nx; ++j) {
            double col = 0.0;
            for (int i = std::max(0, j - X.r); i <= std::min(nx - 1, j + X.r); ++i)
                col += std::fabs(X.get(i, j));
            n1 = std::max(n1, col);
            tr += X.get(j, j);
        }
        ops->cstat_host[(size_t)k * 4] = n1;
        ops->cstat_host[(size_t)k * 4 + 1] = tr;
    }
    // table rows are padded to the rows the kernel shape covers
    int rows = resident_rows(nx, nv);
    if (rows == 0) rows = coop_table_rows(nx, nv);
    ops->nv_pad = std::max(nv, rows);
    // main rows [6][nv_pad][NBP], then the x-term section [6][nv_pad][NCB]
    ops->NCB = ops->NC * (2 * MG_XDIAG_RADIUS + 1);
    ops->basis_host.assign((size_t)MG_NBASIS * ops->nv_pad * (ops->NBP + ops->NCB), 0.0);
    const double fold[3] = {1.0, 1.0 / (2.0 * dx), 1.0 / (4.0 * dx * dx)};
    for (int l = 0; l < MG_NBASIS; ++l)
        for (int j = 0; j < nv; ++j) {
            double* row = ops->basis_host.data() + ((size_t)l * ops->nv_pad + j) * ops->NBP;
            int off = 0;
            for (int q = 0; q < nq; ++q) {
                for (int o = -R[q]; o <= R[q]; ++o) row[off + o + R[q]] = S[l].V[q].get(j, j + o) * fold[q];
                off += 2 * R[q] + 1;
            }
            // the midpoints of the diagonal x-factors, in V0
            for (size_t k = 0; k < S[l].W.size(); ++k) {
                const int sl = slot[S[l].wid[k]];
                if (sl < 0 || xmid[sl] == 0.0) continue;
                for (int o = -R[0]; o <= R[0]; ++o) row[o + R[0]] += xmid[sl] * S[l].W[k].get(j, j + o);
            }
            // x-term bands, with the factors of the word's letters folded in
            double* crow = ops->basis_host.data() + (size_t)MG_NBASIS * ops->nv_pad * ops->NBP +
                           ((size_t)l * ops->nv_pad + j) * ops->NCB;
            for (size_t k = 0; k < S[l].W.size(); ++k) {
                const int id = S[l].wid[k];
                const int sl = slot[id];
                double* w = nullptr;
                if (sl >= 0) {
                    w = row + off + sl * (2 * ops->RW + 1);
                } else {
                    XWord x;
                    x.id[0] = id;
                    const int xs = xterm_slot(x);
                    if (xs < 0) continue;   // only in matrices the order does not use
                    w = crow + xs * (2 * MG_XDIAG_RADIUS + 1);
                }
                for (int o = -MG_XDIAG_RADIUS; o <= MG_XDIAG_RADIUS; ++o)
                    w[o + MG_XDIAG_RADIUS] = S[l].W[k].get(j, j + o);
            }
            for (size_t k = 0; k < S[l].X.size(); ++k) {
                if (band_is_zero(S[l].X[k])) continue;
                const int xs = xterm_slot(S[l].xw[k]);
                if (xs < 0) continue;   // only in matrices the order does not use
                double* w = crow + xs * (2 * MG_XDIAG_RADIUS + 1);
                for (int o = -MG_XDIAG_RADIUS; o <= MG_XDIAG_RADIUS; ++o)
                    w[o + MG_XDIAG_RADIUS] = S[l].X[k].get(j, j + o) * S[l].xw[k].fold(dx);
            }
        }
    return MG_OK;
}
