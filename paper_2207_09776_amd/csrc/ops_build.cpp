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

// sum_{q=0..2} V[q] (x) (D^x)^q
struct KOp {
    Band V[3];
    explicit KOp(int nv) { for (auto& b : V) b = band_zero(nv); }
};

bool kop_mul(const KOp& X, const KOp& Y, KOp& out) {
    int nv = X.V[0].n;
    KOp Z(nv);
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            bool xz = std::all_of(X.V[p].a.begin(), X.V[p].a.end(), [](double v) { return v == 0.0; });
            bool yz = std::all_of(Y.V[q].a.begin(), Y.V[q].a.end(), [](double v) { return v == 0.0; });
            if (xz || yz) continue;
            if (p + q > 2) return false;
            Z.V[p + q] = band_axpby(1.0, Z.V[p + q], 1.0, band_mul(X.V[p], Y.V[q]));
        }
    out = Z;
    return true;
}

bool kop_comm(const KOp& X, const KOp& Y, KOp& out) {
    KOp XY(X.V[0].n), YX(X.V[0].n);
    if (!kop_mul(X, Y, XY) || !kop_mul(Y, X, YX)) return false;
    KOp Z(X.V[0].n);
    for (int q = 0; q < 3; ++q) Z.V[q] = band_axpby(1.0, XY.V[q], -1.0, YX.V[q]);
    out = Z;
    return true;
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
    const double* vonly[7] = {cf->h, cf->fx, cf->fv, cf->gxv, cf->gvv, cf->sig, cf->sv};
    const char* names[7] = {"h", "fx", "fv", "gxv", "gvv", "sig", "sv"};
    std::vector<double> c[7];
    bool nz[7];
    for (int t = 0; t < 7; ++t)
        if (!v_only(vonly[t], nx, nv, c[t], nz[t]))
            return mg_fail(MG_EUNSUPPORTED, std::string("coefficient ") + names[t] +
                                                " must be finite and depend on v only in this build");
    const double dx = (g->bx - g->ax) / (nx + 1), dv = (g->bv - g->av) / (nv + 1);
    Band Dv = first_difference(nv, dv), Dvv = second_difference(nv, dv);

    // B = V_0 (x) I + V_1 (x) D^x
    KOp B(nv), A(nv);
    B.V[0] = band_axpby(1.0, band_diag(c[0]), 1.0, band_mul(band_diag(c[2]), Dv));
    B.V[0] = band_axpby(1.0, B.V[0], 0.5, band_mul(band_diag(c[4]), Dvv));
    B.V[1] = band_axpby(1.0, band_diag(c[1]), 1.0, band_mul(band_diag(c[3]), Dv));
    // A = V_0 (x) I
    A.V[0] = band_axpby(1.0, band_diag(c[5]), 1.0, band_mul(band_diag(c[6]), Dv));

    KOp M[MG_NBASIS] = {B, A, KOp(nv), KOp(nv), KOp(nv), KOp(nv)};
    bool ok = kop_mul(A, A, M[2]) && kop_comm(B, A, M[3]) && kop_comm(M[3], A, M[4]) &&
              kop_comm(M[3], B, M[5]);
    if (!ok) return mg_fail(MG_EUNSUPPORTED, "x-derivative power above 2 in the Magnus basis");

    const int nact = order == 1 ? 2 : (order == 2 ? 4 : 6);
    // Band radii actually used, after dropping cancellation residues.  A
    // factor V_q multiplies (D^x)^q, whose norm is about (1/dx)^q, so entries
    // are compared with the whole matrix through the weight (1/dx)^q: entries
    // below 1e-14 of the largest weighted entry of the same basis matrix are
    // zero in exact arithmetic and stem from rounding in the products (a
    // factor can consist of residues only, e.g. the D^x part of [[B,A],B] for
    // the constant-coefficient operator).
    int R[3] = {0, 0, 0};
    const double wq[3] = {1.0, 1.0 / dx, 1.0 / (dx * dx)};
    for (int l = 0; l < MG_NBASIS; ++l) {
        double mx = 0.0;
        for (int q = 0; q < 3; ++q)
            for (double v : M[l].V[q].a) mx = std::max(mx, std::fabs(v) * wq[q]);
        for (int q = 0; q < 3; ++q) {
            Band& V = M[l].V[q];
            for (double& v : V.a)
                if (std::fabs(v) * wq[q] <= 1e-14 * mx) v = 0.0;
            if (l >= nact) continue;
            for (int i = 0; i < nv; ++i)
                for (int o = -V.r; o <= V.r; ++o)
                    if (V.get(i, i + o) != 0.0) R[q] = std::max(R[q], std::abs(o));
        }
    }
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
    for (int q = 0; q < 3; ++q) R[q] = kShapes[shape][q];
    ops->qmax = kShapes[shape][3];

    ops->grid = *g;
    ops->order = order;
    ops->nactive = nact;
    for (int q = 0; q < 3; ++q) ops->R[q] = R[q];
    ops->NB = (2 * R[0] + 1) + (2 * R[1] + 1) + (2 * R[2] + 1);
    ops->NBP = (ops->NB + 1) & ~1;
    // table rows are padded to the rows the kernel shape covers
    int rows = resident_rows(nx, nv);
    if (rows == 0) {
        const int rw = coop_rows_per_group_member(nx);
        if (rw > 0) rows = (nv + rw - 1) / rw * rw;
    }
    ops->nv_pad = std::max(nv, rows);
    ops->basis_host.assign((size_t)MG_NBASIS * ops->nv_pad * ops->NBP, 0.0);
    const double fold[3] = {1.0, 1.0 / (2.0 * dx), 1.0 / (4.0 * dx * dx)};
    for (int l = 0; l < MG_NBASIS; ++l)
        for (int j = 0; j < nv; ++j) {
            double* row = ops->basis_host.data() + ((size_t)l * ops->nv_pad + j) * ops->NBP;
            int off = 0;
            for (int q = 0; q < 3; ++q) {
                for (int o = -R[q]; o <= R[q]; ++o) row[off + o + R[q]] = M[l].V[q].get(j, j + o) * fold[q];
                off += 2 * R[q] + 1;
            }
        }
    return MG_OK;
}
