// smalleig.cpp -- eigenpairs of the small dense symmetric projected matrix of
// the Krylov method (order ~ 100).  All eigenvalues by implicit QR on the
// Householder tridiagonal form; eigenvectors only for the selected values, by
// inverse iteration on the tridiagonal (with Gram-Schmidt inside clusters) and
// back-transformation.
#include "smalleig.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace mbl {
namespace {

// Householder reduction Q^T A Q = T; reflectors kept in a (column j below j+1)
void tridiag(int m, std::vector<double> &a, std::vector<double> &d, std::vector<double> &e,
             std::vector<double> &tau) {
    d.assign(m, 0.0);
    e.assign(std::max(m - 1, 1), 0.0);
    tau.assign(std::max(m - 1, 1), 0.0);
    std::vector<double> v(m), p(m);
    for (int c = 0; c + 2 < m; c++) {
        int mm = m - c - 1;
        double *col = &a[(size_t)c * m];
        double alpha = col[c + 1], sig = 0.0;
        for (int i = c + 2; i < m; i++) sig += col[i] * col[i];
        if (sig == 0.0) { tau[c] = 0.0; e[c] = alpha; continue; }
        double nrm = std::sqrt(alpha * alpha + sig);
        double beta = alpha > 0.0 ? -nrm : nrm;
        double t = (beta - alpha) / beta, sc = 1.0 / (alpha - beta);
        tau[c] = t;
        e[c] = beta;
        v[0] = 1.0;
        for (int i = 1; i < mm; i++) { col[c + 1 + i] *= sc; v[i] = col[c + 1 + i]; }
        std::fill(p.begin(), p.begin() + mm, 0.0);
        for (int j = 0; j < mm; j++) {             // p = t A v, column by column
            const double *aj = &a[(size_t)(c + 1 + j) * m + (c + 1)];
            const double vj = v[j];
            for (int i = 0; i < mm; i++) p[i] += aj[i] * vj;
        }
        for (int i = 0; i < mm; i++) p[i] *= t;
        double pv = 0.0;
        for (int i = 0; i < mm; i++) pv += p[i] * v[i];
        double K = 0.5 * t * pv;
        for (int i = 0; i < mm; i++) p[i] -= K * v[i];
        for (int j = 0; j < mm; j++)
            for (int i = 0; i < mm; i++)
                a[(size_t)(c + 1 + j) * m + (c + 1 + i)] -= v[i] * p[j] + p[i] * v[j];
    }
    for (int i = 0; i < m; i++) d[i] = a[(size_t)i * m + i];
    if (m >= 2) e[m - 2] = a[(size_t)(m - 2) * m + (m - 1)];
}

// All eigenvalues of the symmetric tridiagonal (d, e) by implicit QR steps with
// the Wilkinson shift (a bulge chased down each unreduced block), ascending.
// Deflation when |e_i| <= u (|d_i| + |d_i+1|).
void tri_qr_values(int m, const double *d0, const double *e0, std::vector<double> &w) {
    std::vector<double> a(d0, d0 + m), b(e0, e0 + std::max(m - 1, 0));
    const double u = std::numeric_limits<double>::epsilon();
    int hi = m - 1, iters = 0;
    while (hi > 0 && iters < 60 * m) {
        if (std::fabs(b[hi - 1]) <= u * (std::fabs(a[hi - 1]) + std::fabs(a[hi])) ||
            b[hi - 1] == 0.0) {
            b[hi - 1] = 0.0;
            hi--;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(b[lo - 1]) > u * (std::fabs(a[lo - 1]) + std::fabs(a[lo])))
            lo--;
        if (lo > 0) b[lo - 1] = 0.0;
        // Wilkinson shift: eigenvalue of the trailing 2 x 2 nearer a[hi]
        double dd = 0.5 * (a[hi - 1] - a[hi]), bb = b[hi - 1];
        double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, bb);
        double mu = a[hi] - (den != 0.0 ? bb * bb / den : 0.0);
        double x = a[lo] - mu, z = b[lo];
        for (int k = lo; k < hi; k++) {
            double r = std::hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) { c = x / r; s = -z / r; }
            if (k > lo) b[k - 1] = r;
            double ak = a[k], bk = b[k], ak1 = a[k + 1];
            a[k] = c * c * ak - 2.0 * c * s * bk + s * s * ak1;
            b[k] = c * s * ak + (c * c - s * s) * bk - c * s * ak1;
            a[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * ak1;
            if (k + 1 < hi) {
                z = -s * b[k + 1];
                b[k + 1] *= c;
                x = b[k];
            }
        }
        iters++;
    }
    w = a;
    std::sort(w.begin(), w.end());
}

// (T - lam) x = b by Gaussian elimination with partial pivoting (tridiagonal)
void tri_shift_solve(int m, const double *d, const double *e, double lam, double tiny, double *x) {
    std::vector<double> u0(m), u1(m), u2(m), l(m);
    std::vector<char> sw(m);
    double a = d[0] - lam, c = m > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < m; i++) {
        double s = e[i], nd = d[i + 1] - lam, nc = (i + 2 < m) ? e[i + 1] : 0.0;
        if (std::fabs(a) >= std::fabs(s)) {
            if (a == 0.0) a = tiny;
            double f = s / a;
            u0[i] = a; u1[i] = c; u2[i] = 0.0; l[i] = f; sw[i] = 0;
            a = nd - f * c;
            c = nc;
        } else {
            double f = a / s;
            u0[i] = s; u1[i] = nd; u2[i] = nc; l[i] = f; sw[i] = 1;
            a = c - f * nd;
            c = -f * nc;
        }
    }
    if (a == 0.0) a = tiny;
    u0[m - 1] = a;
    for (int i = 0; i + 1 < m; i++) {
        if (sw[i]) std::swap(x[i], x[i + 1]);
        x[i + 1] -= l[i] * x[i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double s = x[i];
        if (i + 1 < m) s -= u1[i] * x[i + 1];
        if (i + 2 < m) s -= u2[i] * x[i + 2];
        x[i] = s / u0[i];
    }
}

}  // namespace

void sym_eig_values(int m, const double *A, SymEigWork &wk, std::vector<double> &w) {
    wk.m = m;
    w.assign(m, 0.0);
    if (m == 0) return;
    if (m == 1) {
        w[0] = A[0];
        wk.d.assign(1, A[0]);
        wk.e.assign(1, 0.0);
        wk.tmax = std::fabs(A[0]);
        return;
    }
    wk.a.assign(A, A + (size_t)m * m);
    std::vector<double> &a = wk.a;
    for (int j = 0; j < m; j++)          // symmetrise
        for (int i = j + 1; i < m; i++) {
            double s = 0.5 * (a[(size_t)j * m + i] + a[(size_t)i * m + j]);
            a[(size_t)j * m + i] = a[(size_t)i * m + j] = s;
        }
    tridiag(m, a, wk.d, wk.e, wk.tau);
    const std::vector<double> &d = wk.d, &e = wk.e;
    double tmax = 0.0;
    for (int i = 0; i < m; i++) {
        double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        tmax = std::max(tmax, std::fabs(d[i]) + r);
    }
    wk.tmax = tmax;
    tri_qr_values(m, d.data(), e.data(), w);
}

void sym_eig_vectors(const SymEigWork &wk, const std::vector<double> &w,
                     const std::vector<int> &sel, std::vector<double> &Y) {
    const int m = wk.m;
    Y.assign((size_t)m * sel.size(), 0.0);
    if (m == 0) return;
    if (m == 1) {
        for (size_t j = 0; j < sel.size(); j++) Y[j] = 1.0;
        return;
    }
    const std::vector<double> &d = wk.d, &e = wk.e, &a = wk.a, &tau = wk.tau;
    const double tmax = wk.tmax;
    // eigenvectors of T for the selected values, ascending order of value
    std::vector<int> order(sel.size());
    for (size_t j = 0; j < sel.size(); j++) order[j] = (int)j;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return w[sel[x]] < w[sel[y]]; });
    double tiny = std::numeric_limits<double>::epsilon() * std::max(tmax, 1e-300);
    double ortol = 1e-3 * tmax;
    uint64_t st = 0x2545F4914F6CDD1DULL;
    std::vector<int> done;
    for (size_t q = 0; q < order.size(); q++) {
        int j = order[q];
        double lam = w[sel[j]];
        double *x = &Y[(size_t)j * m];
        for (int i = 0; i < m; i++) {
            st ^= st << 13; st ^= st >> 7; st ^= st << 17;
            x[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        for (int it = 0; it < 3; it++) {
            tri_shift_solve(m, d.data(), e.data(), lam, tiny, x);
            for (int o : done) {
                if (std::fabs(w[sel[o]] - lam) > ortol) continue;
                const double *y = &Y[(size_t)o * m];
                double dot = 0.0;
                for (int i = 0; i < m; i++) dot += x[i] * y[i];
                for (int i = 0; i < m; i++) x[i] -= dot * y[i];
            }
            double nrm = 0.0;
            for (int i = 0; i < m; i++) nrm += x[i] * x[i];
            nrm = std::sqrt(nrm);
            for (int i = 0; i < m; i++) x[i] /= nrm;
        }
        done.push_back(j);
    }
    // back-transform: y = H_0 H_1 ... H_{m-3} x
    for (size_t j = 0; j < sel.size(); j++) {
        double *x = &Y[j * m];
        for (int c = m - 3; c >= 0; c--) {
            if (tau[c] == 0.0) continue;
            const double *col = &a[(size_t)c * m];
            double dot = x[c + 1];
            for (int i = c + 2; i < m; i++) dot += col[i] * x[i];
            dot *= tau[c];
            x[c + 1] -= dot;
            for (int i = c + 2; i < m; i++) x[i] -= dot * col[i];
        }
    }
}

void sym_eig_select(int m, const double *A, std::vector<double> &w, const std::vector<int> &sel,
                    std::vector<double> &Y) {
    SymEigWork wk;
    sym_eig_values(m, A, wk, w);
    sym_eig_vectors(wk, w, sel, Y);
}

bool cholesky_upper(int b, const double *G, std::vector<double> &R, double rel_tiny) {
    R.assign((size_t)b * b, 0.0);
    double dmax = 0.0;
    for (int i = 0; i < b; i++) dmax = std::max(dmax, G[(size_t)i * b + i]);
    bool ok = true;
    for (int j = 0; j < b; j++) {
        for (int i = 0; i <= j; i++) {
            double s = G[(size_t)j * b + i];
            for (int k = 0; k < i; k++) s -= R[(size_t)i * b + k] * R[(size_t)j * b + k];
            if (i == j) {
                if (s <= rel_tiny * dmax) { ok = false; s = std::max(s, rel_tiny * dmax + 1e-300); }
                R[(size_t)j * b + j] = std::sqrt(s);
            } else {
                R[(size_t)j * b + i] = s / R[(size_t)i * b + i];
            }
        }
    }
    return ok;
}

void upper_inverse(int b, const std::vector<double> &R, std::vector<double> &Ri) {
    Ri.assign((size_t)b * b, 0.0);
    for (int j = 0; j < b; j++) {
        Ri[(size_t)j * b + j] = 1.0 / R[(size_t)j * b + j];
        for (int i = j - 1; i >= 0; i--) {
            double s = 0.0;
            for (int k = i + 1; k <= j; k++) s += R[(size_t)k * b + i] * Ri[(size_t)j * b + k];
            Ri[(size_t)j * b + i] = -s / R[(size_t)i * b + i];
        }
    }
}

}  // namespace mbl
