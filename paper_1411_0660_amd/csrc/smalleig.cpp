// smalleig.cpp -- eigenpairs of the small dense symmetric projected matrix of
// the Krylov method (order ~ 100).  All eigenvalues by Sturm bisection on the
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
        for (int i = 0; i < mm; i++) {
            double s = 0.0;
            for (int j = 0; j < mm; j++) s += a[(size_t)(c + 1 + j) * m + (c + 1 + i)] * v[j];
            p[i] = t * s;
        }
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

int sturm(int m, const double *d, const double *e2, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) cnt++;
    for (int i = 1; i < m; i++) {
        q = d[i] - x - e2[i - 1] / q;
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0) cnt++;
    }
    return cnt;
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

void sym_eig_select(int m, const double *A, std::vector<double> &w, const std::vector<int> &sel,
                    std::vector<double> &Y) {
    w.assign(m, 0.0);
    Y.assign((size_t)m * sel.size(), 0.0);
    if (m == 0) return;
    if (m == 1) {
        w[0] = A[0];
        for (size_t j = 0; j < sel.size(); j++) Y[j] = 1.0;
        return;
    }
    std::vector<double> a(A, A + (size_t)m * m), d, e, tau;
    for (int j = 0; j < m; j++)          // symmetrise
        for (int i = j + 1; i < m; i++) {
            double s = 0.5 * (a[(size_t)j * m + i] + a[(size_t)i * m + j]);
            a[(size_t)j * m + i] = a[(size_t)i * m + j] = s;
        }
    tridiag(m, a, d, e, tau);
    std::vector<double> e2(m);
    double tmax = 0.0, lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; i++) {
        double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
        tmax = std::max(tmax, std::fabs(d[i]) + r);
        if (i + 1 < m) e2[i] = e[i] * e[i];
    }
    double pivmin = std::numeric_limits<double>::min() + 1e-30 * tmax * tmax;
    for (int idx = 0; idx < m; idx++) {
        double a0 = lo, b0 = hi;
        for (int it = 0; it < 200 && b0 - a0 > 2e-16 * std::max(tmax, 1e-300); it++) {
            double mid = 0.5 * (a0 + b0);
            if (sturm(m, d.data(), e2.data(), mid, pivmin) > idx) b0 = mid; else a0 = mid;
        }
        w[idx] = 0.5 * (a0 + b0);
    }
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
        for (int it = 0; it < 4; it++) {
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
