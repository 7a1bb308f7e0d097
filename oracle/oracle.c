/*
 * oracle.c -- plain CPU FP64 oracle for the random-field Heisenberg chain
 *             shift-invert eigenproblem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path: it enumerates its own basis (brute force), ranks by binary search,
 * builds the dense Hamiltonian and diagonalises it with a dense symmetric
 * eigensolver (Householder tridiagonalisation + implicit QL with a shift from
 * the leading 2 x 2, Golub & Van Loan, Matrix Computations, section 8.3), with
 * eigenvectors by tridiagonal inverse iteration and back-transformation.
 *
 * What it computes (paper: Luitz, Laflorencie, Alet, "Many-body localization
 * edge in the random-field Heisenberg chain", 2014):
 *   - the model of Eq. (1): H = J sum_i S_i . S_{i+1} + sum_i h_i S^z_i on a
 *     periodic chain, h_i uniform in [-h, h], restricted to the S^z = 0
 *     sector (section "Numerical method").  The sign of the field term is
 *     immaterial: the global spin flip maps the sector to itself and
 *     H(h) to H(-h), so spectra and all observables below are unchanged.
 *   - the extremal energies E_min, E_max, the target sigma = E_min +
 *     eps (E_max - E_min), and the nev eigenpairs closest to sigma
 *     (section "Numerical method");
 *   - the observables of section "Characterization of ergodic and localized
 *     regimes": gap ratio r (item i), half-chain entanglement entropy S_E
 *     (item ii), participation entropy S_1 (item iii); and the remaining
 *     indicators: Kullback-Leibler divergence of neighbouring eigenstates
 *     (item i), bipartite fluctuations F (item ii), participation entropy S_2
 *     (item iii), and the dynamical spin fraction f (Supplementary material,
 *     "Dynamical spin fraction").
 *
 * Conventions (readings where the paper is silent):
 *   - basis: all L-bit words with popcount (L+1)/2 (integer division: L/2,
 *     the S^z = 0 sector, for even L; S^z = +1/2 for odd L), ascending; bit i <-> site i+1,
 *     bit set = spin up;
 *   - fields: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) from state = seed,
 *     u = (z >> 11) * 2^-53, h_i = h (2u - 1), one draw per site in site order;
 *   - subsystem A for S_E and F = sites 1..L/2 = the low L/2 bits.
 *
 * Everything is FP64, unblocked, single-threaded; no LAPACK.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014): the published generator.            */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ULL;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Disorder fields h_i uniform in [-h, h] (Eq. (1) and the sentence after it). */
void orc_fields(int L, double h, uint64_t seed, double *out)
{
    uint64_t st = seed;
    for (int i = 0; i < L; i++) {
        uint64_t z = orc_splitmix64_next(&st);
        double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        out[i] = h * (2.0 * u - 1.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Basis of the sector with nup up spins: brute force over all 2^L words.    */
/* ------------------------------------------------------------------------ */
static int orc_popcount(uint64_t s)
{
    int c = 0;
    while (s) { c += (int)(s & 1u); s >>= 1; }
    return c;
}

long orc_sector_basis(int L, int nup, uint32_t *out)
{
    long n = 0;
    uint64_t top = (uint64_t)1 << L;
    for (uint64_t s = 0; s < top; s++)
        if (orc_popcount(s) == nup) {
            if (out) out[n] = (uint32_t)s;
            n++;
        }
    return n;
}

/* Index of word s in the ascending basis (binary search); -1 if absent. */
long orc_rank(const uint32_t *basis, long dim, uint32_t s)
{
    long lo = 0, hi = dim - 1;
    while (lo <= hi) {
        long mid = lo + (hi - lo) / 2;
        if (basis[mid] == s) return mid;
        if (basis[mid] < s) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Dense Hamiltonian, Eq. (1), column-major n x n.                           */
/*   S_i.S_j = S^z_i S^z_j + (S^+_i S^-_j + S^-_i S^+_j)/2 ;                  */
/*   S^z = sigma/2 with sigma = +-1.  For each bond (i, i+1 mod L):           */
/*   diagonal += J sigma_i sigma_j / 4, and if the two spins differ the       */
/*   exchange term adds J/2 between s and s with both spins flipped.          */
/*   Field term: diagonal += h_i sigma_i / 2.  Entries are added, so the      */
/*   doubled bond of L = 2 is summed.                                         */
/* ------------------------------------------------------------------------ */
void orc_dense_H(int L, double J, const double *fields, const uint32_t *basis,
                 long dim, double *H)
{
    memset(H, 0, sizeof(double) * (size_t)dim * (size_t)dim);
    for (long k = 0; k < dim; k++) {
        uint32_t s = basis[k];
        for (int i = 0; i < L; i++) {
            int j = (i + 1) % L;
            int si = ((s >> i) & 1u) ? 1 : -1;
            int sj = ((s >> j) & 1u) ? 1 : -1;
            H[k * dim + k] += 0.25 * J * (double)(si * sj);
            if (si != sj) {
                uint32_t t = s ^ ((1u << i) | (1u << j));
                long m = orc_rank(basis, dim, t);
                H[k * dim + m] += 0.5 * J;  /* column k, row m */
            }
        }
        for (int i = 0; i < L; i++) {
            int si = ((s >> i) & 1u) ? 1 : -1;
            H[k * dim + k] += 0.5 * fields[i] * (double)si;
        }
    }
}

/* y = H x without forming H (same terms as orc_dense_H); for certificates
 * at sizes where the dense matrix does not fit. */
void orc_apply_H(int L, double J, const double *fields, const uint32_t *basis,
                 long dim, const double *x, double *y)
{
    for (long k = 0; k < dim; k++) y[k] = 0.0;
    for (long k = 0; k < dim; k++) {
        uint32_t s = basis[k];
        double dg = 0.0;
        for (int i = 0; i < L; i++) {
            int j = (i + 1) % L;
            int si = ((s >> i) & 1u) ? 1 : -1;
            int sj = ((s >> j) & 1u) ? 1 : -1;
            dg += 0.25 * J * (double)(si * sj);
            if (si != sj) {
                uint32_t t = s ^ ((1u << i) | (1u << j));
                long m = orc_rank(basis, dim, t);
                y[m] += 0.5 * J * x[k];
            }
        }
        for (int i = 0; i < L; i++) {
            int si = ((s >> i) & 1u) ? 1 : -1;
            dg += 0.5 * fields[i] * (double)si;
        }
        y[k] += dg * x[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Householder tridiagonalisation (Golub & Van Loan Alg. 8.3.1).             */
/* A: column-major n x n symmetric, lower triangle referenced.  On return    */
/* d[0..n-1] is the diagonal, e[0..n-2] the subdiagonal of T = Q^T A Q, and  */
/* the reflector H_k = I - tau_k v_k v_k^T (acting on rows k+1..n-1, with    */
/* v_k(k+1) = 1 implicit) is stored in A(k+2..n-1, k) and tau[k].            */
/* Only the first `steps` reflections are applied when steps >= 0 (used to   */
/* time a bounded sample of a large run); steps < 0 means all n-2.           */
/* ------------------------------------------------------------------------ */
long orc_tridiagonalize(long n, double *A, double *d, double *e, double *tau,
                        long steps)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    long kend = n - 2;
    if (steps >= 0 && steps < kend) kend = steps;
    long k;
    for (k = 0; k < kend; k++) {
        double *col = A + k * n;
        double alpha = col[k + 1];
        double sig2 = 0.0;
        for (long i = k + 2; i < n; i++) sig2 += col[i] * col[i];
        if (sig2 == 0.0) {              /* already reduced in this column */
            tau[k] = 0.0;
            e[k] = alpha;
            continue;
        }
        double nrm = sqrt(alpha * alpha + sig2);
        double beta = (alpha <= 0.0) ? nrm : -nrm;
        double t = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        tau[k] = t;
        e[k] = beta;
        long m = n - k - 1;             /* trailing block size, rows k+1..n-1 */
        v[0] = 1.0;
        for (long i = 1; i < m; i++) { col[k + 1 + i] *= scale; v[i] = col[k + 1 + i]; }
        /* p = t * B v, B = A(k+1.., k+1..) symmetric, lower triangle stored */
        for (long i = 0; i < m; i++) p[i] = 0.0;
        for (long j = 0; j < m; j++) {
            const double *bj = A + (k + 1 + j) * n + (k + 1);
            double vj = v[j], acc = bj[j] * vj;
            for (long i = j + 1; i < m; i++) {
                acc += bj[i] * v[i];
                p[i] += bj[i] * vj;
            }
            p[j] += acc;
        }
        double pv = 0.0;
        for (long i = 0; i < m; i++) { p[i] *= t; pv += p[i] * v[i]; }
        double K = 0.5 * t * pv;
        for (long i = 0; i < m; i++) p[i] -= K * v[i];      /* p := w */
        for (long j = 0; j < m; j++) {                       /* B -= v w^T + w v^T */
            double *bj = A + (k + 1 + j) * n + (k + 1);
            double vj = v[j], wj = p[j];
            for (long i = j; i < m; i++) bj[i] -= v[i] * wj + p[i] * vj;
        }
    }
    for (long i = 0; i < n; i++) d[i] = A[i * n + i];
    if (kend == n - 2 && n >= 2) e[n - 2] = A[(n - 2) * n + (n - 1)];
    free(p); free(v);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Implicit symmetric tridiagonal QL with a shift from the leading 2 x 2     */
/* (G&VL section 8.3; the QL form works from the bottom of each unreduced    */
/* block upward, so eigenvalues deflate at its top).  d[0..n-1] diagonal,    */
/* e[0..n-2] the coupling of i and i+1 (e must have room for n entries).     */
/* On return d holds the eigenvalues (unsorted).  If Z is non-NULL           */
/* (column-major ldz x n), each plane rotation G in the plane (j-1, j) is    */
/* accumulated as Z <- Z G.  Returns 0 on success, -1 if an iteration cap is */
/* hit.                                                                      */
/* ------------------------------------------------------------------------ */
int orc_tridiag_ql(long n, double *d, double *e, double *Z, long ldz)
{
    long top = 0, iters = 0, cap = 60 * (n > 1 ? n : 1);
    while (top < n) {
        /* bottom of the unreduced block that starts at top */
        long bot = top;
        while (bot < n - 1 &&
               fabs(e[bot]) > DBL_EPSILON * (fabs(d[bot]) + fabs(d[bot + 1])))
            bot++;
        if (bot < n - 1) e[bot] = 0.0;
        if (bot == top) { top++; continue; }     /* d[top] has converged */
        if (++iters > cap) return -1;
        /* shift: eigenvalue of [[d_top, e_top], [e_top, d_top+1]] nearer d_top */
        double half = 0.5 * (d[top + 1] - d[top]);
        double den = half + (half >= 0.0 ? 1.0 : -1.0) * hypot(half, e[top]);
        double mu = d[top] - e[top] * e[top] / den;
        /* first rotation from the last column of T - mu I, then chase the
         * bulge up to the top of the block */
        double x = d[bot] - mu, z = e[bot - 1];
        for (long j = bot; j > top; j--) {
            double r = hypot(x, z), c = 1.0, s = 0.0;
            if (r != 0.0) { c = x / r; s = z / r; }
            if (j < bot) e[j] = r;
            double a = d[j], b = e[j - 1], a1 = d[j - 1];
            d[j] = c * c * a + 2.0 * c * s * b + s * s * a1;
            d[j - 1] = s * s * a - 2.0 * c * s * b + c * c * a1;
            e[j - 1] = c * s * (a1 - a) + (c * c - s * s) * b;
            if (j > top + 1) {
                x = e[j - 1];
                z = s * e[j - 2];
                e[j - 2] = c * e[j - 2];
            }
            if (Z) {
                double *zj = Z + j * ldz, *zj1 = Z + (j - 1) * ldz;
                for (long i = 0; i < ldz; i++) {
                    double u = zj[i], w = zj1[i];
                    zj[i] = c * u + s * w;
                    zj1[i] = -s * u + c * w;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Inverse iteration on the tridiagonal T (d, e) for the k eigenvalues lam[] */
/* (ascending).  Each solve of (T - lam I) x = b uses Gaussian elimination    */
/* with partial pivoting; vectors whose eigenvalues are closer than           */
/* 1e-3 ||T||_1 are Gram-Schmidt orthogonalised against one another.          */
/* Z: column-major n x k, unit 2-norm columns.                                */
/* ------------------------------------------------------------------------ */
static void orc_tri_solve_shifted(long n, const double *d, const double *e,
                                  double lam, double tiny, double *b,
                                  double *u0, double *u1, double *u2, double *l,
                                  int *swp)
{
    /* Factor P (T - lam I) = L U, U upper with two superdiagonals. */
    double a = d[0] - lam, c = (n > 1) ? e[0] : 0.0, c2 = 0.0;
    for (long i = 0; i < n - 1; i++) {
        double sub = e[i];                    /* entry (i+1, i) */
        double nd = d[i + 1] - lam;
        double nc = (i + 1 < n - 1) ? e[i + 1] : 0.0;
        if (fabs(a) >= fabs(sub)) {           /* no interchange */
            if (a == 0.0) a = tiny;
            double m = sub / a;
            u0[i] = a; u1[i] = c; u2[i] = c2; l[i] = m; swp[i] = 0;
            a = nd - m * c;
            c = nc - m * c2;
            c2 = 0.0;
        } else {                              /* swap rows i and i+1 */
            double m = a / sub;
            u0[i] = sub; u1[i] = nd; u2[i] = nc; l[i] = m; swp[i] = 1;
            a = c - m * nd;
            c = c2 - m * nc;
            c2 = 0.0;
        }
    }
    if (a == 0.0) a = tiny;
    u0[n - 1] = a;
    /* forward: apply the row operations to b */
    for (long i = 0; i < n - 1; i++) {
        if (swp[i]) { double t = b[i]; b[i] = b[i + 1]; b[i + 1] = t; }
        b[i + 1] -= l[i] * b[i];
    }
    /* back substitution with U */
    for (long i = n - 1; i >= 0; i--) {
        double s = b[i];
        if (i + 1 < n) s -= u1[i] * b[i + 1];
        if (i + 2 < n) s -= u2[i] * b[i + 2];
        b[i] = s / u0[i];
    }
}

void orc_tridiag_invit(long n, const double *d, const double *e, long k,
                       const double *lam, double *Z)
{
    double tn = 0.0;                          /* ||T||_1 */
    for (long i = 0; i < n; i++) {
        double s = fabs(d[i]);
        if (i > 0) s += fabs(e[i - 1]);
        if (i < n - 1) s += fabs(e[i]);
        if (s > tn) tn = s;
    }
    double ortol = 1e-3 * tn;
    double tiny = DBL_EPSILON * (tn > 0 ? tn : 1.0);
    double *u0 = malloc(sizeof(double) * n), *u1 = malloc(sizeof(double) * n);
    double *u2 = malloc(sizeof(double) * n), *l = malloc(sizeof(double) * n);
    int *swp = malloc(sizeof(int) * n);
    uint64_t st = 0x0123456789ABCDEFULL;      /* fixed start vectors */
    long cstart = 0;                          /* first index of current cluster */
    for (long j = 0; j < k; j++) {
        if (j > 0 && lam[j] - lam[j - 1] > ortol) cstart = j;
        double *x = Z + j * n;
        for (long i = 0; i < n; i++) {
            uint64_t z = orc_splitmix64_next(&st);
            x[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        for (int it = 0; it < 5; it++) {
            orc_tri_solve_shifted(n, d, e, lam[j], tiny, x, u0, u1, u2, l, swp);
            for (long q = cstart; q < j; q++) {   /* Gram-Schmidt in the cluster */
                const double *y = Z + q * n;
                double dot = 0.0;
                for (long i = 0; i < n; i++) dot += y[i] * x[i];
                for (long i = 0; i < n; i++) x[i] -= dot * y[i];
            }
            double nrm = 0.0;
            for (long i = 0; i < n; i++) nrm += x[i] * x[i];
            nrm = sqrt(nrm);
            for (long i = 0; i < n; i++) x[i] /= nrm;
        }
    }
    free(u0); free(u1); free(u2); free(l); free(swp);
}

/* psi = Q z with Q = H_0 H_1 ... H_{n-3} from orc_tridiagonalize. */
void orc_backtransform(long n, const double *A, const double *tau, long k,
                       double *Z)
{
    for (long j = 0; j < k; j++) {
        double *z = Z + j * n;
        for (long q = n - 3; q >= 0; q--) {
            if (tau[q] == 0.0) continue;
            const double *v = A + q * n;      /* v(q+1) = 1, v(q+2..) stored */
            double dot = z[q + 1];
            for (long i = q + 2; i < n; i++) dot += v[i] * z[i];
            dot *= tau[q];
            z[q + 1] -= dot;
            for (long i = q + 2; i < n; i++) z[i] -= dot * v[i];
        }
    }
}

static int orc_cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* All eigenvalues (ascending) of a symmetric n x n matrix; A is destroyed. */
int orc_eigvalsh(long n, double *A, double *w)
{
    double *e = malloc(sizeof(double) * (n > 1 ? n : 1));
    double *tau = malloc(sizeof(double) * (n > 1 ? n : 1));
    if (n >= 2) orc_tridiagonalize(n, A, w, e, tau, -1);
    else if (n == 1) w[0] = A[0];
    int rc = (n >= 2) ? orc_tridiag_ql(n, w, e, NULL, 0) : 0;
    qsort(w, (size_t)n, sizeof(double), orc_cmp_double);
    free(e); free(tau);
    return rc;
}

/* All eigenpairs by accumulating the rotations (small n only):
 * Z = Q_householder * R^T...; columns sorted ascending by eigenvalue. */
int orc_eigh_full(long n, double *A, double *w, double *Z)
{
    double *e = malloc(sizeof(double) * (n > 1 ? n : 1));
    double *tau = malloc(sizeof(double) * (n > 1 ? n : 1));
    double *Q = malloc(sizeof(double) * (size_t)n * (size_t)n);
    if (n == 1) { w[0] = A[0]; Z[0] = 1.0; free(e); free(tau); free(Q); return 0; }
    orc_tridiagonalize(n, A, w, e, tau, -1);
    /* Q = H_0 ... H_{n-3}: apply to the identity column by column */
    memset(Q, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (long i = 0; i < n; i++) Q[i * n + i] = 1.0;
    orc_backtransform(n, A, tau, n, Q);
    int rc = orc_tridiag_ql(n, w, e, Q, n);
    /* selection sort of eigenpairs, ascending */
    for (long i = 0; i < n; i++) {
        long m = i;
        for (long j = i + 1; j < n; j++) if (w[j] < w[m]) m = j;
        if (m != i) {
            double t = w[i]; w[i] = w[m]; w[m] = t;
            for (long r = 0; r < n; r++) {
                double u = Q[i * n + r]; Q[i * n + r] = Q[m * n + r]; Q[m * n + r] = u;
            }
        }
    }
    memcpy(Z, Q, sizeof(double) * (size_t)n * (size_t)n);
    free(e); free(tau); free(Q);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The eigenpairs nearest the target (section "Numerical method").           */
/*   sigma = E_min + eps (E_max - E_min) unless sigma_in is finite;          */
/*   the nev eigenvalues with smallest |lambda - sigma| (ties: lower first)  */
/*   are returned ascending, with unit eigenvectors if evecs != NULL.        */
/* H: dense symmetric dim x dim (destroyed).  all_evals (optional) receives  */
/* the full ascending spectrum.  Returns 0 on success.                       */
/* ------------------------------------------------------------------------ */
typedef struct { double dist, lam; } orc_pair;

static int orc_cmp_pair(const void *a, const void *b)
{
    const orc_pair *x = a, *y = b;
    if (x->dist < y->dist) return -1;
    if (x->dist > y->dist) return 1;
    return (x->lam > y->lam) - (x->lam < y->lam);
}

int orc_nearest_eigenpairs_multi(long dim, double *H, long nt, const double *eps,
                                 const double *sigma_in, long nev, double *evals,
                                 double *evecs, double *all_evals, double *out3)
{
    double *d = malloc(sizeof(double) * dim), *e = malloc(sizeof(double) * dim);
    double *tau = malloc(sizeof(double) * dim), *w = malloc(sizeof(double) * dim);
    double *ew = malloc(sizeof(double) * dim);
    orc_pair *pr = malloc(sizeof(orc_pair) * dim);
    int rc = 0;
    if (dim == 1) d[0] = H[0];
    else orc_tridiagonalize(dim, H, d, e, tau, -1);
    memcpy(w, d, sizeof(double) * dim);
    memcpy(ew, e, sizeof(double) * dim);
    if (dim > 1) rc = orc_tridiag_ql(dim, w, ew, NULL, 0);
    qsort(w, (size_t)dim, sizeof(double), orc_cmp_double);
    double emin = w[0], emax = w[dim - 1];
    if (all_evals) memcpy(all_evals, w, sizeof(double) * dim);
    for (long t = 0; t < nt; t++) {
        double sg = sigma_in ? sigma_in[t] : NAN;
        double sigma = isfinite(sg) ? sg : emin + eps[t] * (emax - emin);
        double *ev = evals + t * nev;
        for (long i = 0; i < dim; i++) { pr[i].dist = fabs(w[i] - sigma); pr[i].lam = w[i]; }
        qsort(pr, (size_t)dim, sizeof(orc_pair), orc_cmp_pair);
        for (long i = 0; i < nev; i++) ev[i] = pr[i].lam;
        qsort(ev, (size_t)nev, sizeof(double), orc_cmp_double);
        if (out3) { out3[3 * t] = emin; out3[3 * t + 1] = emax; out3[3 * t + 2] = sigma; }
        if (evecs) {
            double *Z = evecs + t * nev * dim;
            if (dim == 1) Z[0] = 1.0;
            else {
                orc_tridiag_invit(dim, d, e, nev, ev, Z);
                orc_backtransform(dim, H, tau, nev, Z);
                for (long j = 0; j < nev; j++) {     /* normalise in FP64 */
                    double *z = Z + j * dim, s = 0.0;
                    for (long i = 0; i < dim; i++) s += z[i] * z[i];
                    s = sqrt(s);
                    for (long i = 0; i < dim; i++) z[i] /= s;
                }
            }
        }
    }
    free(d); free(e); free(tau); free(w); free(pr); free(ew);
    return rc;
}

int orc_nearest_eigenpairs(long dim, double *H, double eps, double sigma_in,
                           long nev, double *evals, double *evecs,
                           double *all_evals, double *out3)
{
    return orc_nearest_eigenpairs_multi(dim, H, 1, &eps, &sigma_in, nev, evals,
                                        evecs, all_evals, out3);
}

/* ------------------------------------------------------------------------ */
/* Observables.                                                              */
/* ------------------------------------------------------------------------ */

/* Gap ratios of ascending levels E[0..n-1]: delta_m = E_m - E_{m-1},
 * r = min(delta_m, delta_{m+1}) / max(...), m = 1..n-2 (item (i)).
 * NaN when both gaps vanish.  Returns the mean over finite entries. */
double orc_gap_ratios(long n, const double *E, double *r)
{
    double sum = 0.0;
    long cnt = 0;
    for (long m = 1; m + 1 < n; m++) {
        double a = E[m] - E[m - 1], b = E[m + 1] - E[m];
        double mx = a > b ? a : b, mn = a > b ? b : a;
        double v = (mx > 0.0) ? mn / mx : NAN;
        r[m - 1] = v;
        if (!isnan(v)) { sum += v; cnt++; }
    }
    return cnt ? sum / (double)cnt : NAN;
}

/* Participation entropy S^P_q of a state (item (iii)); p_i = psi_i^2 /
 * sum psi^2.  q = 1 gives -sum p ln p.  States outside the sector have
 * p = 0 and contribute nothing. */
double orc_participation_entropy(long dim, const double *psi, double q)
{
    double nrm = 0.0;
    for (long i = 0; i < dim; i++) nrm += psi[i] * psi[i];
    if (q == 1.0) {
        double s = 0.0;
        for (long i = 0; i < dim; i++) {
            double p = psi[i] * psi[i] / nrm;
            if (p > 0.0) s -= p * log(p);
        }
        return s;
    }
    double s = 0.0;
    for (long i = 0; i < dim; i++) {
        double p = psi[i] * psi[i] / nrm;
        if (p > 0.0) s += pow(p, q);
    }
    return log(s) / (1.0 - q);
}

/* Half-chain entanglement entropy S_E = -Tr rho_A ln rho_A (item (ii)).
 * A = sites 1..L/2 = low bits b, B = high bits a.  M[a][b] = psi(s) with
 * s = (a << L/2) | b (zero outside the sector), rho_A = M^T M over the full
 * 2^{L/2}-dimensional subsystem space; its eigenvalues come from the same
 * dense symmetric eigensolver as the spectrum. */
double orc_entanglement_entropy(int L, const uint32_t *basis, long dim,
                                const double *psi)
{
    int la = L / 2;
    long na = 1L << la, nb = 1L << (L - la);
    double nrm = 0.0;
    for (long i = 0; i < dim; i++) nrm += psi[i] * psi[i];
    double *M = calloc((size_t)nb * (size_t)na, sizeof(double));  /* row a, col b: M[a*na + b] */
    for (long k = 0; k < dim; k++) {
        uint32_t s = basis[k];
        long b = s & (uint32_t)(na - 1), a = s >> la;
        M[a * na + b] = psi[k] / sqrt(nrm);
    }
    double *rho = calloc((size_t)na * (size_t)na, sizeof(double));
    for (long b1 = 0; b1 < na; b1++)
        for (long b2 = 0; b2 < na; b2++) {
            double acc = 0.0;
            for (long a = 0; a < nb; a++) acc += M[a * na + b1] * M[a * na + b2];
            rho[b2 * na + b1] = acc;
        }
    double *w = malloc(sizeof(double) * na);
    orc_eigvalsh(na, rho, w);
    double s = 0.0;
    for (long i = 0; i < na; i++) if (w[i] > 0.0) s -= w[i] * log(w[i]);
    free(M); free(rho); free(w);
    return s;
}

/* Bipartite fluctuations F = <(S^z_A)^2> - <S^z_A>^2, A = sites 1..L/2
 * (item (ii)); S^z_A is diagonal in the basis. */
double orc_bipartite_fluct(int L, const uint32_t *basis, long dim,
                           const double *psi)
{
    int la = L / 2;
    double nrm = 0.0, m1 = 0.0, m2 = 0.0;
    for (long k = 0; k < dim; k++) nrm += psi[k] * psi[k];
    for (long k = 0; k < dim; k++) {
        uint32_t s = basis[k];
        double sz = 0.0;
        for (int i = 0; i < la; i++) sz += ((s >> i) & 1u) ? 0.5 : -0.5;
        double p = psi[k] * psi[k] / nrm;
        m1 += p * sz;
        m2 += p * sz * sz;
    }
    return m2 - m1 * m1;
}

/* Kullback-Leibler divergence KL = sum_i p_i ln(p_i / q_i) between two states
 * (item (i)).  Terms with p_i = 0 contribute 0; a term with p_i > 0 and
 * q_i = 0 makes KL infinite. */
double orc_kl_divergence(long dim, const double *psi, const double *phi)
{
    double np = 0.0, nq = 0.0, s = 0.0;
    for (long i = 0; i < dim; i++) { np += psi[i] * psi[i]; nq += phi[i] * phi[i]; }
    for (long i = 0; i < dim; i++) {
        double p = psi[i] * psi[i] / np, q = phi[i] * phi[i] / nq;
        if (p > 0.0) {
            if (q == 0.0) return INFINITY;
            s += p * log(p / q);
        }
    }
    return s;
}

/* Dynamical spin fraction of an eigenstate (Supplementary material):
 * M = sum_{j=1..L} S^z_j exp(i 2 pi j / L) (site j = bit j-1),
 * f = 1 - <M^dag><M> / <M^dag M>.  M is diagonal in the basis, so
 * <M> = sum_s p_s m(s) and <M^dag M> = sum_s p_s |m(s)|^2. */
double orc_dynamical_fraction(int L, const uint32_t *basis, long dim,
                              const double *psi)
{
    double nrm = 0.0, re = 0.0, im = 0.0, mm = 0.0;
    for (long k = 0; k < dim; k++) nrm += psi[k] * psi[k];
    for (long k = 0; k < dim; k++) {
        uint32_t s = basis[k];
        double mr = 0.0, mi = 0.0;
        for (int j = 1; j <= L; j++) {
            double sz = ((s >> (j - 1)) & 1u) ? 0.5 : -0.5;
            double ang = 2.0 * M_PI * (double)j / (double)L;
            mr += sz * cos(ang);
            mi += sz * sin(ang);
        }
        double p = psi[k] * psi[k] / nrm;
        re += p * mr;
        im += p * mi;
        mm += p * (mr * mr + mi * mi);
    }
    return 1.0 - (re * re + im * im) / mm;
}

/* ||H psi - E psi||_2 for a unit psi, with H applied by orc_apply_H. */
double orc_residual(int L, double J, const double *fields, const uint32_t *basis,
                    long dim, const double *psi, double E)
{
    double *y = malloc(sizeof(double) * dim);
    orc_apply_H(L, J, fields, basis, dim, psi, y);
    double s = 0.0;
    for (long i = 0; i < dim; i++) { double t = y[i] - E * psi[i]; s += t * t; }
    free(y);
    return sqrt(s);
}

/* Rayleigh quotient psi^T H psi / psi^T psi. */
double orc_rayleigh(int L, double J, const double *fields, const uint32_t *basis,
                    long dim, const double *psi)
{
    double *y = malloc(sizeof(double) * dim);
    orc_apply_H(L, J, fields, basis, dim, psi, y);
    double a = 0.0, b = 0.0;
    for (long i = 0; i < dim; i++) { a += psi[i] * y[i]; b += psi[i] * psi[i]; }
    free(y);
    return a / b;
}
