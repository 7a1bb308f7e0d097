// k_obs.hip -- eigenvector observables on gfx950 (section "Characterization of
// ergodic and localized regimes"): participation entropies S_1, S_2 (item iii),
// half-chain entanglement entropy S_E (item ii), bipartite fluctuations F
// (item ii), Kullback-Leibler divergence of neighbouring eigenstates (item i),
// the dynamical spin fraction f (Supplementary material), and the gap ratio r
// (item i).
//
// S_E: with A = sites 1..L/2 (low bits b) and B the rest (high bits a), the
// amplitude matrix M[a][b] = psi(a b) vanishes unless popcount(a) + popcount(b)
// is the sector's up-spin count, so it is block diagonal over k = popcount(b):
// block k is C(L - L/2, nup - k) x C(L/2, k) and the blocks tile the sector
// exactly (Vandermonde).  The squared Schmidt values of psi are the squared
// singular values of these blocks, i.e. the eigenvalues of their Gram
// matrices.  Each (vector, block) is one workgroup: the Gram matrix, its
// Lanczos tridiagonalisation with full reorthogonalisation, Sturm bisection on
// the tridiagonal, and -sum lambda ln lambda over lambda = sigma^2 / |psi|^2.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"
#include "obs.hpp"

namespace mbl {
namespace {

__constant__ uint32_t o_binom[33][17];
bool g_obinom_ready = false;

void ensure_obinom() {
    if (g_obinom_ready) return;
    uint32_t t[33][17] = {};
    for (int n = 0; n <= 32; n++)
        for (int k = 0; k <= 16; k++) t[n][k] = (uint32_t)binom(n, k);
    MBL_HIP(hipMemcpyToSymbol(HIP_SYMBOL(o_binom), t, sizeof(t)));
    g_obinom_ready = true;
}

// Where each magnetization block of the reshaped vector lives: block k starts
// at off[k] of a vector's concatenated blocks (cnt_k lines of len_k values),
// and its Lanczos scratch (3 cnt_k^2 doubles) at goff[k] of a per-vector
// stride gstride.  Passed to the kernels by value.
struct SeLayout {
    int L = 0, nup = 0, la = 0;
    int64_t dim = 0, gstride = 0;
    int64_t off[MBL_L_MAX / 2 + 2] = {}, goff[MBL_L_MAX / 2 + 1] = {};
};

// index of word w among the words of its popcount (colex = ascending order)
__device__ __forceinline__ int sub_rank(uint32_t w) {
    int r = 0, j = 1;
    while (w) {
        int c = __ffs(w) - 1;
        r += o_binom[c][j];
        j++;
        w &= w - 1;
    }
    return r;
}

// destination of each sector state in the concatenated blocks: block k holds
// the states with k up spins in A (the low la = L / 2 bits b), nr = C(L - la,
// nup - k) rows a by d = C(la, k) columns b, stored as the fewer of the two
// kinds of lines, each contiguous (row-major if nr <= d, else column-major)
__global__ void k_block_index(SeLayout lay, const uint32_t *basis, int32_t *dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= lay.dim) return;
    const int la = lay.la, lb = lay.L - la, nup = lay.nup;
    uint32_t s = basis[i];
    uint32_t b = s & ((1u << la) - 1u), a = s >> la;
    int k = __popc(b);
    int d = (int)o_binom[la][k];
    int nr = (int)o_binom[lb][nup - k];
    int ra = sub_rank(a), rb = sub_rank(b);
    int64_t o = (nr <= d) ? (int64_t)ra * d + rb : (int64_t)rb * nr + ra;
    dst[i] = (int32_t)(lay.off[k] + o);
}

__global__ void k_scatter_blocks(int64_t dim, int nvec, const int32_t *dst, const double *psi,
                                 int64_t ldpsi, double *M) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dim) return;
    int32_t o = dst[i];
    for (int v = 0; v < nvec; v++) M[(int64_t)v * dim + o] = psi[(int64_t)v * ldpsi + i];
}

constexpr int SEB = 256;

__device__ double block_reduce_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = SEB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

constexpr int SGT = 1024;                 // threads of an S_E workgroup
constexpr int SGW = SGT / 64;             // its wavefronts
constexpr int SG_MAXN = 512;              // longest line (C(11, 5) = 462 at L = 22)
constexpr int SG_LDSG = 96;               // Gram matrices up to this order live in LDS
constexpr int SG_PARTS = 4;               // partial sums per output in the Lanczos passes

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the workgroup, same value in every thread
__device__ __forceinline__ double group_sum(double v, double *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < SGW; q++) t += red[q];
    __syncthreads();
    return t;
}

// Components in [-1/2, 1/2) of the start / restart vectors: SplitMix64
// (Steele, Lea, Flood 2014) of a key per (block, draw) and the index.
__device__ __forceinline__ double gkl_rand(uint64_t key, int i) {
    uint64_t z = key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// sum_{t < n} A[t sa] B[t sb] with four partial sums, unrolled so that the
// loads of several terms are in flight at once (the operands sit in L2 / LDS
// and the loop would otherwise wait one round trip per term)
__device__ __forceinline__ double dot_s(const double *A, int64_t sa, const double *B, int64_t sb,
                                        int n) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int t = 0;
#pragma unroll 2
    for (; t + 4 <= n; t += 4) {
        a0 += A[(int64_t)t * sa] * B[(int64_t)t * sb];
        a1 += A[(int64_t)(t + 1) * sa] * B[(int64_t)(t + 1) * sb];
        a2 += A[(int64_t)(t + 2) * sa] * B[(int64_t)(t + 2) * sb];
        a3 += A[(int64_t)(t + 3) * sa] * B[(int64_t)(t + 3) * sb];
    }
    for (; t < n; t++) a0 += A[(int64_t)t * sa] * B[(int64_t)t * sb];
    return (a0 + a1) + (a2 + a3);
}

// y[r] = sum_{c < nc} A[c lda + r] x[c] for r < nr (A in global or LDS, x and
// y in LDS): each output is split over SG_PARTS threads, each summing a
// contiguous quarter of c (so a pass is a few batches of loads per thread),
// and the quarters are added in a fixed order.  sign = -1 subtracts from y.
__device__ void pass_sum(const double *A, int64_t lda, const double *x, int nr, int nc,
                         double *y, double sign, double *pbuf) {
    const int chunk = (nc + SG_PARTS - 1) / SG_PARTS;
    for (int t = threadIdx.x; t < nr * SG_PARTS; t += SGT) {
        const int r = t % nr, part = t / nr;
        const int c0 = part * chunk, c1 = min(nc, c0 + chunk);
        pbuf[part * SG_MAXN + r] = c1 > c0 ? dot_s(A + (int64_t)c0 * lda + r, lda, x + c0, 1, c1 - c0) : 0.0;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += SGT) {
        double a = 0.0;
        for (int part = 0; part < SG_PARTS; part++) a += pbuf[part * SG_MAXN + r];
        y[r] = (sign > 0.0) ? a : y[r] - a;
    }
    __syncthreads();
}

// Orthogonalise x (length n, LDS) against the k orthonormal vectors of Q,
// classical Gram-Schmidt applied twice.  Q is kept in two layouts so that both
// halves of a pass read coalesced: Qt (component e of every vector at Qt + e
// ld) for the coefficients, Qv (vector q at Qv + q ld) for the update.
__device__ void lz_orth(double *x, int n, const double *Qv, const double *Qt, int ld, int k,
                        double *coef, double *pbuf) {
    for (int pass = 0; pass < 2 && k > 0; pass++) {
        pass_sum(Qt, ld, x, k, n, coef, 1.0, pbuf);      // coef = Q^T x
        pass_sum(Qv, ld, coef, n, k, x, -1.0, pbuf);     // x -= Q coef
    }
}

// x <- x / |x| if |x| > tiny; otherwise x <- a fresh direction orthogonal to
// the k vectors of Q (random, key).  Returns |x|, or 0 for a fresh direction.
__device__ double lz_normalize(double *x, int n, const double *Qv, const double *Qt, int ld,
                               int k, double tiny, uint64_t key, double *coef, double *red,
                               double *pbuf) {
    auto norm2 = [&] {
        double a = 0.0;
        for (int e = threadIdx.x; e < n; e += SGT) a += x[e] * x[e];
        return group_sum(a, red);
    };
    double nr = sqrt(norm2());
    double keep = nr;
    for (int draw = 0; nr <= tiny && draw < 4; draw++) {
        keep = 0.0;
        for (int e = threadIdx.x; e < n; e += SGT) x[e] = gkl_rand(key + 7919ULL * draw, e);
        __syncthreads();
        lz_orth(x, n, Qv, Qt, ld, k, coef, pbuf);
        nr = sqrt(norm2());
    }
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    for (int e = threadIdx.x; e < n; e += SGT) x[e] *= inv;
    __syncthreads();
    return keep;
}

// number of eigenvalues below x of the symmetric tridiagonal (a, b2 = squared
// off-diagonals), by the Sturm sequence of its LDL^T pivots
__device__ int tri_count(int m, const double *a, const double *b2, double x, double pivmin) {
    int c = 0;
    double q = a[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) c++;
    for (int i = 1; i < m; i++) {
        q = a[i] - x - b2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) c++;
    }
    return c;
}

// One workgroup per (vector, block): entropy contribution of block k of vector
// v.  The block M is cnt lines of length len (cnt <= len); the squared Schmidt
// values are the eigenvalues of its Gram matrix G = M M^T (cnt x cnt).  G is
// formed once, then reduced to a tridiagonal T = Q^T G Q by the Lanczos
// recurrence with full reorthogonalisation (a step whose new vector vanishes
// continues from a fresh orthogonal direction with a zero coupling, so after
// cnt steps Q is square and T has the eigenvalues of G), and the eigenvalues
// of T are found by Sturm bisection, one thread each.
// work: per (vector, block) 3 cnt^2 doubles (G, Q by vector, Q by component).
__global__ __launch_bounds__(SGT) void k_se_lanczos(SeLayout lay, const double *norms2,
                                                    const double *M, double *work, double *part) {
    __shared__ double xw[SG_MAXN], qj[SG_MAXN], qp[SG_MAXN], coef[SG_MAXN];
    __shared__ double al[SG_MAXN], b2[SG_MAXN];
    __shared__ double red[SGW];
    __shared__ double Gl[SG_LDSG * SG_LDSG];      // G itself when cnt <= SG_LDSG
    __shared__ double pbuf[SG_PARTS * SG_MAXN];   // partial sums of the passes
    const int la = lay.la, lb = lay.L - la, nup = lay.nup;
    const int v = blockIdx.x / (la + 1), k = blockIdx.x % (la + 1);
    const int d = (int)o_binom[la][k];
    const int nr = (nup - k >= 0 && nup - k <= lb) ? (int)o_binom[lb][nup - k] : 0;
    const int cnt = min(nr, d), len = max(nr, d);
    if (cnt == 0) {                               // no state of the sector in this block
        if (threadIdx.x == 0) part[blockIdx.x] = 0.0;
        return;
    }
    const double *X = M + (int64_t)v * lay.dim + lay.off[k];
    double *Gw = work + (int64_t)v * lay.gstride + lay.goff[k];
    double *Qv = Gw + (int64_t)cnt * cnt, *Qt = Qv + (int64_t)cnt * cnt;
    double *G = (cnt <= SG_LDSG) ? Gl : Gw;
    // G = X X^T, register tiles of 2 x 2 entries (upper triangle, mirrored)
    const int nt = (cnt + 1) / 2;
    for (int t = threadIdx.x; t < nt * nt; t += SGT) {
        const int ti = t % nt, tj = t / nt;
        if (ti > tj) continue;
        const int i0 = 2 * ti, j0 = 2 * tj;
        const bool i1 = i0 + 1 < cnt, j1 = j0 + 1 < cnt;
        const double *xa = X + (int64_t)i0 * len, *xb = X + (int64_t)(i1 ? i0 + 1 : i0) * len;
        const double *ya = X + (int64_t)j0 * len, *yb = X + (int64_t)(j1 ? j0 + 1 : j0) * len;
        double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
#pragma unroll 4
        for (int e = 0; e < len; e++) {
            const double a0 = xa[e], a1 = xb[e], c0 = ya[e], c1 = yb[e];
            s00 += a0 * c0; s01 += a0 * c1; s10 += a1 * c0; s11 += a1 * c1;
        }
        G[(int64_t)j0 * cnt + i0] = s00; G[(int64_t)i0 * cnt + j0] = s00;
        if (j1) { G[(int64_t)(j0 + 1) * cnt + i0] = s01; G[(int64_t)i0 * cnt + j0 + 1] = s01; }
        if (i1) { G[(int64_t)j0 * cnt + i0 + 1] = s10; G[(int64_t)(i0 + 1) * cnt + j0] = s10; }
        if (i1 && j1) { G[(int64_t)(j0 + 1) * cnt + i0 + 1] = s11; G[(int64_t)(i0 + 1) * cnt + j0 + 1] = s11; }
    }
    double tr = 0.0;                               // trace of G = |M|^2
    for (int64_t e = threadIdx.x; e < (int64_t)cnt * len; e += SGT) tr += X[e] * X[e];
    tr = group_sum(tr, red);                       // (its barriers also publish G)
    // a new Lanczos vector below tiny counts as vanished
    const double tiny = 1e-13 * tr;
    // start vectors depend on the block only, so a vector's result does not
    // depend on which other vectors share the launch
    const uint64_t key = 0x5E5EC0DEULL + 0x100000001B3ULL * (uint64_t)k;
    for (int i = threadIdx.x; i < cnt; i += SGT) { qj[i] = gkl_rand(key, i); qp[i] = 0.0; }
    __syncthreads();
    lz_normalize(qj, cnt, Qv, Qt, cnt, 0, -1.0, key + 1, coef, red, pbuf);
    double bprev = 0.0;
    for (int j = 0; j < cnt; j++) {
        for (int i = threadIdx.x; i < cnt; i += SGT) {
            Qv[(int64_t)j * cnt + i] = qj[i];
            Qt[(int64_t)i * cnt + j] = qj[i];
        }
        __syncthreads();
        // w = G q_j (G symmetric: read by columns, coalesced)
        pass_sum(G, cnt, qj, cnt, cnt, xw, 1.0, pbuf);
        const double a = group_sum([&] {
            double t = 0.0;
            for (int i = threadIdx.x; i < cnt; i += SGT) t += qj[i] * xw[i];
            return t;
        }(), red);
        if (threadIdx.x == 0) al[j] = a;
        if (j + 1 == cnt) break;
        for (int i = threadIdx.x; i < cnt; i += SGT) xw[i] -= a * qj[i] + bprev * qp[i];
        __syncthreads();
        lz_orth(xw, cnt, Qv, Qt, cnt, j + 1, coef, pbuf);
        const double b = lz_normalize(xw, cnt, Qv, Qt, cnt, j + 1, tiny,
                                      key + 2 * (uint64_t)j + 3, coef, red, pbuf);
        if (threadIdx.x == 0) b2[j] = b * b;
        for (int i = threadIdx.x; i < cnt; i += SGT) { qp[i] = qj[i]; qj[i] = xw[i]; }
        bprev = b;
        __syncthreads();
    }
    __syncthreads();
    // Gershgorin interval of T, then bisection for every eigenvalue
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < cnt; i++) {
        const double r = (i > 0 ? sqrt(b2[i - 1]) : 0.0) + (i + 1 < cnt ? sqrt(b2[i]) : 0.0);
        lo = fmin(lo, al[i] - r);
        hi = fmax(hi, al[i] + r);
    }
    const double span = fmax(hi - lo, 1e-300);
    const double pivmin = 1e-300 + 1e-30 * span * span;
    const double inv = 1.0 / norms2[v];
    double ent = 0.0;
    for (int i = threadIdx.x; i < cnt; i += SGT) {
        double a = lo, c = hi;                      // count(a) <= i < count(c)
        for (int it = 0; it < 200 && c - a > 2.3e-16 * span; it++) {
            const double mid = 0.5 * (a + c);
            if (tri_count(cnt, al, b2, mid, pivmin) > i) c = mid; else a = mid;
        }
        const double lam = 0.5 * (a + c) * inv;
        if (lam > 0.0) ent -= lam * log(lam);
    }
    ent = group_sum(ent, red);
    if (threadIdx.x == 0) part[blockIdx.x] = ent;
}

__global__ void k_se_sum(int nblk, int nvec, const double *part, double *se) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    double s = 0.0;
    for (int k = 0; k < nblk; k++) s += part[v * nblk + k];
    se[v] = s;
}

// per-vector sums over the basis: |psi|^2, S_1 part, sum p^2, <S^z_A>, <(S^z_A)^2>,
// Re<M>, Im<M>, <|M|^2>, KL to the next vector
constexpr int NQ = 9;
constexpr int OBS_PARTS = 64;

__global__ __launch_bounds__(SEB) void k_vec_sums(int L, int64_t dim, int nvec,
                                                  const uint32_t *basis, const double *psi,
                                                  int64_t ld, const double *norms2, int pass,
                                                  double *part) {
    __shared__ double sh[SEB];
    int v = blockIdx.y;
    const double *x = psi + (int64_t)v * ld;
    const double *y = (v + 1 < nvec) ? psi + (int64_t)(v + 1) * ld : nullptr;
    double q[NQ];
    for (int j = 0; j < NQ; j++) q[j] = 0.0;
    double inv = (pass == 1) ? 1.0 / norms2[v] : 1.0;
    double invy = (pass == 1 && y) ? 1.0 / norms2[v + 1] : 1.0;
    int la = L / 2;
    for (int64_t i = (int64_t)blockIdx.x * SEB + threadIdx.x; i < dim;
         i += (int64_t)gridDim.x * SEB) {
        double a = x[i];
        q[0] += a * a;
        if (pass == 0) continue;
        double p = a * a * inv;
        if (p > 0.0) q[1] -= p * log(p);
        q[2] += p * p;
        uint32_t s = basis[i];
        double sza = (double)__popc(s & ((1u << la) - 1u)) - 0.5 * la;
        q[3] += p * sza;
        q[4] += p * sza * sza;
        double mr = 0.0, mi = 0.0;
        for (int j = 1; j <= L; j++) {
            double sz = ((s >> (j - 1)) & 1u) ? 0.5 : -0.5;
            double sn, cs;
            sincospi(2.0 * (double)j / (double)L, &sn, &cs);
            mr += sz * cs;
            mi += sz * sn;
        }
        q[5] += p * mr;
        q[6] += p * mi;
        q[7] += p * (mr * mr + mi * mi);
        if (y && p > 0.0) {
            double qq = y[i] * y[i] * invy;
            q[8] += (qq > 0.0) ? p * log(p / qq) : INFINITY;
        }
    }
    for (int j = 0; j < NQ; j++) {
        double r = block_reduce_sum(q[j], sh);
        if (threadIdx.x == 0) part[((int64_t)v * gridDim.x + blockIdx.x) * NQ + j] = r;
    }
}

__global__ void k_vec_final(int nvec, int nparts, const double *part, double *out, int pass) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    for (int j = 0; j < NQ; j++) {
        if (pass == 0 && j > 0) break;
        double s = 0.0;
        for (int b = 0; b < nparts; b++) s += part[((int64_t)v * nparts + b) * NQ + j];
        out[(int64_t)v * NQ + j] = s;
    }
}

__global__ void k_gap_ratio(int nev, const double *E, double *r) {
    int m = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (m + 1 >= nev) return;
    double a = E[m] - E[m - 1], b = E[m + 1] - E[m];
    double mx = fmax(a, b), mn = fmin(a, b);
    r[m - 1] = (mx > 0.0) ? mn / mx : NAN;
}

__global__ void k_stride_copy(int n, const double *src, int stride, double *dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[(int64_t)i * stride];
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

namespace {

SeLayout se_layout(int L) {
    SeLayout lay;
    lay.L = L;
    lay.la = L / 2;
    lay.nup = sector_nup(L);
    lay.dim = binom(L, lay.nup);
    const int la = lay.la, lb = L - la;
    for (int k = 0; k <= la; k++) {
        int64_t d = binom(la, k), nr = (lay.nup - k >= 0 && lay.nup - k <= lb) ? binom(lb, lay.nup - k) : 0;
        lay.off[k + 1] = lay.off[k] + nr * d;
        const int64_t cnt = std::min(nr, d), len = std::max(nr, d);
        MBL_REQUIRE(len <= SG_MAXN, MBL_EINVAL, "entanglement: subsystem block above 512");
        lay.goff[k] = lay.gstride;
        lay.gstride += 3 * cnt * cnt;               // G and the Lanczos basis in two layouts
    }
    MBL_REQUIRE(lay.off[la + 1] == lay.dim, MBL_EINVAL, "entanglement blocks do not cover the sector");
    return lay;
}

// S_E of nvec vectors psi (ld) into se_dev: scatter into blocks, bidiagonalise,
// sum the block entropies.  M: dim x nvec, gkl: gstride x nvec, part: (la + 1) nvec.
void se_launch(const SeLayout &lay, const int32_t *dst, const double *psi, int64_t ldpsi, int nvec,
               const double *norms2, double *M, double *gkl, double *part, double *se_dev,
               hipStream_t s) {
    const int la = lay.la;
    hipLaunchKernelGGL(k_scatter_blocks, dim3(cdiv(lay.dim, 256)), dim3(256), 0, s, lay.dim, nvec,
                       dst, psi, ldpsi, M);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_se_lanczos, dim3(nvec * (la + 1)), dim3(SGT), 0, s, lay, norms2, M, gkl, part);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_se_sum, dim3(cdiv(nvec, 64)), dim3(64), 0, s, la + 1, nvec, part, se_dev);
    MBL_CHECK_LAUNCH();
}

// Norms (pass 0), then S_1, S_2, F, f moments and KL (pass 1) of nvec vectors;
// out: NQ doubles per vector; nrm: nvec norms; part: OBS_PARTS NQ nvec.
void sums_launch(int L, int64_t dim, const uint32_t *basis, const double *psi, int64_t ld, int nvec,
                 double *part, double *nrm, double *out_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_vec_sums, dim3(OBS_PARTS, nvec), dim3(SEB), 0, s, L, dim, nvec, basis, psi,
                       ld, nrm, 0, part);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vec_final, dim3(cdiv(nvec, 64)), dim3(64), 0, s, nvec, OBS_PARTS, part,
                       out_dev, 0);
    MBL_CHECK_LAUNCH();
    // gather the norms (column 0 of out) into nrm
    hipLaunchKernelGGL(k_stride_copy, dim3(cdiv(nvec, 64)), dim3(64), 0, s, nvec, out_dev, NQ, nrm);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vec_sums, dim3(OBS_PARTS, nvec), dim3(SEB), 0, s, L, dim, nvec, basis, psi,
                       ld, nrm, 1, part);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vec_final, dim3(cdiv(nvec, 64)), dim3(64), 0, s, nvec, OBS_PARTS, part,
                       out_dev, 1);
    MBL_CHECK_LAUNCH();
}

}  // namespace

void ObsWork::prepare(int L_, const uint32_t *basis, int64_t dim_, int nvec_max, Budget *bud,
                      hipStream_t s) {
    ensure_obinom();
    if (L == L_ && dim == dim_ && nvec_max <= nvmax) return;
    const SeLayout lay = se_layout(L_);
    MBL_REQUIRE(lay.dim == dim_, MBL_EINVAL, "observables: sector dimension mismatch");
    // unprepared until every buffer is in place: DevBuf::alloc frees before it
    // allocates, so an allocation refused part way leaves empty buffers, and a
    // size recorded before it would let the next call skip straight to kernels
    // on them
    L = -1;
    dim = 0;
    nvmax = 0;
    gkl_stride_ = 0;
    d_dst.alloc(sizeof(int32_t) * dim_, bud);
    hipLaunchKernelGGL(k_block_index, dim3(cdiv(dim_, 256)), dim3(256), 0, s, lay, basis,
                       d_dst.ptr<int32_t>());
    MBL_CHECK_LAUNCH();
    d_M.alloc(sizeof(double) * dim_ * nvec_max, bud);
    d_gkl.alloc(sizeof(double) * lay.gstride * nvec_max, bud);
    d_part.alloc(sizeof(double) * (size_t)std::max<int64_t>((int64_t)(lay.la + 1) * nvec_max,
                                                            (int64_t)OBS_PARTS * NQ * nvec_max),
                 bud);
    d_out.alloc(sizeof(double) * NQ * nvec_max + sizeof(double) * 4 * nvec_max, bud);
    L = L_;
    dim = dim_;
    nvmax = nvec_max;
    gkl_stride_ = lay.gstride;
}

void ObsWork::release() {
    L = -1;
    dim = 0;
    nvmax = 0;
    gkl_stride_ = 0;
    for (DevBuf *b : {&d_dst, &d_M, &d_gkl, &d_part, &d_out}) b->reset();
}

void ObsWork::entanglement(const double *psi, int64_t ldpsi, int nvec, const double *norms2,
                           double *se_dev, hipStream_t s) {
    se_launch(se_layout(L), d_dst.ptr<int32_t>(), psi, ldpsi, nvec, norms2, d_M.ptr<double>(),
              d_gkl.ptr<double>(), d_part.ptr<double>(), se_dev, s);
}

void ObsWork::vector_sums(const uint32_t *basis, const double *psi, int64_t ld, int nvec,
                          double *out_dev, hipStream_t s) {
    // pass 0: norms; pass 1: everything else with the normalised weights
    sums_launch(L, dim, basis, psi, ld, nvec, d_part.ptr<double>(), d_out.ptr<double>() + NQ * nvmax,
                out_dev, s);
}

void ObsWork::gap_ratios(int nev, const double *E_dev, double *r_dev, hipStream_t s) {
    if (nev < 3) return;
    hipLaunchKernelGGL(k_gap_ratio, dim3(cdiv(nev, 64)), dim3(64), 0, s, nev, E_dev, r_dev);
    MBL_CHECK_LAUNCH();
}

// ---- allocation-free observables --------------------------------------------
// One fixed work array per device, for callers that cannot allocate device
// memory.  In host code the array's name stands for a host-side placeholder;
// its device address on each device comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[MBL_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[64] = {};

unsigned char *noalloc_scratch(int dev) {
    MBL_REQUIRE(dev >= 0 && dev < 64, MBL_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        MBL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_noalloc_ptr[dev]);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

void observables_noalloc(int L, int nev, const double *evals_dev, const double *psi_dev,
                         int64_t ld, double *r_dev, double *s1_dev, double *se_dev,
                         hipStream_t s) {
    MBL_REQUIRE(L >= 2 && L <= MBL_L_MAX, MBL_EINVAL, "L must satisfy 2 <= L <= 22");
    MBL_REQUIRE(nev >= 1 && nev <= MBL_NOALLOC_MAX_NEV, MBL_EINVAL,
                "mbl_observables_noalloc: nev must satisfy 1 <= nev <= 256");
    MBL_REQUIRE(psi_dev != nullptr, MBL_EINVAL, "mbl_observables_noalloc: evecs_dev is NULL");
    MBL_REQUIRE(!r_dev || evals_dev, MBL_EINVAL, "mbl_observables_noalloc: r needs evals_dev");
    const SeLayout lay = se_layout(L);
    const int64_t dim = lay.dim;
    MBL_REQUIRE(ld >= dim, MBL_EINVAL, "mbl_observables_noalloc: ld below the sector dimension");
    int dev = 0;
    MBL_HIP(hipGetDevice(&dev));
    unsigned char *base = noalloc_scratch(dev);
    ensure_obinom();
    // layout of the work array
    const int nmax = MBL_NOALLOC_MAX_NEV;
    size_t o = 0;
    uint32_t *basis = reinterpret_cast<uint32_t *>(base + o);  o += align256(sizeof(uint32_t) * dim);
    int32_t *dst = reinterpret_cast<int32_t *>(base + o);      o += align256(sizeof(int32_t) * dim);
    double *part = reinterpret_cast<double *>(base + o);       o += align256(sizeof(double) * OBS_PARTS * NQ * nmax);
    double *out = reinterpret_cast<double *>(base + o);        o += align256(sizeof(double) * NQ * nmax);
    double *nrm = reinterpret_cast<double *>(base + o);        o += align256(sizeof(double) * nmax);
    double *separt = reinterpret_cast<double *>(base + o);     o += align256(sizeof(double) * (MBL_L_MAX / 2 + 1) * nmax);
    MBL_REQUIRE(o < MBL_NOALLOC_SCRATCH_BYTES, MBL_EINVAL,
                "mbl_observables_noalloc: sector too large for the fixed work array");
    // vectors whose entanglement blocks and bidiagonalisation fit at once
    const size_t per_vec = sizeof(double) * (size_t)(dim + lay.gstride);
    const int64_t chunk = std::min<int64_t>(nev, (int64_t)((MBL_NOALLOC_SCRATCH_BYTES - o) / per_vec));
    MBL_REQUIRE(!se_dev || chunk >= 1, MBL_EINVAL,
                "mbl_observables_noalloc: one vector's entanglement work exceeds the fixed work array");
    double *M = reinterpret_cast<double *>(base + o);
    double *gkl = M + (chunk > 0 ? chunk : 0) * dim;

    launch_basis(L, dim, basis, s);
    hipLaunchKernelGGL(k_block_index, dim3(cdiv(dim, 256)), dim3(256), 0, s, lay, basis, dst);
    MBL_CHECK_LAUNCH();
    sums_launch(L, dim, basis, psi_dev, ld, nev, part, nrm, out, s);
    if (s1_dev) {
        hipLaunchKernelGGL(k_stride_copy, dim3(cdiv(nev, 64)), dim3(64), 0, s, nev, out + 1, NQ, s1_dev);
        MBL_CHECK_LAUNCH();
    }
    if (r_dev && nev >= 3) {
        hipLaunchKernelGGL(k_gap_ratio, dim3(cdiv(nev, 64)), dim3(64), 0, s, nev, evals_dev, r_dev);
        MBL_CHECK_LAUNCH();
    }
    if (se_dev)
        for (int64_t v0 = 0; v0 < nev; v0 += chunk) {
            const int cv = (int)std::min<int64_t>(chunk, nev - v0);
            se_launch(lay, dst, psi_dev + v0 * ld, ld, cv, nrm + v0, M, gkl, separt, se_dev + v0, s);
        }
}

}  // namespace mbl
