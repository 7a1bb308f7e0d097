// k_obs.hip -- eigenvector observables on gfx950 (section "Characterization of
// ergodic and localized regimes"): participation entropies S_1, S_2 (item iii),
// half-chain entanglement entropy S_E (item ii), bipartite fluctuations F
// (item ii), Kullback-Leibler divergence of neighbouring eigenstates (item i),
// the dynamical spin fraction f (Supplementary material), and the gap ratio r
// (item i).
//
// S_E: with A = sites 1..L/2 (low bits b) and B the rest (high bits a), the
// amplitude matrix M[a][b] = psi(a b) vanishes unless popcount(a) + popcount(b)
// = L/2, so it is block diagonal over k = popcount(b): block k is
// C(L/2, k) x C(L/2, k) and the blocks tile the sector exactly (Vandermonde).
// rho_A is the direct sum of G_k = M_k^T M_k.  Each (vector, block) is one
// workgroup: Gram matrix, Householder tridiagonalisation, then all eigenvalues
// by Sturm-sequence bisection in parallel, and -sum lambda ln lambda.
#include <cmath>

#include "common.hpp"
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

// destination of each sector state in the concatenated blocks (row a, col b,
// row-major): block k holds the states with k up spins in A (the low la =
// L / 2 bits b), C(L - la, nup - k) rows a by C(la, k) columns b
__global__ void k_block_index(int L, int64_t dim, const uint32_t *basis, const int64_t *blockoff,
                              int32_t *dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dim) return;
    int la = L / 2;
    uint32_t s = basis[i];
    uint32_t b = s & ((1u << la) - 1u), a = s >> la;
    int k = __popc(b);
    int d = (int)o_binom[la][k];
    dst[i] = (int32_t)(blockoff[k] + (int64_t)sub_rank(a) * d + sub_rank(b));
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

// Sturm count: number of eigenvalues of the tridiagonal (d, e) below x
__device__ int sturm_count(int n, const double *d, const double *e2, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) cnt++;
    for (int i = 1; i < n; i++) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) cnt++;
    }
    return cnt;
}

// one workgroup per (vector, block): entropy contribution of block k of vector v
// (rows a: the nup - k up spins of B among L - la sites; columns b: the k up
// spins of A; square for even L, one site more on the B side for odd L)
__global__ __launch_bounds__(SEB) void k_se_block(int L, int nup, int nvec, int64_t dim,
                                                  const int64_t *blockoff, const double *norms2,
                                                  const double *M,
                                                  double *scratch, int64_t scratch_stride,
                                                  double *part) {
    __shared__ double sh[SEB];
    __shared__ double dd[512], ee[512], e2[512], vv[512], pp[512];
    const int la = L / 2, lb = L - la;
    int v = blockIdx.x / (la + 1), k = blockIdx.x % (la + 1);
    int d = (int)o_binom[la][k];
    int nr = (nup - k >= 0 && nup - k <= lb) ? (int)o_binom[lb][nup - k] : 0;
    if (nr == 0 || d == 0) {                      // no state of the sector in this block
        if (threadIdx.x == 0) part[blockIdx.x] = 0.0;
        return;
    }
    const double *Mk = M + (int64_t)v * dim + blockoff[k];   // nr x d, row a, col b
    double *G = scratch + (int64_t)blockIdx.x * scratch_stride;  // d x d column-major
    // Gram G = Mk^T Mk (the reduced density matrix of A on this block)
    for (int e = threadIdx.x; e < d * d; e += SEB) {
        int i = e % d, j = e / d;
        double s = 0.0;
        for (int a = 0; a < nr; a++) s += Mk[(int64_t)a * d + i] * Mk[(int64_t)a * d + j];
        G[e] = s;
    }
    __syncthreads();
    // Householder tridiagonalisation of G (full symmetric storage)
    for (int c = 0; c + 2 < d; c++) {
        int mm = d - c - 1;
        double sig = 0.0;
        for (int i = 1 + threadIdx.x; i < mm; i += SEB) {
            double x = G[(c + 1 + i) + (int64_t)c * d];
            sig += x * x;
        }
        sig = block_reduce_sum(sig, sh);
        double alpha = G[(c + 1) + (int64_t)c * d];
        if (threadIdx.x == 0) dd[c] = G[c + (int64_t)c * d];
        if (sig == 0.0) {
            if (threadIdx.x == 0) ee[c] = alpha;
            __syncthreads();
            continue;
        }
        double nrm = sqrt(alpha * alpha + sig);
        double beta = (alpha <= 0.0) ? nrm : -nrm;
        double tau = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int i = threadIdx.x; i < mm; i += SEB)
            vv[i] = (i == 0) ? 1.0 : G[(c + 1 + i) + (int64_t)c * d] * scal;
        if (threadIdx.x == 0) ee[c] = beta;
        __syncthreads();
        // p = tau * B v with B = G[c+1.., c+1..]
        for (int i = threadIdx.x; i < mm; i += SEB) {
            double s = 0.0;
            for (int j = 0; j < mm; j++) s += G[(c + 1 + i) + (int64_t)(c + 1 + j) * d] * vv[j];
            pp[i] = tau * s;
        }
        __syncthreads();
        double pv = 0.0;
        for (int i = threadIdx.x; i < mm; i += SEB) pv += pp[i] * vv[i];
        pv = block_reduce_sum(pv, sh);
        double K = 0.5 * tau * pv;
        for (int i = threadIdx.x; i < mm; i += SEB) pp[i] -= K * vv[i];
        __syncthreads();
        for (int e = threadIdx.x; e < mm * mm; e += SEB) {
            int i = e % mm, j = e / mm;
            G[(c + 1 + i) + (int64_t)(c + 1 + j) * d] -= vv[i] * pp[j] + pp[i] * vv[j];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (d >= 2) {
            dd[d - 2] = G[(d - 2) + (int64_t)(d - 2) * d];
            ee[d - 2] = G[(d - 1) + (int64_t)(d - 2) * d];
        }
        dd[d - 1] = G[(d - 1) + (int64_t)(d - 1) * d];
    }
    __syncthreads();
    // bisection for every eigenvalue, in parallel
    double lo = 1e300, hi = -1e300, tmax = 0.0;
    for (int i = 0; i < d; i++) {
        double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < d ? fabs(ee[i]) : 0.0);
        lo = fmin(lo, dd[i] - r);
        hi = fmax(hi, dd[i] + r);
        tmax = fmax(tmax, fabs(dd[i]) + r);
    }
    for (int i = threadIdx.x; i + 1 < d; i += SEB) e2[i] = ee[i] * ee[i];
    __syncthreads();
    double pivmin = 1e-300 + 1e-30 * tmax * tmax;
    double ent = 0.0;
    for (int idx = threadIdx.x; idx < d; idx += SEB) {
        double a = lo, b = hi;
        for (int it = 0; it < 100 && b - a > 4e-17 * fmax(tmax, 1e-300); it++) {
            double mid = 0.5 * (a + b);
            if (sturm_count(d, dd, e2, mid, pivmin) > idx) b = mid; else a = mid;
        }
        double lam = 0.5 * (a + b) / norms2[v];
        if (lam > 0.0) ent -= lam * log(lam);
    }
    ent = block_reduce_sum(ent, sh);
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

void ObsWork::prepare(int L_, const uint32_t *basis, int64_t dim_, int nvec_max, Budget *bud,
                      hipStream_t s) {
    ensure_obinom();
    if (L == L_ && dim == dim_ && nvec_max <= nvmax) return;
    L = L_;
    dim = dim_;
    nvmax = nvec_max;
    const int la = L / 2, lb = L - la, nup = sector_nup(L);
    std::vector<int64_t> off(la + 2, 0);
    int64_t maxd = 0;
    for (int k = 0; k <= la; k++) {
        int64_t d = binom(la, k), nr = (nup - k >= 0 && nup - k <= lb) ? binom(lb, nup - k) : 0;
        off[k + 1] = off[k] + nr * d;
        maxd = std::max(maxd, d);
    }
    MBL_REQUIRE(off[la + 1] == dim_, MBL_EINVAL, "entanglement blocks do not cover the sector");
    maxd_ = maxd;
    d_blockoff.alloc(sizeof(int64_t) * (la + 2), bud);
    h2d(d_blockoff.ptr<int64_t>(), off.data(), off.size(), s);
    d_dst.alloc(sizeof(int32_t) * dim, bud);
    hipLaunchKernelGGL(k_block_index, dim3(cdiv(dim, 256)), dim3(256), 0, s, L, dim, basis,
                       d_blockoff.ptr<int64_t>(), d_dst.ptr<int32_t>());
    MBL_CHECK_LAUNCH();
    d_M.alloc(sizeof(double) * dim * nvmax, bud);
    d_scratch.alloc(sizeof(double) * maxd * maxd * (la + 1) * nvmax, bud);
    d_part.alloc(sizeof(double) * (size_t)std::max<int64_t>((int64_t)(la + 1) * nvmax,
                                                            (int64_t)OBS_PARTS * NQ * nvmax), bud);
    d_out.alloc(sizeof(double) * NQ * nvmax + sizeof(double) * 4 * nvmax, bud);
}

void ObsWork::entanglement(const double *psi, int64_t ldpsi, int nvec, const double *norms2,
                           double *se_dev, hipStream_t s) {
    int la = L / 2;
    hipLaunchKernelGGL(k_scatter_blocks, dim3(cdiv(dim, 256)), dim3(256), 0, s, dim, nvec,
                       d_dst.ptr<int32_t>(), psi, ldpsi, d_M.ptr<double>());
    MBL_CHECK_LAUNCH();
    MBL_REQUIRE(maxd_ <= 512, MBL_EINVAL, "entanglement: subsystem block above 512");
    hipLaunchKernelGGL(k_se_block, dim3(nvec * (la + 1)), dim3(SEB), 0, s, L, sector_nup(L), nvec, dim,
                       d_blockoff.ptr<int64_t>(), norms2, d_M.ptr<double>(), d_scratch.ptr<double>(),
                       (int64_t)(maxd_ * maxd_), d_part.ptr<double>());
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_se_sum, dim3(cdiv(nvec, 64)), dim3(64), 0, s, la + 1, nvec,
                       d_part.ptr<double>(), se_dev);
    MBL_CHECK_LAUNCH();
}

void ObsWork::vector_sums(const uint32_t *basis, const double *psi, int64_t ld, int nvec,
                          double *out_dev, hipStream_t s) {
    // pass 0: norms; pass 1: everything else with the normalised weights
    double *nrm = d_out.ptr<double>() + NQ * nvmax;
    hipLaunchKernelGGL(k_vec_sums, dim3(OBS_PARTS, nvec), dim3(SEB), 0, s, L, dim, nvec, basis, psi,
                       ld, nrm, 0, d_part.ptr<double>());
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vec_final, dim3(cdiv(nvec, 64)), dim3(64), 0, s, nvec, OBS_PARTS,
                       d_part.ptr<double>(), out_dev, 0);
    MBL_CHECK_LAUNCH();
    // gather the norms (column 0 of out) into nrm
    hipLaunchKernelGGL(k_stride_copy, dim3(cdiv(nvec, 64)), dim3(64), 0, s, nvec, out_dev, NQ, nrm);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vec_sums, dim3(OBS_PARTS, nvec), dim3(SEB), 0, s, L, dim, nvec, basis, psi,
                       ld, nrm, 1, d_part.ptr<double>());
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vec_final, dim3(cdiv(nvec, 64)), dim3(64), 0, s, nvec, OBS_PARTS,
                       d_part.ptr<double>(), out_dev, 1);
    MBL_CHECK_LAUNCH();
}

void ObsWork::gap_ratios(int nev, const double *E_dev, double *r_dev, hipStream_t s) {
    if (nev < 3) return;
    hipLaunchKernelGGL(k_gap_ratio, dim3(cdiv(nev, 64)), dim3(64), 0, s, nev, E_dev, r_dev);
    MBL_CHECK_LAUNCH();
}

}  // namespace mbl
