// k_basis.hip -- S^z = 0 sector basis, ranking and Hamiltonian assembly on gfx950.
//
// Sector (section "Numerical method", S^z = 0 of even L): the L-bit words with
// K = L/2 bits set, in ascending order.  Ascending integer order of words with
// a fixed popcount is colexicographic order of their set-bit positions
// c_1 < ... < c_K, whose index is the combinatorial number system value
//     rank(s) = sum_{j=1..K} C(c_j, j)
// (Knuth, TAOCP 7.2.1.3).  So each lane unranks its own index independently
// and ranks a neighbour word with K table lookups; no search.
//
// Hamiltonian, Eq. (1): H = J sum_i S_i.S_{i+1} + sum_i h_i S^z_i on the ring.
// Diagonal: J/4 sum_i s_i s_{i+1} + 1/2 sum_i h_i s_i (s = +-1).  Off-diagonal:
// J/2 between s and s with an antiparallel bond (i, i+1 mod L) exchanged; at
// L = 2 both bonds are the same pair and the entry is J.
#include "common.hpp"
#include "kernels.hpp"

namespace mbl {
namespace {

// C(n, k) for 0 <= n <= 32, 0 <= k <= 16
__constant__ uint32_t c_binom[33][17];
bool g_binom_ready = false;

void ensure_binom() {
    if (g_binom_ready) return;
    uint32_t t[33][17] = {};
    for (int n = 0; n <= 32; n++)
        for (int k = 0; k <= 16; k++) t[n][k] = (uint32_t)binom(n, k);
    MBL_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), t, sizeof(t)));
    g_binom_ready = true;
}

__device__ __forceinline__ int64_t rank_word(uint32_t s, int K) {
    if (__popc(s) != K) return -1;
    int64_t r = 0;
    int j = 1;
    while (s) {
        int c = __ffs(s) - 1;
        r += c_binom[c][j];
        j++;
        s &= s - 1;
    }
    return r;
}

__device__ __forceinline__ uint32_t rotl1(uint32_t s, int L) {
    uint32_t m = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
    return ((s << 1) | (s >> (L - 1))) & m;
}

__global__ void k_fields(int L, double h, uint64_t seed, double *out) {
    int i = threadIdx.x;
    if (i >= L) return;
    // SplitMix64 is counter based: the state before draw i is seed + (i+1) gamma
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    out[i] = h * (2.0 * u - 1.0);
}

__global__ void k_basis(int L, int K, int64_t dim, uint32_t *basis) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= dim) return;
    uint32_t r = (uint32_t)k, s = 0;
    int c = L - 1;
    for (int j = K; j >= 1; j--) {
        while (c_binom[c][j] > r) c--;   // largest c with C(c, j) <= r
        s |= 1u << c;
        r -= c_binom[c][j];
        c--;
    }
    basis[k] = s;
}

__global__ void k_rank(int L, int K, const uint32_t *words, int64_t count, int64_t *ranks) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint32_t s = words[i];
    uint32_t m = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
    ranks[i] = (s & ~m) ? -1 : rank_word(s, K);
}

// nonzeros per row: diagonal + one per antiparallel bond (the doubled bond of
// L = 2 is a single entry)
__global__ void k_row_count(int L, int64_t dim, const uint32_t *basis, int32_t *cnt) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= dim) return;
    uint32_t s = basis[k];
    int n = (L == 2) ? 1 : __popc(s ^ rotl1(s, L));
    cnt[k] = 1 + n;
}

// ---- exclusive scan over int32 (three passes, fixed order) ------------------
constexpr int SCAN_BLOCK = 1024;

__device__ int32_t block_excl_scan(int32_t v, int32_t *sh, int32_t *total) {
    // Hillis-Steele over a 1024-wide block in LDS
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int32_t a = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    int32_t incl = sh[t];
    *total = sh[SCAN_BLOCK - 1];
    return incl - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_partial(const int32_t *in, int64_t n,
                                                             int32_t *block_sums) {
    __shared__ int32_t sh[SCAN_BLOCK];
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    int32_t v = (i < n) ? in[i] : 0;
    int32_t tot;
    block_excl_scan(v, sh, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(int32_t *block_sums, int nb) {
    __shared__ int32_t sh[SCAN_BLOCK];
    int32_t carry = 0;
    for (int base = 0; base < nb; base += SCAN_BLOCK) {
        int i = base + threadIdx.x;
        int32_t v = (i < nb) ? block_sums[i] : 0;
        int32_t tot;
        int32_t ex = block_excl_scan(v, sh, &tot);
        __syncthreads();
        if (i < nb) block_sums[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[nb] = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_final(const int32_t *in, int64_t n,
                                                           const int32_t *block_offs,
                                                           int32_t *out) {
    __shared__ int32_t sh[SCAN_BLOCK];
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    int32_t v = (i < n) ? in[i] : 0;
    int32_t tot;
    int32_t ex = block_excl_scan(v, sh, &tot);
    if (i < n) out[i] = ex + block_offs[blockIdx.x];
    if (i == n - 1) out[n] = ex + v + block_offs[blockIdx.x];
}

// columns of row k, ascending: the diagonal and the ranks of the exchanged
// words (rank is monotone in the word value, so sorting words sorts ranks)
__global__ void k_fill_csr(int L, int K, int64_t dim, const uint32_t *basis,
                           const int32_t *rowptr, int32_t *col) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= dim) return;
    uint32_t s = basis[k];
    uint32_t w[33];
    int n = 0;
    w[n++] = s;
    if (L == 2) {
        w[n++] = s ^ 3u;
    } else {
        for (int i = 0; i < L; i++) {
            int j = (i + 1 == L) ? 0 : i + 1;
            if (((s >> i) ^ (s >> j)) & 1u) w[n++] = s ^ ((1u << i) | (1u << j));
        }
    }
    for (int a = 1; a < n; a++) {           // insertion sort, n <= L + 1
        uint32_t v = w[a];
        int b = a - 1;
        while (b >= 0 && w[b] > v) { w[b + 1] = w[b]; b--; }
        w[b + 1] = v;
    }
    int32_t base = rowptr[k];
    for (int a = 0; a < n; a++) col[base + a] = (int32_t)rank_word(w[a], K);
}

__global__ void k_diag(int L, double J, const double *fields, int64_t dim,
                       const uint32_t *basis, double *diag) {
    __shared__ double f[32];
    if (threadIdx.x < L) f[threadIdx.x] = fields[threadIdx.x];
    __syncthreads();
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= dim) return;
    uint32_t s = basis[k];
    double d = 0.0;
    for (int i = 0; i < L; i++) {
        int j = (i + 1 == L) ? 0 : i + 1;
        int si = ((s >> i) & 1u) ? 1 : -1, sj = ((s >> j) & 1u) ? 1 : -1;
        d += 0.25 * J * (double)(si * sj);
    }
    for (int i = 0; i < L; i++) {
        int si = ((s >> i) & 1u) ? 1 : -1;
        d += 0.5 * f[i] * (double)si;
    }
    diag[k] = d;
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_fields(int L, double h, uint64_t seed, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_fields, dim3(1), dim3(64), 0, s, L, h, seed, out);
    MBL_CHECK_LAUNCH();
}

void launch_basis(int L, int64_t dim, uint32_t *basis, hipStream_t s) {
    ensure_binom();
    if (dim == 0) return;
    hipLaunchKernelGGL(k_basis, dim3(grid_for(dim, 256)), dim3(256), 0, s, L, sector_nup(L), dim, basis);
    MBL_CHECK_LAUNCH();
}

void launch_rank(int L, const uint32_t *words, int64_t count, int64_t *ranks, hipStream_t s) {
    ensure_binom();
    if (count == 0) return;
    hipLaunchKernelGGL(k_rank, dim3(grid_for(count, 256)), dim3(256), 0, s, L, sector_nup(L), words,
                       count, ranks);
    MBL_CHECK_LAUNCH();
}

size_t scan_scratch_bytes(int64_t n) {
    int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    return sizeof(int32_t) * (size_t)(n + nb + 2);
}

void launch_row_ptr(int L, int64_t dim, const uint32_t *basis, int32_t *rowptr, void *scratch,
                    hipStream_t s) {
    int32_t *cnt = static_cast<int32_t *>(scratch);
    int64_t nb = (dim + SCAN_BLOCK - 1) / SCAN_BLOCK;
    int32_t *bsum = cnt + dim;
    hipLaunchKernelGGL(k_row_count, dim3(grid_for(dim, 256)), dim3(256), 0, s, L, dim, basis, cnt);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, cnt, dim, bsum);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, s, bsum, (int)nb);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, cnt, dim, bsum,
                       rowptr);
    MBL_CHECK_LAUNCH();
}

void launch_fill_csr(int L, int64_t dim, const uint32_t *basis, const int32_t *rowptr,
                     int32_t *col, hipStream_t s) {
    ensure_binom();
    hipLaunchKernelGGL(k_fill_csr, dim3(grid_for(dim, 256)), dim3(256), 0, s, L, sector_nup(L), dim,
                       basis, rowptr, col);
    MBL_CHECK_LAUNCH();
}

void launch_diag(int L, double J, const double *fields, int64_t dim, const uint32_t *basis,
                 double *diag, hipStream_t s) {
    hipLaunchKernelGGL(k_diag, dim3(grid_for(dim, 256)), dim3(256), 0, s, L, J, fields, dim,
                       basis, diag);
    MBL_CHECK_LAUNCH();
}

}  // namespace mbl
