// k_blas.hip -- FP64 sparse matrix-vector products with H and the tall-skinny
// dense kernels of the Krylov method (projections, block updates) on gfx950.
//
// H is stored as its CSR pattern (diagonal included, int32 columns) plus a
// per-realization FP64 diagonal; every off-diagonal entry of Eq. (1) has the
// same value (J/2, or J for the doubled bond of L = 2), so it is passed as a
// scalar instead of streaming a value array.
//
// All reductions use a fixed grid and a fixed combination order so results are
// bitwise reproducible run to run and independent of what else is in flight.
#include "common.hpp"
#include "kernels.hpp"

namespace mbl {
namespace {

constexpr int BS = 256;

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__global__ __launch_bounds__(BS) void k_spmv(int64_t n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ col,
                                             const double *__restrict__ diag, double offv,
                                             double shift, int nvec, const double *__restrict__ x,
                                             double *__restrict__ y) {
    int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    int32_t a = rowptr[k], e = rowptr[k + 1];
    double dk = diag[k] - shift;
    for (int v = 0; v < nvec; v++) {
        const double *xv = x + (int64_t)v * n;
        double acc = 0.0;
        for (int32_t p = a; p < e; p++) {
            int32_t c = col[p];
            if (c != k) acc += xv[c];
        }
        y[(int64_t)v * n + k] = dk * xv[k] + offv * acc;
    }
}

// r = b - (H - shift) x; per-block partial sums of r^2, x^2, b^2 per vector.
// Segment blockIdx.y is rows [seg n, (seg + 1) n) of a block-diagonal H (the
// CSR columns are global), vectors packed with ld = nseg n; its partials
// follow those of the segments before it.
__global__ __launch_bounds__(BS) void k_residual(int64_t n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ diag, double offv,
                                                 double shift, int nvec,
                                                 const double *__restrict__ b,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ r,
                                                 double *__restrict__ partials, int64_t ld) {
    __shared__ double red[3][BS];
    const int64_t g0 = (int64_t)blockIdx.y * n;
    partials += (int64_t)blockIdx.y * gridDim.x * nvec * 3;
    for (int v = 0; v < nvec; v++) {
        const double *xv = x + (int64_t)v * ld;
        const double *bv = b + (int64_t)v * ld;
        double sr = 0.0, sx = 0.0, sb = 0.0;
        for (int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x; k < n;
             k += (int64_t)gridDim.x * BS) {
            const int64_t gk = g0 + k;
            int32_t a = rowptr[gk], e = rowptr[gk + 1];
            double acc = 0.0;
            for (int32_t p = a; p < e; p++) {
                int32_t c = col[p];
                if (c != gk) acc += xv[c];
            }
            double xk = xv[gk], bk = bv[gk];
            double rk = bk - ((diag[gk] - shift) * xk + offv * acc);
            r[(int64_t)v * ld + gk] = rk;
            sr += rk * rk; sx += xk * xk; sb += bk * bk;
        }
        red[0][threadIdx.x] = sr; red[1][threadIdx.x] = sx; red[2][threadIdx.x] = sb;
        __syncthreads();
        for (int off = BS / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off)
                for (int q = 0; q < 3; q++) red[q][threadIdx.x] += red[q][threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x < 3)
            partials[((int64_t)blockIdx.x * nvec + v) * 3 + threadIdx.x] = red[threadIdx.x][0];
        __syncthreads();
    }
}

// C = A^T B (A n x k, B n x b, column major).  The rows are cut into nparts
// fixed contiguous ranges and the columns of A into chunks of TN_KC; block
// (range, chunk) walks its range in LDS tiles of TN_ROWS rows.  A thread owns
// one column of A and all b columns of B over one row group of the tile; the
// row groups are combined in a fixed order at the end, so the partials (and
// the fixed-order sum over ranges) are reproducible.
constexpr int TN_ROWS = 32;
constexpr int TN_KC = 128;

template <int NB>
__global__ __launch_bounds__(BS) void k_gemm_tn_part(int64_t n, int k, int b,
                                                     const double *__restrict__ A, int64_t lda,
                                                     const double *__restrict__ B, int64_t ldb,
                                                     double *__restrict__ partials,
                                                     int64_t rows_per_part, int64_t segA,
                                                     int64_t segB) {
    extern __shared__ double sm[];
    // segment blockIdx.z: its own rows of A and B, its own partials
    A += (int64_t)blockIdx.z * segA;
    B += (int64_t)blockIdx.z * segB;
    partials += (int64_t)blockIdx.z * gridDim.x * (int64_t)k * b;
    const int c0 = blockIdx.y * TN_KC;
    const int kc = min(TN_KC, k - c0);
    const int lda_s = kc + 1;                 // odd stride: rows of a tile fall in different banks
    double *sA = sm;                          // [TN_ROWS][kc + 1]
    double *sB = sm + TN_ROWS * lda_s;        // [TN_ROWS][NB]
    const int G = min(TN_ROWS, BS / kc);      // row groups
    const int i = threadIdx.x % kc, g = threadIdx.x / kc;
    const bool active = g < G;
    int64_t r0 = (int64_t)blockIdx.x * rows_per_part;
    int64_t r1 = min(r0 + rows_per_part, n);
    double acc[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) acc[j] = 0.0;
    for (int64_t r = r0; r < r1; r += TN_ROWS) {
        int nr = (int)min((int64_t)TN_ROWS, r1 - r);
        for (int t = threadIdx.x; t < TN_ROWS * kc; t += BS) {
            int rr = t % TN_ROWS, c = t / TN_ROWS;
            sA[rr * lda_s + c] = rr < nr ? A[r + rr + (int64_t)(c0 + c) * lda] : 0.0;
        }
        for (int t = threadIdx.x; t < TN_ROWS * NB; t += BS) {
            int rr = t % TN_ROWS, j = t / TN_ROWS;
            sB[rr * NB + j] = (rr < nr && j < b) ? B[r + rr + (int64_t)j * ldb] : 0.0;
        }
        __syncthreads();
        if (active)
            for (int rr = g; rr < nr; rr += G) {
                double x = sA[rr * lda_s + i];
#pragma unroll
                for (int j = 0; j < NB; j++) acc[j] += x * sB[rr * NB + j];
            }
        __syncthreads();
    }
    // combine the row groups: red[g][j][i]
    double *red = sm;
    if (active)
#pragma unroll
        for (int j = 0; j < NB; j++) red[((int64_t)g * NB + j) * kc + i] = acc[j];
    __syncthreads();
    int kb = k * b;
    for (int o = threadIdx.x; o < kc * b; o += BS) {
        int ii = o % kc, j = o / kc;
        double sum = 0.0;
        for (int q = 0; q < G; q++) sum += red[((int64_t)q * NB + j) * kc + ii];
        partials[(int64_t)blockIdx.x * kb + c0 + ii + (int64_t)j * k] = sum;
    }
}

// C[o] = sum over the ranges in order: SP_G groups of consecutive ranges per
// output, combined in a fixed order
constexpr int SP_G = 8;

__global__ __launch_bounds__(64 * SP_G) void k_sum_parts(int kb, int nparts,
                                                        const double *__restrict__ partials,
                                                        double *__restrict__ C, int64_t segC) {
    __shared__ double red[SP_G][64];
    partials += (int64_t)blockIdx.y * nparts * (int64_t)kb;   // segment blockIdx.y
    C += (int64_t)blockIdx.y * segC;
    int l = threadIdx.x % 64, g = threadIdx.x / 64;
    int o = blockIdx.x * 64 + l;
    int p0 = (int)((int64_t)nparts * g / SP_G), p1 = (int)((int64_t)nparts * (g + 1) / SP_G);
    double s = 0.0;
    if (o < kb) {
        const double *q = partials + o;
#pragma unroll 8
        for (int p = p0; p < p1; p++) s += q[(int64_t)p * kb];
    }
    red[g][l] = s;
    __syncthreads();
    if (g == 0 && o < kb) {
        double t = red[0][l];
#pragma unroll
        for (int q = 1; q < SP_G; q++) t += red[q][l];
        C[o] = t;
    }
}

// C = beta C + alpha A Y for up to 16 output columns per launch: 64 rows per
// block, the k columns of A split over four waves and combined in order
constexpr int NN_MAXB = 16;
constexpr int NN_ROWS = 64;
constexpr int NN_KG = BS / NN_ROWS;

template <int NB>
__global__ __launch_bounds__(BS) void k_gemm_nn(int64_t n, int k, int b, double alpha,
                                                const double *__restrict__ A, int64_t lda,
                                                const double *__restrict__ Y, int ldy, double beta,
                                                double *__restrict__ C, int64_t ldc, int64_t segA,
                                                int64_t segY, int64_t segC) {
    extern __shared__ double sm[];
    A += (int64_t)blockIdx.y * segA;                 // segment blockIdx.y
    Y += (int64_t)blockIdx.y * segY;
    C += (int64_t)blockIdx.y * segC;
    double *sY = sm;                                  // [k][NB]
    double *red = sm + (int64_t)k * NB;               // [NN_KG][NN_ROWS][NB]
    for (int t = threadIdx.x; t < k * NB; t += BS) {
        int i = t / NB, j = t % NB;
        sY[t] = j < b ? Y[i + (int64_t)j * ldy] : 0.0;
    }
    __syncthreads();
    int lane = threadIdx.x % NN_ROWS, g = threadIdx.x / NN_ROWS;
    int64_t row = (int64_t)blockIdx.x * NN_ROWS + lane;
    int i0 = k * g / NN_KG, i1 = k * (g + 1) / NN_KG;
    double acc[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) acc[j] = 0.0;
    if (row < n) {
        const double *a = A + row;
#pragma unroll 4
        for (int i = i0; i < i1; i++) {
            double x = a[(int64_t)i * lda];
#pragma unroll
            for (int j = 0; j < NB; j++) acc[j] += x * sY[i * NB + j];
        }
    }
#pragma unroll
    for (int j = 0; j < NB; j++) red[(g * NN_ROWS + lane) * NB + j] = acc[j];
    __syncthreads();
    for (int t = threadIdx.x; t < NN_ROWS * b; t += BS) {
        int l = t % NN_ROWS, j = t / NN_ROWS;
        int64_t r = (int64_t)blockIdx.x * NN_ROWS + l;
        if (r >= n) continue;
        double sum = 0.0;
        for (int q = 0; q < NN_KG; q++) sum += red[(q * NN_ROWS + l) * NB + j];
        double *c = C + r + (int64_t)j * ldc;
        *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * sum;
    }
}

__global__ void k_gather(int64_t n, int nvec, const int32_t *__restrict__ idx,
                         const double *__restrict__ x, double *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t s = idx[i];
    for (int v = 0; v < nvec; v++) y[(int64_t)v * n + i] = x[(int64_t)v * n + s];
}

// start block: components u - 1/2 with u from SplitMix64 (counter based);
// segment blockIdx.y draws from its own seed, element (i, j) with counter
// i + j n, stored at v[i + segment n + j ld]
__global__ void k_fill_start(int64_t n, int nvec, SegSeeds seeds, double *v, int64_t ld) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nvec) return;
    const int sg = blockIdx.y;
    uint64_t z = seeds.seed[sg] + (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    const int64_t i = e % n, j = e / n;
    v[i + sg * n + j * ld] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

__global__ void k_copy(int64_t count, const double *__restrict__ x, double *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) y[i] = x[i];
}

__global__ void k_axpy(int64_t count, double a, const double *__restrict__ x,
                       double *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) y[i] += a * x[i];
}

__global__ void k_shift_seg(int64_t n, const double *__restrict__ x, SegVals shift,
                            double *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sg = blockIdx.y;
    if (i < n) y[i + sg * n] = x[i + sg * n] - shift.v[sg];
}

// y += x on the segments whose flag is set (packed vectors: nseg segments of n
// rows per column, nvec columns of ld = nseg n)
__global__ void k_axpy_masked(int64_t n, int nseg, int nvec, const int *__restrict__ on,
                              const double *__restrict__ x, double *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sg = blockIdx.y;
    if (i >= n * nvec || !on[sg]) return;
    const int64_t r = i % n, j = i / n, o = r + sg * n + j * n * nseg;
    y[o] += x[o];
}

// out[j] = sum_i A[i, j] B[i, j] for j < ncol (partials per block, fixed order)
__global__ __launch_bounds__(BS) void k_coldot_part(int64_t n, int ncol, const double *__restrict__ A,
                                                    int64_t lda, const double *__restrict__ B,
                                                    int64_t ldb, double *__restrict__ part,
                                                    int64_t seg) {
    __shared__ double red[BS];
    int j = blockIdx.y;
    A += (int64_t)blockIdx.z * seg;                  // segment blockIdx.z: rows, partials
    B += (int64_t)blockIdx.z * seg;
    part += (int64_t)blockIdx.z * ncol * gridDim.x;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        s += A[i + (int64_t)j * lda] * B[i + (int64_t)j * ldb];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_coldot_sum(int ncol, int nparts, const double *__restrict__ part,
                             double *__restrict__ out) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    part += (int64_t)blockIdx.y * ncol * nparts;     // segment blockIdx.y
    out += (int64_t)blockIdx.y * ncol;
    if (j >= ncol) return;
    double s = 0.0;
    for (int p = 0; p < nparts; p++) s += part[(int64_t)j * nparts + p];
    out[j] = s;
}

// Y[:, j] -= e[j] X[:, j]
__global__ void k_sub_scaled_cols(int64_t n, int ncol, const double *__restrict__ e,
                                  const double *__restrict__ X, int64_t ldx, double *__restrict__ Y,
                                  int64_t ldy) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    e += (int64_t)blockIdx.z * ncol;                 // segment blockIdx.z
    X += (int64_t)blockIdx.z * n;
    Y += (int64_t)blockIdx.z * n;
    if (i < n) Y[i + (int64_t)j * ldy] -= e[j] * X[i + (int64_t)j * ldx];
}

// Per-column dots against a stack of nb blocks (block i at V + i * bs, each
// n x nrhs with ld n): part[(blk * nrhs + j) * nb + i] = sum over the block's
// rows of V_i[r, j] W[r, j].  Wave shuffles then a fixed-order sum over the
// four waves, so the partials are reproducible.
constexpr int BD_MAX = 32;

__global__ __launch_bounds__(BS) void k_bdot_part(int64_t n, int nb, int nrhs,
                                                  const double *__restrict__ V, int64_t bs,
                                                  const double *__restrict__ W,
                                                  double *__restrict__ part) {
    __shared__ double red[BS / 64][BD_MAX];
    const int j = blockIdx.y;
    double acc[BD_MAX];
#pragma unroll
    for (int i = 0; i < BD_MAX; i++) acc[i] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n; r += (int64_t)gridDim.x * BS) {
        const double w = W[r + (int64_t)j * n];
        const double *v = V + r + (int64_t)j * n;
#pragma unroll
        for (int i = 0; i < BD_MAX; i++)
            if (i < nb) acc[i] += v[(int64_t)i * bs] * w;
    }
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int i = 0; i < BD_MAX; i++) {
        if (i >= nb) break;
        double v = acc[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wv][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < nb) {
        double t = red[0][threadIdx.x];
        for (int q = 1; q < BS / 64; q++) t += red[q][threadIdx.x];
        part[((int64_t)blockIdx.x * nrhs + j) * nb + threadIdx.x] = t;
    }
}

// out[:, j] = beta out[:, j] + alpha sum_i coef[i + j nb] V_i[:, j]
__global__ __launch_bounds__(BS) void k_bcomb(int64_t n, int nb, int nrhs,
                                              const double *__restrict__ V, int64_t bs,
                                              const double *__restrict__ coef, double alpha,
                                              double beta, double *__restrict__ out) {
    const int j = blockIdx.y;
    const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (r >= n) return;
    const double *v = V + r + (int64_t)j * n;
    double s = 0.0;
    for (int i = 0; i < nb; i++) s += coef[i + (int64_t)j * nb] * v[(int64_t)i * bs];
    double *o = out + r + (int64_t)j * n;
    *o = (beta == 0.0 ? 0.0 : beta * *o) + alpha * s;
}

// Cholesky G = R^T R of a small b x b Gram matrix (b <= 16) and R^-1, by one
// lane (a few hundred flops, kept on the device so the Krylov expansion needs
// no host round trip): R (upper, column-major, zeros below) to Rout, R^-1 to
// Rinv; *flag = 1 if a pivot fell below rel_tiny * max diag (it is then
// floored there, so the factor stays finite).
__global__ void k_small_chol(int b, const double *__restrict__ G, double *__restrict__ Rout,
                             double *__restrict__ Rinv, int *__restrict__ flag, double rel_tiny,
                             int64_t segG, int64_t segR, int64_t segRi, int64_t segF) {
    __shared__ double R[16 * 16], Ri[16 * 16];
    if (threadIdx.x != 0) return;
    G += blockIdx.x * segG;                          // matrix blockIdx.x
    Rout += blockIdx.x * segR;
    Rinv += blockIdx.x * segRi;
    flag += blockIdx.x * segF;
    double dmax = 0.0;
    for (int i = 0; i < b; i++) dmax = fmax(dmax, G[i * b + i]);
    int fl = 0;
    for (int q = 0; q < b * b; q++) { R[q] = 0.0; Ri[q] = 0.0; }
    for (int j = 0; j < b; j++)
        for (int i = 0; i <= j; i++) {
            double sum = G[j * b + i];
            for (int k = 0; k < i; k++) sum -= R[i * b + k] * R[j * b + k];
            if (i == j) {
                if (sum <= rel_tiny * dmax) { fl = 1; sum = fmax(sum, rel_tiny * dmax + 1e-300); }
                R[j * b + j] = sqrt(sum);
            } else {
                R[j * b + i] = sum / R[i * b + i];
            }
        }
    for (int j = 0; j < b; j++) {
        Ri[j * b + j] = 1.0 / R[j * b + j];
        for (int i = j - 1; i >= 0; i--) {
            double sum = 0.0;
            for (int k = i + 1; k <= j; k++) sum += R[k * b + i] * Ri[j * b + k];
            Ri[j * b + i] = -sum / R[i * b + i];
        }
    }
    for (int q = 0; q < b * b; q++) { Rout[q] = R[q]; Rinv[q] = Ri[q]; }
    *flag = fl;
}

}  // namespace

void launch_coldot_seg(int nseg, int64_t n, int ncol, const double *A, int64_t lda,
                       const double *B, int64_t ldb, int64_t seg, double *out, double *partials,
                       int nparts, hipStream_t s) {
    if (ncol == 0 || nseg == 0) return;
    hipLaunchKernelGGL(k_coldot_part, dim3(nparts, ncol, nseg), dim3(BS), 0, s, n, ncol, A, lda, B,
                       ldb, partials, seg);
    MBL_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_coldot_sum, dim3(grid_for(ncol, 64), nseg), dim3(64), 0, s, ncol, nparts,
                       partials, out);
    MBL_CHECK_LAUNCH();
}

void launch_coldot(int64_t n, int ncol, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *out, double *partials, int nparts, hipStream_t s) {
    launch_coldot_seg(1, n, ncol, A, lda, B, ldb, 0, out, partials, nparts, s);
}

void launch_sub_scaled_cols_seg(int nseg, int64_t n, int ncol, const double *e, const double *X,
                                int64_t ldx, double *Y, int64_t ldy, hipStream_t s) {
    if (ncol == 0 || n == 0 || nseg == 0) return;
    hipLaunchKernelGGL(k_sub_scaled_cols, dim3(grid_for(n, 256), ncol, nseg), dim3(256), 0, s, n,
                       ncol, e, X, ldx, Y, ldy);
    MBL_CHECK_LAUNCH();
}

void launch_sub_scaled_cols(int64_t n, int ncol, const double *e, const double *X, int64_t ldx,
                            double *Y, int64_t ldy, hipStream_t s) {
    launch_sub_scaled_cols_seg(1, n, ncol, e, X, ldx, Y, ldy, s);
}

void launch_small_chol_batch(int count, int b, const double *G, int64_t segG, double *R,
                             int64_t segR, double *Rinv, int64_t segRi, int *flag, int64_t segF,
                             double rel_tiny, hipStream_t s) {
    MBL_REQUIRE(b >= 1 && b <= 16, MBL_EINVAL, "small_chol: b must be 1..16");
    if (count == 0) return;
    k_small_chol<<<dim3(count), dim3(64), 0, s>>>(b, G, R, Rinv, flag, rel_tiny, segG, segR, segRi,
                                                  segF);
    MBL_CHECK_LAUNCH();
}

void launch_small_chol(int b, const double *G, double *R, double *Rinv, int *flag,
                       double rel_tiny, hipStream_t s) {
    launch_small_chol_batch(1, b, G, 0, R, 0, Rinv, 0, flag, 0, rel_tiny, s);
}

void launch_bdot(int64_t n, int nb, int nrhs, const double *V, int64_t bs, const double *W,
                 double *out, double *partials, int nparts, hipStream_t s) {
    MBL_REQUIRE(nb >= 0 && nb <= BD_MAX, MBL_EINVAL, "bdot: too many blocks");
    if (nb == 0 || nrhs == 0) return;
    k_bdot_part<<<dim3((unsigned)nparts, (unsigned)nrhs), dim3(BS), 0, s>>>(n, nb, nrhs, V, bs, W,
                                                                            partials);
    MBL_CHECK_LAUNCH();
    int kb = nb * nrhs;
    k_sum_parts<<<dim3(grid_for(kb, 64)), dim3(64 * SP_G), 0, s>>>(kb, nparts, partials, out, 0);
    MBL_CHECK_LAUNCH();
}

void launch_bcomb(int64_t n, int nb, int nrhs, const double *V, int64_t bs, const double *coef,
                  double alpha, double beta, double *out, hipStream_t s) {
    if (n == 0 || nrhs == 0) return;
    k_bcomb<<<dim3(grid_for(n, BS), (unsigned)nrhs), dim3(BS), 0, s>>>(n, nb, nrhs, V, bs, coef,
                                                                      alpha, beta, out);
    MBL_CHECK_LAUNCH();
}

void launch_spmv(int64_t n, const int32_t *rowptr, const int32_t *col, const double *diag,
                 double offv, double shift, int nvec, const double *x, double *y, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_spmv, dim3(grid_for(n, BS)), dim3(BS), 0, s, n, rowptr, col, diag, offv,
                       shift, nvec, x, y);
    MBL_CHECK_LAUNCH();
}

void launch_residual_seg(int nseg, int64_t n, const int32_t *rowptr, const int32_t *col,
                         const double *diag, double offv, double shift, int nvec, const double *b,
                         const double *x, double *r, double *partials, int nparts, hipStream_t s) {
    if (nseg == 0) return;
    hipLaunchKernelGGL(k_residual, dim3(nparts, nseg), dim3(BS), 0, s, n, rowptr, col, diag, offv,
                       shift, nvec, b, x, r, partials, n * nseg);
    MBL_CHECK_LAUNCH();
}

void launch_residual(int64_t n, const int32_t *rowptr, const int32_t *col, const double *diag,
                     double offv, double shift, int nvec, const double *b, const double *x,
                     double *r, double *partials, int nparts, hipStream_t s) {
    launch_residual_seg(1, n, rowptr, col, diag, offv, shift, nvec, b, x, r, partials, nparts, s);
}

int gemm_tn_parts(int64_t n) {
    // ranges of at least 64 rows, at most 512 of them
    int64_t p = (n + 63) / 64;
    if (p < 1) p = 1;
    if (p > 512) p = 512;
    return (int)p;
}

void launch_gemm_tn(int64_t n, int k, int b, const double *A, int64_t lda, const double *B,
                    int64_t ldb, double *C, double *partials, int nparts, hipStream_t s) {
    launch_gemm_tn_seg(1, n, k, b, A, lda, 0, B, ldb, 0, C, 0, partials, nparts, s);
}

void launch_gemm_tn_seg(int nseg, int64_t n, int k, int b, const double *A, int64_t lda,
                        int64_t segA, const double *B, int64_t ldb, int64_t segB, double *C,
                        int64_t segC, double *partials, int nparts, hipStream_t s) {
    MBL_REQUIRE(b >= 0 && b <= NN_MAXB && k >= 0, MBL_EINVAL, "gemm_tn: b must be at most 16");
    if (k == 0 || b == 0 || nseg == 0) return;
    int64_t rpp = (n + nparts - 1) / nparts;
    rpp = (rpp + TN_ROWS - 1) / TN_ROWS * TN_ROWS;
    int kc = std::min(k, TN_KC);
    auto go = [&](auto nbc) {
        constexpr int NB = decltype(nbc)::value;
        int G = std::min(TN_ROWS, BS / kc);
        size_t tile = sizeof(double) * TN_ROWS * ((size_t)kc + 1 + NB);
        size_t red = sizeof(double) * (size_t)G * NB * kc;
        size_t sh = std::max(tile, red);
        k_gemm_tn_part<NB><<<dim3((unsigned)nparts, (unsigned)((k + TN_KC - 1) / TN_KC),
                                  (unsigned)nseg), dim3(BS), sh, s>>>(n, k, b, A, lda, B, ldb,
                                                                      partials, rpp, segA, segB);
    };
    if (b <= 4) go(std::integral_constant<int, 4>{});
    else if (b <= 8) go(std::integral_constant<int, 8>{});
    else go(std::integral_constant<int, 16>{});
    MBL_CHECK_LAUNCH();
    int kb = k * b;
    k_sum_parts<<<dim3(grid_for(kb, 64), (unsigned)nseg), dim3(64 * SP_G), 0, s>>>(kb, nparts,
                                                                                 partials, C, segC);
    MBL_CHECK_LAUNCH();
}

void launch_gemm_nn(int64_t n, int k, int b, double alpha, const double *A, int64_t lda,
                    const double *Y, int ldy, double beta, double *C, int64_t ldc, hipStream_t s) {
    launch_gemm_nn_seg(1, n, k, b, alpha, A, lda, 0, Y, ldy, 0, beta, C, ldc, 0, s);
}

void launch_gemm_nn_seg(int nseg, int64_t n, int k, int b, double alpha, const double *A,
                        int64_t lda, int64_t segA, const double *Y, int ldy, int64_t segY,
                        double beta, double *C, int64_t ldc, int64_t segC, hipStream_t s) {
    if (n == 0 || b == 0 || nseg == 0) return;
    constexpr int KN = 256;    // columns of A per launch (LDS for Y stays under 64 KB)
    for (int j0 = 0; j0 < b; j0 += NN_MAXB) {
        int bb = (b - j0) < NN_MAXB ? (b - j0) : NN_MAXB;
        auto go = [&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            for (int k0 = 0; k0 < std::max(k, 1); k0 += KN) {
                int kk = std::min(KN, k - k0);
                size_t sh = sizeof(double) * ((size_t)kk * NB + (size_t)NN_KG * NN_ROWS * NB);
                k_gemm_nn<NB><<<dim3(grid_for(n, NN_ROWS), (unsigned)nseg), dim3(BS), sh, s>>>(
                    n, kk, bb, alpha, A + (int64_t)k0 * lda, lda, Y + k0 + (int64_t)j0 * ldy, ldy,
                    k0 == 0 ? beta : 1.0, C + (int64_t)j0 * ldc, ldc, segA, segY, segC);
            }
        };
        if (bb <= 4) go(std::integral_constant<int, 4>{});
        else if (bb <= 8) go(std::integral_constant<int, 8>{});
        else go(std::integral_constant<int, 16>{});
        MBL_CHECK_LAUNCH();
    }
}

void launch_gather(int64_t n, int nvec, const int32_t *idx, const double *x, double *y,
                   hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, s, n, nvec, idx, x, y);
    MBL_CHECK_LAUNCH();
}

void launch_fill_start_seg(int nseg, int64_t n, int nvec, const uint64_t *seeds, double *v,
                           int64_t ld, hipStream_t s) {
    MBL_REQUIRE(nseg >= 0 && nseg <= MBL_SEG_MAX, MBL_EINVAL, "fill_start: too many segments");
    if (n * nvec == 0 || nseg == 0) return;
    SegSeeds sd;
    for (int q = 0; q < nseg; q++) sd.seed[q] = seeds[q];
    hipLaunchKernelGGL(k_fill_start, dim3(grid_for(n * nvec, 256), nseg), dim3(256), 0, s, n, nvec,
                       sd, v, ld);
    MBL_CHECK_LAUNCH();
}

void launch_fill_start(int64_t n, int nvec, uint64_t seed, double *v, hipStream_t s) {
    launch_fill_start_seg(1, n, nvec, &seed, v, n, s);
}

void launch_axpy_masked(int64_t n, int nseg, int nvec, const int *on, const double *x, double *y,
                        hipStream_t s) {
    if (n * nvec == 0 || nseg == 0) return;
    hipLaunchKernelGGL(k_axpy_masked, dim3(grid_for(n * nvec, 256), nseg), dim3(256), 0, s, n, nseg,
                       nvec, on, x, y);
    MBL_CHECK_LAUNCH();
}

void launch_shift_seg(int nseg, int64_t n, const double *x, SegVals shift, double *y,
                      hipStream_t s) {
    MBL_REQUIRE(nseg >= 0 && nseg <= MBL_SEG_MAX, MBL_EINVAL, "shift_seg: at most 16 segments");
    if (n == 0 || nseg == 0) return;
    hipLaunchKernelGGL(k_shift_seg, dim3(grid_for(n, 256), nseg), dim3(256), 0, s, n, x, shift, y);
    MBL_CHECK_LAUNCH();
}

void launch_copy(int64_t count, const double *x, double *y, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(count, 256)), dim3(256), 0, s, count, x, y);
    MBL_CHECK_LAUNCH();
}

void launch_axpy(int64_t count, double a, const double *x, double *y, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(count, 256)), dim3(256), 0, s, count, a, x, y);
    MBL_CHECK_LAUNCH();
}

}  // namespace mbl
