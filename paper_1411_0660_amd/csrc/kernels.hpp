// kernels.hpp -- host-callable launch wrappers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mbl {

// Segmented launches: nseg independent problems of the same size n whose
// vectors are stacked (segment s is rows [s n, (s + 1) n) of a packed column,
// ld = nseg n), each processed with exactly the arithmetic of a lone launch.
constexpr int MBL_SEG_MAX = 16;
struct SegSeeds {
    uint64_t seed[MBL_SEG_MAX];
};
struct SegVals {
    double v[MBL_SEG_MAX];
};

// ---- basis, ranking, assembly (k_basis.hip) ---------------------------------
void launch_fields(int L, double h, uint64_t seed, double *out, hipStream_t s);
void launch_basis(int L, int64_t dim, uint32_t *basis, hipStream_t s);
void launch_rank(int L, const uint32_t *words, int64_t count, int64_t *ranks, hipStream_t s);
// rowptr[dim+1] (exclusive scan of per-row counts); scratch >= scan_scratch_bytes(dim)
size_t scan_scratch_bytes(int64_t n);
void launch_row_ptr(int L, int64_t dim, const uint32_t *basis, int32_t *rowptr,
                    void *scratch, hipStream_t s);
void launch_fill_csr(int L, int64_t dim, const uint32_t *basis, const int32_t *rowptr,
                     int32_t *col, hipStream_t s);
void launch_diag(int L, double J, const double *fields, int64_t dim, const uint32_t *basis,
                 double *diag, hipStream_t s);

// ---- sparse and dense FP64 level-1/2/3 helpers (k_blas.hip) -----------------
// segmented variants (see MBL_SEG_MAX): segment s offsets its operands by
// s * seg* elements; partial-sum scratch grows nseg times
void launch_gemm_tn_seg(int nseg, int64_t n, int k, int b, const double *A, int64_t lda,
                        int64_t segA, const double *B, int64_t ldb, int64_t segB, double *C,
                        int64_t segC, double *partials, int nparts, hipStream_t s);
void launch_gemm_nn_seg(int nseg, int64_t n, int k, int b, double alpha, const double *A,
                        int64_t lda, int64_t segA, const double *Y, int ldy, int64_t segY,
                        double beta, double *C, int64_t ldc, int64_t segC, hipStream_t s);
void launch_small_chol_batch(int count, int b, const double *G, int64_t segG, double *R,
                             int64_t segR, double *Rinv, int64_t segRi, int *flag, int64_t segF,
                             double rel_tiny, hipStream_t s);
void launch_fill_start_seg(int nseg, int64_t n, int nvec, const uint64_t *seeds, double *v,
                           int64_t ld, hipStream_t s);
void launch_coldot_seg(int nseg, int64_t n, int ncol, const double *A, int64_t lda,
                       const double *B, int64_t ldb, int64_t seg, double *out, double *partials,
                       int nparts, hipStream_t s);
void launch_sub_scaled_cols_seg(int nseg, int64_t n, int ncol, const double *e, const double *X,
                                int64_t ldx, double *Y, int64_t ldy, hipStream_t s);
// rows of segment s of a block-diagonal H: [s n, (s + 1) n), CSR columns global
void launch_residual_seg(int nseg, int64_t n, const int32_t *rowptr, const int32_t *col,
                         const double *diag, double offv, double shift, int nvec, const double *b,
                         const double *x, double *r, double *partials, int nparts, hipStream_t s);
// y[s n + i] = x[s n + i] - shift.v[s] (one shift per segment)
void launch_shift_seg(int nseg, int64_t n, const double *x, SegVals shift, double *y,
                      hipStream_t s);
// y += x on the segments s with on[s] != 0 (device flags)
void launch_axpy_masked(int64_t n, int nseg, int nvec, const int *on, const double *x, double *y,
                        hipStream_t s);

// y = (H - shift) x for nvec column-major vectors; off-diagonal value offv.
void launch_spmv(int64_t n, const int32_t *rowptr, const int32_t *col, const double *diag,
                 double offv, double shift, int nvec, const double *x, double *y, hipStream_t s);
// r = b - (H - shift) x, plus per-block partial sums of |r|^2, |x|^2, |b|^2
void launch_residual(int64_t n, const int32_t *rowptr, const int32_t *col, const double *diag,
                     double offv, double shift, int nvec, const double *b, const double *x,
                     double *r, double *partials, int nparts, hipStream_t s);
// C[k x b] = A[n x k]^T B[n x b], deterministic two-level reduction
void launch_gemm_tn(int64_t n, int k, int b, const double *A, int64_t lda, const double *B,
                    int64_t ldb, double *C, double *partials, int nparts, hipStream_t s);
int gemm_tn_parts(int64_t n);
// C[n x b] = beta C + alpha A[n x k] Y[k x b] (Y in device memory, column-major ldy)
void launch_gemm_nn(int64_t n, int k, int b, double alpha, const double *A, int64_t lda,
                    const double *Y, int ldy, double beta, double *C, int64_t ldc, hipStream_t s);
// x[idx[i]] style permutations for nvec vectors
void launch_gather(int64_t n, int nvec, const int32_t *idx, const double *x, double *y,
                   hipStream_t s);
void launch_fill_start(int64_t n, int nvec, uint64_t seed, double *v, hipStream_t s);
void launch_copy(int64_t count, const double *x, double *y, hipStream_t s);
void launch_axpy(int64_t count, double a, const double *x, double *y, hipStream_t s);
void launch_coldot(int64_t n, int ncol, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *out, double *partials, int nparts, hipStream_t s);
// G = R^T R (b x b, b <= 16): R and R^-1 (upper, column-major) on the device;
// *flag = 1 if a pivot fell below rel_tiny * max diag
void launch_small_chol(int b, const double *G, double *R, double *Rinv, int *flag,
                       double rel_tiny, hipStream_t s);
// per-column dots of W against nb stacked blocks (block i at V + i bs, n x nrhs,
// ld n): out[i + j nb]; partials >= nparts * nb * nrhs, nb <= 32
void launch_bdot(int64_t n, int nb, int nrhs, const double *V, int64_t bs, const double *W,
                 double *out, double *partials, int nparts, hipStream_t s);
// out[:, j] = beta out[:, j] + alpha sum_i coef[i + j nb] V_i[:, j]  (coef on the device)
void launch_bcomb(int64_t n, int nb, int nrhs, const double *V, int64_t bs, const double *coef,
                  double alpha, double beta, double *out, hipStream_t s);
void launch_sub_scaled_cols(int64_t n, int ncol, const double *e, const double *X, int64_t ldx,
                            double *Y, int64_t ldy, hipStream_t s);


// ---- small dense symmetric eigenproblems (k_jacobi.hip) ---------------------
// A (m x m symmetric, column-major, overwritten) -> eigenvalues w[m] (unsorted)
// and eigenvectors V (m x m, column j for w[j]); *info = sweeps used or -1;
// m <= 1024.
// count independent matrices at strides m^2 (A, V), m (w), 1 (info), each
// with its own threshold tol_abs[k] (device), one workgroup each.  general:
// use the kernel of the larger orders also for m <= 128 (same results; a
// check of the two kernels against each other)
void launch_jacobi_eig_batch(int count, int m, double *A, double *V, double *w, int *info,
                             const double *tol_abs, hipStream_t s, bool general = false);

}  // namespace mbl
