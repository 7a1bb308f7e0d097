// k_trsv.hip -- forward and backward substitution through the multifrontal
// factors on gfx950: the operator (H - sigma)^-1 applied inside the Krylov
// method of section "Numerical method".
//
// The factor streams from HBM once per pass, shared by a block of up to 16
// right-hand sides (vectors stay FP64 whatever the factor precision).  The
// SB x SB diagonal blocks of L11 and U11 are stored inverted and folded into
// the panels beside them (L~ = L Linv_tt below, U~ = U Uinv_tt above; see
// k_front.hip), so one launch per solve block and tree level does both the
// diagonal product and the update of the other rows, from the same input:
//   forward (leaves to root), front f:
//     V = P([b(pivots); 0] + children's updates)        (row-parallel gather)
//     block t:  Y_t = Linv_tt V_t  and  V[rows below] -= L~[., t] V_t
//     afterwards Y = L11^-1 P b and V[p:m] is the update the parent gathers.
//   backward (root to leaves):
//     V[p:m] = x(contribution rows); Y -= U12 V[p:m]   (64 x 256 tiles, fixed-order sum)
//     block t from the last:  V_t = Uinv_tt Y_t  and  Y[rows above] -= U~[., t] Y_t
//     afterwards V[0:p] = x of the pivots.
// Work items are 64 rows x one SB block: the four waves of a workgroup take a
// quarter of the columns each and are summed through LDS.
#include <type_traits>

#include "common.hpp"
#include "frontal.hpp"

namespace mbl {
namespace {

constexpr int MAXRHS = 16;
constexpr int RW = 64;          // rows per update work item (one per lane)
constexpr int CQ = SB / 4;      // columns per wave

__device__ __forceinline__ int find_task(const int64_t *prefix, int n, int64_t w) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// row-parallel gather of the forward right-hand side of every front
// (including its children's updates and the row permutation of its pivots)
__global__ __launch_bounds__(256) void k_fwd_gather(const FrontDesc *__restrict__ fd,
                                                    const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ prow,
                                                    const int32_t *__restrict__ inv_ptr,
                                                    const int2 *__restrict__ inv_src, TaskList tl,
                                                    int nrhs, const double *__restrict__ b,
                                                    int64_t ldb, double *vec) {
    int k = find_task(tl.prefix, tl.n, blockIdx.x);
    FrontDesc d = fd[tl.fronts[k]];
    int i = (int)(blockIdx.x - tl.prefix[k]) * 256 + threadIdx.x;
    if (i >= d.m) return;
    int u = (i < d.p) ? prow[d.first + i] : i;        // row before the interchanges
    double val[MAXRHS];
    for (int r = 0; r < nrhs; r++)
        val[r] = (u < d.p) ? b[perm[d.first + u] + (int64_t)r * ldb] : 0.0;
    int64_t base = d.voff;                            // inverse relative map of this front
    int32_t a = inv_ptr[d.cptr_inv + u], e = inv_ptr[d.cptr_inv + u + 1];
    for (int32_t q = a; q < e; q++) {
        int2 s = inv_src[q];                          // (child front, row of its update)
        FrontDesc c = fd[s.x];
        const double *cu = vec + c.voff + c.p + s.y;
        for (int r = 0; r < nrhs; r++) val[r] += cu[(int64_t)r * c.m];
    }
    for (int r = 0; r < nrhs; r++) vec[base + i + (int64_t)r * d.m] = val[r];
}

// out rows of one 64-row chunk from M[rows, SB block] times src (LDS):
//   MODE 0: out -= M src            (panel update, in place)
//   MODE 1: out  = src_i + sum_{j<i} M_ij src_j   (unit-lower inverse block)
//   MODE 2: out  = sum_{j>=i} M_ij src_j           (upper inverse block)
// lane = row, wave = quarter of the columns, sum over waves through LDS.
template <class T, int NR, int MODE>
__device__ __forceinline__ void chunk_apply(const T *__restrict__ Mrow0, int64_t m, int ncols,
                                            int nrows, int rowoff, const double (*src)[NR],
                                            double (*red)[RW][NR], double *out, int64_t ldo) {
    int lane = threadIdx.x % RW, w = threadIdx.x / RW;
    int j0 = w * CQ, j1 = min(j0 + CQ, ncols);
    int i = rowoff + lane;                       // row index inside the diagonal block
    if (MODE == 1) j1 = min(j1, i);
    if (MODE == 2) j0 = max(j0, i);
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
    if (lane < nrows) {
        const T *Mr = Mrow0 + lane;
#pragma unroll 8
        for (int j = j0; j < j1; j++) {
            double x = (double)Mr[(int64_t)j * m];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] += x * src[j][r];
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) red[w][lane][r] = acc[r];
    __syncthreads();
    if (w == 0 && lane < nrows) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            double sum = red[0][lane][r] + red[1][lane][r] + red[2][lane][r] + red[3][lane][r];
            double *o = out + lane + (int64_t)r * ldo;
            if (MODE == 0) *o -= sum;
            else if (MODE == 1) *o = src[i][r] + sum;
            else *o = sum;
        }
    }
}

// one solve block t of every listed front: the first ceil(st/64) items apply
// the inverted diagonal block, the others update the remaining rows
template <class T, int NR, bool FWD>
__global__ __launch_bounds__(SB) void k_solve_step(const T *__restrict__ arena,
                                                   const FrontDesc *__restrict__ fd, TaskList tl,
                                                   int t, double *vec, double *yv) {
    __shared__ double src[SB][NR];
    __shared__ double red[4][RW][NR];
    int k = find_task(tl.prefix, tl.n, blockIdx.x);
    FrontDesc d = fd[tl.fronts[k]];
    int w = (int)(blockIdx.x - tl.prefix[k]);
    int m = d.m, p = d.p, t0 = t * SB, st = min(SB, p - t0), tend = t0 + st;
    int nA = (st + RW - 1) / RW;
    double *V = vec + d.voff;          // ld m
    double *Y = yv + d.yoff;           // ld p
    const double *S = FWD ? V + t0 : Y + t0;
    int64_t lds = FWD ? m : p;
    for (int e = threadIdx.x; e < st * NR; e += blockDim.x) {
        int j = e % st, r = e / st;
        src[j][r] = S[j + (int64_t)r * lds];
    }
    __syncthreads();
    const T *F = arena + d.off;
    if (w < nA) {
        int i0 = w * RW;
        const T *M = F + (t0 + i0) + (int64_t)t0 * m;
        if (FWD) chunk_apply<T, NR, 1>(M, m, st, min(RW, st - i0), i0, src, red, Y + t0 + i0, p);
        else chunk_apply<T, NR, 2>(M, m, st, min(RW, st - i0), i0, src, red, V + t0 + i0, m);
    } else {
        int c = w - nA;
        if (FWD) {
            int r0 = tend + c * RW;
            chunk_apply<T, NR, 0>(F + r0 + (int64_t)t0 * m, m, st, min(RW, m - r0), 0, src, red,
                                  V + r0, m);
        } else {
            int r0 = c * RW;
            chunk_apply<T, NR, 0>(F + r0 + (int64_t)t0 * m, m, st, min(RW, t0 - r0), 0, src, red,
                                  Y + r0, p);
        }
    }
}

__global__ __launch_bounds__(256) void k_bwd_gather(const FrontDesc *__restrict__ fd,
                                                    const int32_t *__restrict__ contrib,
                                                    TaskList tl, int nrhs,
                                                    const double *__restrict__ xnew, int64_t n,
                                                    double *vec) {
    int k = find_task(tl.prefix, tl.n, blockIdx.x);
    FrontDesc d = fd[tl.fronts[k]];
    int i = (int)(blockIdx.x - tl.prefix[k]) * 256 + threadIdx.x;
    int cc = d.m - d.p;
    if (i >= cc) return;
    int32_t g = contrib[d.cptr + i];
    double *v = vec + d.voff + d.p + i;
    for (int r = 0; r < nrhs; r++) v[(int64_t)r * d.m] = xnew[g + (int64_t)r * n];
}

// partial U12 x_c over one 64-row x SB-column tile
template <class T, int NR>
__global__ __launch_bounds__(SB) void k_bwd_u12(const T *__restrict__ arena,
                                                const FrontDesc *__restrict__ fd, TaskList tl,
                                                const double *__restrict__ vec,
                                                double *__restrict__ part) {
    __shared__ double src[SB][NR];
    __shared__ double red[4][RW][NR];
    int k = find_task(tl.prefix, tl.n, blockIdx.x);
    FrontDesc d = fd[tl.fronts[k]];
    int w = (int)(blockIdx.x - tl.prefix[k]);
    int m = d.m, p = d.p, c = m - p;
    int nrc = (p + RW - 1) / RW;
    int rc = w % nrc, cc = w / nrc;
    int c0 = cc * SB, cw = min(SB, c - c0);
    const double *v = vec + d.voff;
    for (int e = threadIdx.x; e < cw * NR; e += blockDim.x) {
        int j = e % cw, r = e / cw;
        src[j][r] = v[p + c0 + j + (int64_t)r * m];
    }
    __syncthreads();
    int lane = threadIdx.x % RW, wv = threadIdx.x / RW;
    int row = rc * RW + lane;
    int j0 = wv * CQ, j1 = min(j0 + CQ, cw);
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
    if (row < p) {
        const T *U = arena + d.off + row + (int64_t)(p + c0) * m;
#pragma unroll 8
        for (int j = j0; j < j1; j++) {
            double x = (double)U[(int64_t)j * m];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] += x * src[j][r];
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) red[wv][lane][r] = acc[r];
    __syncthreads();
    if (wv == 0 && row < p)
#pragma unroll
        for (int r = 0; r < NR; r++)
            part[d.poff + ((int64_t)cc * MAXRHS + r) * p + row] =
                red[0][lane][r] + red[1][lane][r] + red[2][lane][r] + red[3][lane][r];
}

template <int NR>
__global__ __launch_bounds__(256) void k_bwd_u12_reduce(const FrontDesc *__restrict__ fd,
                                                        TaskList tl, double *yv,
                                                        const double *__restrict__ part) {
    int k = find_task(tl.prefix, tl.n, blockIdx.x);
    FrontDesc d = fd[tl.fronts[k]];
    int row = (int)(blockIdx.x - tl.prefix[k]) * 256 + threadIdx.x;
    int m = d.m, p = d.p, ncc = (m - p + SB - 1) / SB;
    if (row >= p) return;
    double *y = yv + d.yoff;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double s = 0.0;
        for (int q = 0; q < ncc; q++) s += part[d.poff + ((int64_t)q * MAXRHS + r) * p + row];
        y[row + (int64_t)r * p] -= s;
    }
}

__global__ __launch_bounds__(256) void k_bwd_scatter(const FrontDesc *__restrict__ fd,
                                                     const int32_t *__restrict__ perm, TaskList tl,
                                                     int nrhs, const double *__restrict__ vec,
                                                     double *xnew, int64_t n, double *xout,
                                                     int64_t ldx) {
    int k = find_task(tl.prefix, tl.n, blockIdx.x);
    FrontDesc d = fd[tl.fronts[k]];
    int i = (int)(blockIdx.x - tl.prefix[k]) * 256 + threadIdx.x;
    if (i >= d.p) return;
    int g = d.first + i;
    int32_t o = perm[g];
    for (int r = 0; r < nrhs; r++) {
        double x = vec[d.voff + i + (int64_t)r * d.m];
        xnew[g + (int64_t)r * n] = x;
        xout[o + (int64_t)r * ldx] = x;
    }
}

inline int rhs_class(int nrhs) { return nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : 16; }

}  // namespace

// run f with the compile-time right-hand-side count NR >= nrhs (1, 2, 4, 8, 16)
template <class F>
void rhs_dispatch(int nrhs, F &&f) {
    switch (rhs_class(nrhs)) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        default: f(std::integral_constant<int, 16>{}); break;
    }
}

void launch_fwd_gather(const FrontDesc *fd, const int32_t *perm, const int32_t *prow,
                       const int32_t *inv_ptr, const int2 *inv_src, TaskList tl, int nrhs,
                       const double *b, int64_t ldb, double *vec, hipStream_t s) {
    if (tl.total == 0) return;
    hipLaunchKernelGGL(k_fwd_gather, dim3((unsigned)tl.total), dim3(256), 0, s, fd, perm, prow,
                       inv_ptr, inv_src, tl, nrhs, b, ldb, vec);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_solve_step(const T *arena, const FrontDesc *fd, TaskList tl, int t, int nrhs, bool fwd,
                       double *vec, double *yv, hipStream_t s) {
    if (tl.total == 0) return;
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        if (fwd)
            k_solve_step<T, NR, true><<<dim3((unsigned)tl.total), dim3(SB), 0, s>>>(arena, fd, tl, t,
                                                                                    vec, yv);
        else
            k_solve_step<T, NR, false><<<dim3((unsigned)tl.total), dim3(SB), 0, s>>>(arena, fd, tl,
                                                                                     t, vec, yv);
    });
    MBL_CHECK_LAUNCH();
}

void launch_bwd_gather(const FrontDesc *fd, const int32_t *contrib, TaskList tl, int nrhs,
                       const double *xnew, int64_t n, double *vec, hipStream_t s) {
    if (tl.total == 0) return;
    hipLaunchKernelGGL(k_bwd_gather, dim3((unsigned)tl.total), dim3(256), 0, s, fd, contrib, tl,
                       nrhs, xnew, n, vec);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_bwd_u12(const T *arena, const FrontDesc *fd, TaskList tl, int nrhs, const double *vec,
                    double *part, hipStream_t s) {
    if (tl.total == 0) return;
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        k_bwd_u12<T, NR><<<dim3((unsigned)tl.total), dim3(SB), 0, s>>>(arena, fd, tl, vec, part);
    });
    MBL_CHECK_LAUNCH();
}

void launch_bwd_u12_reduce(const FrontDesc *fd, TaskList tl, int nrhs, double *yv,
                           const double *part, hipStream_t s) {
    if (tl.total == 0) return;
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        k_bwd_u12_reduce<NR><<<dim3((unsigned)tl.total), dim3(256), 0, s>>>(fd, tl, yv, part);
    });
    MBL_CHECK_LAUNCH();
}

void launch_bwd_scatter(const FrontDesc *fd, const int32_t *perm, TaskList tl, int nrhs,
                        const double *vec, double *xnew, int64_t n, double *xout, int64_t ldx,
                        hipStream_t s) {
    if (tl.total == 0) return;
    hipLaunchKernelGGL(k_bwd_scatter, dim3((unsigned)tl.total), dim3(256), 0, s, fd, perm, tl, nrhs,
                       vec, xnew, n, xout, ldx);
    MBL_CHECK_LAUNCH();
}

#define MBL_INST_TRSV(T)                                                                          \
    template void launch_solve_step<T>(const T *, const FrontDesc *, TaskList, int, int, bool,    \
                                       double *, double *, hipStream_t);                          \
    template void launch_bwd_u12<T>(const T *, const FrontDesc *, TaskList, int, const double *,  \
                                    double *, hipStream_t);

MBL_INST_TRSV(float)
MBL_INST_TRSV(double)

}  // namespace mbl
