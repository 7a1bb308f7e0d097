// k_trsv.hip -- forward and backward substitution through the multifrontal
// factors on gfx950: the operator (H - sigma)^-1 applied inside the Krylov
// method of section "Numerical method".
//
// The factor streams from HBM once per pass, shared by a block of up to 16
// right-hand sides (vectors stay FP64 whatever the factor precision).  The
// SSB x SSB diagonal blocks of L11 and U11 (two factorization blocks) are
// stored inverted and folded into the panels beside them (L~ = L Linv_tt
// below, U~ = U Uinv_tt above; see k_front.hip), so one launch per solve
// block and tree level does both the diagonal product and the update of the
// other rows, from the same input:
//   forward (leaves to root), front f:
//     V = P([b(pivots); 0] + children's updates)        (row-parallel gather)
//     block t:  Y_t = Linv_tt V_t  and  V[rows below] -= L~[., t] V_t
//     afterwards Y = L11^-1 P b and V[p:m] is the update the parent gathers.
//   backward (root to leaves):
//     Y -= U12 x(contribution rows)   (64 x 256 tiles reading x through the
//                                      contribution lists, fixed-order sum)
//     block t from the last:  x_t = Uinv_tt Y_t  and  Y[rows above] -= U~[., t] Y_t,
//     x_t written straight to the solution vectors (by new and original index).
// Work items of a step are STEP_RW rows x one SSB block (the off-diagonal
// products: 64 rows x SB columns): the 8 or 16 waves of a workgroup take an
// equal share of the columns each and are summed through LDS, which keeps the
// dependent load chain of a lane short.
#include <type_traits>

#include "common.hpp"
#include "frontal.hpp"

namespace mbl {
namespace {

constexpr int MAXRHS = 16;
constexpr int RW = 64;          // rows per update work item (one per lane)

// Workgroup b of a launch is dispatched to XCD b % 8 (round robin); each XCD
// takes a contiguous range of the work items instead, so that neighbouring
// row chunks of one column run, which share the cache line at their boundary,
// are read through the same L2.  A bijection of [0, n).
__device__ __forceinline__ unsigned xcd_item(unsigned b, unsigned n) {
    const unsigned x = b % 8, s = b / 8, q = n / 8, r = n % 8;
    return x * q + min(x, r) + s;
}

// column groups (waves) per work item (STEP_RW rows of a solve step, 64 rows of
// an L21 / U12 tile): 16 for up to 8 right-hand sides,
// 8 for 16 (LDS: the SSB x NR source block plus CG x 64 x NR partial sums)
template <int NR> struct StepCfg {
    static constexpr int CG = NR <= 8 ? 16 : 8;
    static constexpr int THREADS = 64 * CG;
    static constexpr int CW = SSB / CG;         // columns per wave (solve steps)
    static constexpr int CWU = SB / CG;         // columns per wave (U12 tiles)
};

// row-parallel gather of the forward right-hand side of every front
// (including its children's updates and the row permutation of its pivots);
// inv_src holds, per contribution, the element of the child's update row in
// the solve vectors and the child's order (stride between right-hand sides)
template <int NR>
__global__ __launch_bounds__(256) void k_fwd_gather(const FrontDesc *__restrict__ fd,
                                                    const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ prow,
                                                    const int32_t *__restrict__ inv_ptr,
                                                    const int2 *__restrict__ inv_src, TaskList tl,
                                                    int nrhs, const double *__restrict__ b,
                                                    int64_t ldb, double *vec) {
    const int2 tk = tl.items[blockIdx.x];
    FrontDesc d = fd[tk.x];
    int i = tk.y * 256 + threadIdx.x;
    if (i >= d.m) return;
    int u = (i < d.p) ? prow[d.first + i] : i;        // row before the interchanges
    int32_t a = inv_ptr[d.cptr_inv + u], e = inv_ptr[d.cptr_inv + u + 1];
    double val[NR];
    if (u < d.p) {
        int32_t g = perm[d.first + u];
#pragma unroll
        for (int r = 0; r < NR; r++) val[r] = r < nrhs ? b[g + (int64_t)r * ldb] : 0.0;
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) val[r] = 0.0;
    }
    for (int32_t q = a; q < e; q++) {
        int2 sv = inv_src[q];
        const double *cu = vec + sv.x;
#pragma unroll
        for (int r = 0; r < NR; r++) val[r] += cu[(int64_t)r * sv.y];
    }
    double *o = vec + d.voff + i;
#pragma unroll
    for (int r = 0; r < NR; r++) o[(int64_t)r * d.m] = val[r];
}

// One work item of solve block t: STEP_RW rows, out rows from M[rows, SSB
// block] and the block's source values src (LDS):
//   mode 0: out -= M src                            (panel update, in place)
//   mode 1: out  = src_i + sum_{j<i} M_ij src_j     (unit-lower inverse block)
//   mode 2: out  = sum_{j>=i} M_ij src_j            (upper inverse block)
// Each wave takes an equal share of the columns; inside a wave, lane % STEP_RW
// is the row and lane / STEP_RW one of 64 / STEP_RW interleaved column slices,
// so one load brings 64 / STEP_RW adjacent column segments of STEP_RW rows.
// The slices are summed by a butterfly over the wave and the waves in a fixed
// order through LDS.  The factor entries (and the rows updated in place) are
// loaded before the source block is staged, so the two memory round trips
// overlap.
// In the backward pass the diagonal products write the solution of their rows
// straight to xnew (by new index) and xout (by original index).
template <class T, int NR, bool FWD>
__global__ __launch_bounds__(StepCfg<NR>::THREADS) void k_solve_step(
    const T *__restrict__ arena, const FrontDesc *__restrict__ fd, TaskList tl, int t,
    double *vec, double *yv, BwdIO bio) {
    constexpr int CG = StepCfg<NR>::CG, CW = StepCfg<NR>::CW;
    constexpr int HG = CG / 2;                       // partial sums: two phases of CG / 2
    constexpr int R = STEP_RW, LS = 64 / R, CQ = CW / LS;
    static_assert(CW % LS == 0, "columns per wave split over the slices");
    __shared__ double src[SSB][NR];
    __shared__ double red[HG][R][NR];
    const int2 tk = tl.items[xcd_item(blockIdx.x, gridDim.x)];
    const FrontDesc d = fd[tk.x];
    const int w = tk.y;
    const int m = d.m, p = d.p, t0 = t * SSB, st = min(SSB, p - t0), tend = t0 + st;
    const int nA = (st + R - 1) / R;
    double *V = vec + d.voff;          // ld m
    double *Y = yv + d.yoff;           // ld p
    int mode, r0, nrows, rowoff = 0;
    double *out;
    int64_t ldo;
    if (w < nA) {                      // diagonal product
        rowoff = w * R;
        r0 = t0 + rowoff;
        nrows = min(R, st - rowoff);
        mode = FWD ? 1 : 2;
        out = FWD ? Y + r0 : V + r0;
        ldo = FWD ? p : m;
    } else if (FWD) {                  // pivot rows below the block (the contribution
        r0 = tend + (w - nA) * R;      // rows are updated once per level by k_fwd_l21)
        nrows = min(R, p - r0);
        mode = 0;
        out = V + r0;
        ldo = m;
    } else {                           // pivot rows above the block
        r0 = (w - nA) * R;
        nrows = min(R, t0 - r0);
        mode = 0;
        out = Y + r0;
        ldo = p;
    }
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int rl = lane % R, sl = lane / R;
    const int i = rowoff + rl;         // row inside the diagonal block (modes 1, 2)
    const bool rowok = rl < nrows;
    double mv[CQ];
    {
        const T *Mr = arena + d.off + r0 + rl + (int64_t)(t0 + wv * CW + sl) * m;
#pragma unroll
        for (int q = 0; q < CQ; q++) {
            const int j = wv * CW + q * LS + sl;
            const bool ok = rowok && j < st && (mode == 0 || (mode == 1 ? j < i : j >= i));
            mv[q] = ok ? (double)Mr[(int64_t)q * LS * m] : 0.0;
        }
    }
    double prev[NR];
    if (mode == 0 && wv == 0 && sl == 0 && rowok) {
#pragma unroll
        for (int r = 0; r < NR; r++) prev[r] = out[rl + (int64_t)r * ldo];
    }
    {
        const double *S = FWD ? V + t0 : Y + t0;
        const int64_t lds = FWD ? m : p;
        for (int e = threadIdx.x; e < SSB * NR; e += blockDim.x) {
            int j = e % SSB, r = e / SSB;
            src[j][r] = j < st ? S[j + (int64_t)r * lds] : 0.0;
        }
    }
    __syncthreads();
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
#pragma unroll
    for (int q = 0; q < CQ; q++) {
        const double x = mv[q];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] += x * src[wv * CW + q * LS + sl][r];
    }
    // slices of a row: butterfly (every lane of the row ends with the same sum)
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) {
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] += __shfl_xor(acc[r], off);
    }
    // fixed-order sum over the waves: g + HG into g, then g = 0 .. HG-1
    if (wv >= HG && sl == 0) {
#pragma unroll
        for (int r = 0; r < NR; r++) red[wv - HG][rl][r] = acc[r];
    }
    __syncthreads();
    if (wv < HG && sl == 0) {
#pragma unroll
        for (int r = 0; r < NR; r++) red[wv][rl][r] += acc[r];
    }
    __syncthreads();
    if (wv == 0 && sl == 0 && rowok) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            double sum = red[0][rl][r];
#pragma unroll
            for (int g = 1; g < HG; g++) sum += red[g][rl][r];
            if (mode == 2) {               // solution of pivot row r0 + rl
                if (r < bio.nrhs) {
                    const int g = d.first + r0 + rl;
                    bio.xnew[g + (int64_t)r * bio.n] = sum;
                    bio.xout[bio.perm[g] + (int64_t)r * bio.ldx] = sum;
                }
                continue;
            }
            double *o = out + rl + (int64_t)r * ldo;
            if (mode == 0) *o = prev[r] - sum;
            else *o = src[i][r] + sum;
        }
    }
}

// The off-diagonal products of the solves, as 64-row x SB-column tiles of
// partial sums (a fixed-order reduction over the column chunks follows):
//  - forward, contribution rows (U12 = false): once every solve block of a
//    front is done, V[0:p] holds the source values of all blocks (a block's
//    rows are not touched after its own step), so V[p:m] -= L~21 V[0:p] in one
//    pass with the folded panel L~21 = L[p:m, 0:p] (per block times its
//    inverse); partial sums of tile (row chunk, column chunk cc) go to part;
//    k_fwd_l21_reduce sums them;
//  - backward (U12 = true): Y -= U12 x_c over the pivot rows, x of the
//    contribution rows (pivots of ancestors, already solved) read through the
//    front's contribution-row list; k_bwd_u12_reduce sums them.
// A workgroup takes IPW consecutive tiles of the task list (1 or 2, chosen per
// tree level by the solve autotuner): their factor entries are all loaded
// before any is used, so IPW = 2 keeps twice the bytes in flight per lane.
// The arithmetic of a row does not depend on IPW: the same column split over
// the waves and the same fixed-order sums.
template <class T, int NR, int IPW, bool U12>
__global__ __launch_bounds__(StepCfg<NR>::THREADS) void k_offdiag(
    const T *__restrict__ arena, const FrontDesc *__restrict__ fd, TaskList tl,
    const double *__restrict__ vec, const int32_t *__restrict__ contrib,
    const double *__restrict__ xnew, int64_t n, double *__restrict__ part) {
    constexpr int CG = StepCfg<NR>::CG, CW = StepCfg<NR>::CWU, HG = CG / 2;
    __shared__ double src[IPW][SB][NR];
    __shared__ double red[HG][RW][NR];
    const int lane = threadIdx.x % RW, wv = threadIdx.x / RW;
    const int64_t base = (int64_t)xcd_item(blockIdx.x, gridDim.x) * IPW;
    FrontDesc d[IPW];
    int row[IPW], nr[IPW], cc[IPW], c0[IPW], cw[IPW];
    bool live[IPW];
    double mv[IPW][CW];
#pragma unroll
    for (int k = 0; k < IPW; k++) {
        live[k] = base + k < tl.total;
        const int2 tk = tl.items[live[k] ? base + k : base];
        d[k] = fd[tk.x];
        const int w = tk.y, m = d[k].m, p = d[k].p, c = m - p;
        nr[k] = U12 ? p : c;                          // rows of the product
        const int ncol = U12 ? c : p;                 // its columns
        const int nrc = (nr[k] + RW - 1) / RW;
        const int rc = w % nrc;
        cc[k] = w / nrc;
        c0[k] = cc[k] * SB;
        cw[k] = min(SB, ncol - c0[k]);
        row[k] = rc * RW + lane;
        const T *M = U12 ? arena + d[k].off + row[k] + (int64_t)(p + c0[k] + wv * CW) * m
                         : arena + d[k].off + p + row[k] + (int64_t)(c0[k] + wv * CW) * m;
        const bool rok = live[k] && row[k] < nr[k];
#pragma unroll
        for (int q = 0; q < CW; q++)
            mv[k][q] = (rok && wv * CW + q < cw[k]) ? (double)M[(int64_t)q * m] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < IPW; k++) {
        if (!live[k]) continue;                       // uniform over the workgroup
        const int32_t *cr = contrib + d[k].cptr + c0[k];
        const double *v = vec + d[k].voff;
        for (int e = threadIdx.x; e < SB * NR; e += blockDim.x) {
            int j = e % SB, r = e / SB;
            double x = 0.0;
            if (j < cw[k]) x = U12 ? xnew[cr[j] + (int64_t)r * n] : v[c0[k] + j + (int64_t)r * d[k].m];
            src[k][j][r] = x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPW; k++) {
        if (!live[k]) break;
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] = 0.0;
#pragma unroll
        for (int q = 0; q < CW; q++) {
            const double x = mv[k][q];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] += x * src[k][wv * CW + q][r];
        }
        if (k > 0) __syncthreads();                   // red of the previous tile is read
        if (wv >= HG) {
#pragma unroll
            for (int r = 0; r < NR; r++) red[wv - HG][lane][r] = acc[r];
        }
        __syncthreads();
        if (wv < HG) {
#pragma unroll
            for (int r = 0; r < NR; r++) red[wv][lane][r] += acc[r];
        }
        __syncthreads();
        if (wv == 0 && row[k] < nr[k])
#pragma unroll
            for (int r = 0; r < NR; r++) {
                double sum = red[0][lane][r];
#pragma unroll
                for (int g = 1; g < HG; g++) sum += red[g][lane][r];
                part[d[k].poff + ((int64_t)cc[k] * MAXRHS + r) * nr[k] + row[k]] = sum;
            }
    }
}

template <int NR>
__global__ __launch_bounds__(256) void k_fwd_l21_reduce(const FrontDesc *__restrict__ fd,
                                                        TaskList tl, double *vec,
                                                        const double *__restrict__ part) {
    const int2 tk = tl.items[blockIdx.x];
    FrontDesc d = fd[tk.x];
    int row = tk.y * 256 + threadIdx.x;
    int m = d.m, p = d.p, c = m - p, ncc = (p + SB - 1) / SB;
    if (row >= c) return;
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) s[r] = 0.0;
    const double *pp = part + d.poff + row;
#pragma unroll 2
    for (int q = 0; q < ncc; q++)
#pragma unroll
        for (int r = 0; r < NR; r++) s[r] += pp[((int64_t)q * MAXRHS + r) * c];
    double *o = vec + d.voff + p + row;
#pragma unroll
    for (int r = 0; r < NR; r++) o[(int64_t)r * m] -= s[r];
}

template <int NR>
__global__ __launch_bounds__(256) void k_bwd_u12_reduce(const FrontDesc *__restrict__ fd,
                                                        TaskList tl, double *yv,
                                                        const double *__restrict__ part) {
    const int2 tk = tl.items[blockIdx.x];
    FrontDesc d = fd[tk.x];
    int row = tk.y * 256 + threadIdx.x;
    int m = d.m, p = d.p, ncc = (m - p + SB - 1) / SB;
    if (row >= p) return;
    double *y = yv + d.yoff;
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) s[r] = 0.0;
    const double *pp = part + d.poff + row;
#pragma unroll 2
    for (int q = 0; q < ncc; q++)
#pragma unroll
        for (int r = 0; r < NR; r++) s[r] += pp[((int64_t)q * MAXRHS + r) * p];
#pragma unroll
    for (int r = 0; r < NR; r++) y[row + (int64_t)r * p] -= s[r];
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
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        k_fwd_gather<NR><<<dim3((unsigned)tl.total), dim3(256), 0, s>>>(fd, perm, prow, inv_ptr,
                                                                         inv_src, tl, nrhs, b, ldb,
                                                                         vec);
    });
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_solve_step(const T *arena, const FrontDesc *fd, TaskList tl, int t, int nrhs, bool fwd,
                       double *vec, double *yv, BwdIO bio, hipStream_t s) {
    if (tl.total == 0) return;
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        constexpr int TH = StepCfg<NR>::THREADS;
        if (fwd)
            k_solve_step<T, NR, true><<<dim3((unsigned)tl.total), dim3(TH), 0, s>>>(arena, fd, tl, t,
                                                                                    vec, yv, bio);
        else
            k_solve_step<T, NR, false><<<dim3((unsigned)tl.total), dim3(TH), 0, s>>>(arena, fd, tl,
                                                                                     t, vec, yv, bio);
    });
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_bwd_u12(const T *arena, const FrontDesc *fd, TaskList tl, int nrhs,
                    const int32_t *contrib, const double *xnew, int64_t n, double *part, int ipw,
                    hipStream_t s) {
    if (tl.total == 0) return;
    const unsigned g1 = (unsigned)tl.total, g2 = (unsigned)((tl.total + 1) / 2);
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        constexpr int TH = StepCfg<NR>::THREADS;
        if (ipw == 2)
            k_offdiag<T, NR, 2, true><<<dim3(g2), dim3(TH), 0, s>>>(arena, fd, tl, nullptr, contrib,
                                                                    xnew, n, part);
        else
            k_offdiag<T, NR, 1, true><<<dim3(g1), dim3(TH), 0, s>>>(arena, fd, tl, nullptr, contrib,
                                                                    xnew, n, part);
    });
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_fwd_l21(const T *arena, const FrontDesc *fd, TaskList tl, int nrhs, const double *vec,
                    double *part, int ipw, hipStream_t s) {
    if (tl.total == 0) return;
    const unsigned g1 = (unsigned)tl.total, g2 = (unsigned)((tl.total + 1) / 2);
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        constexpr int TH = StepCfg<NR>::THREADS;
        if (ipw == 2)
            k_offdiag<T, NR, 2, false><<<dim3(g2), dim3(TH), 0, s>>>(arena, fd, tl, vec, nullptr,
                                                                     nullptr, 0, part);
        else
            k_offdiag<T, NR, 1, false><<<dim3(g1), dim3(TH), 0, s>>>(arena, fd, tl, vec, nullptr,
                                                                     nullptr, 0, part);
    });
    MBL_CHECK_LAUNCH();
}

void launch_fwd_l21_reduce(const FrontDesc *fd, TaskList tl, int nrhs, double *vec,
                           const double *part, hipStream_t s) {
    if (tl.total == 0) return;
    rhs_dispatch(nrhs, [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        k_fwd_l21_reduce<NR><<<dim3((unsigned)tl.total), dim3(256), 0, s>>>(fd, tl, vec, part);
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

#define MBL_INST_TRSV(T)                                                                          \
    template void launch_solve_step<T>(const T *, const FrontDesc *, TaskList, int, int, bool,    \
                                       double *, double *, BwdIO, hipStream_t);                   \
    template void launch_bwd_u12<T>(const T *, const FrontDesc *, TaskList, int, const int32_t *, \
                                    const double *, int64_t, double *, int, hipStream_t);          \
    template void launch_fwd_l21<T>(const T *, const FrontDesc *, TaskList, int, const double *,  \
                                    double *, int, hipStream_t);

MBL_INST_TRSV(float)
MBL_INST_TRSV(double)

}  // namespace mbl
