// k_front.hip -- numeric multifrontal LU of H - sigma on gfx950.
//
// The paper's shift-invert step rests on a parallel sparse LU of H - E
// (section "Numerical method").  Here every node of the nested-dissection tree
// is a dense front F (m x m, column-major, pivots first).  A front is
// assembled from the original entries of H - sigma and the contribution blocks
// of its children (extend-add, done as a gather so that each entry is written
// once), then partially factored: a right-looking
// blocked LU over its p pivot columns, panel width FNB.
//
// Pivoting: partial pivoting restricted to the FNB x FNB diagonal block of the
// current panel (rows outside the block are not candidates), with static pivot
// perturbation |u_jj| < thresh -> +-thresh.  The interchanges are applied to
// every column of the front (P A = L U with one row permutation per front,
// applied to the right-hand side by the forward solve).  FP64 iterative
// refinement of each solve absorbs the perturbations.
//
// Every launch covers all fronts of one tree level (independent subtrees), so
// the number of launches grows with the tree height times the panel count of
// the largest front per level, not with the number of fronts.
#include <algorithm>

#include "common.hpp"
#include "frontal.hpp"

namespace mbl {
namespace {

// Assembly of the fronts of one level from their children: every entry
// F[i][j] = sum over children s whose update rows include both front rows i
// and j of that child's updated entry (zero where no child contributes), so
// each entry is written exactly once and the level needs no zero fill; the
// original entries of H - sigma are added afterwards (k_front_assemble).  A
// work item is one front column: the children that hold column j are found
// once, then each lane sums its rows over them in child order.
template <class T>
__global__ __launch_bounds__(256) void k_front_pull(T *arena, const FrontDesc *__restrict__ fd,
                                                    const int32_t *__restrict__ pullmap,
                                                    const int32_t *__restrict__ child_ids,
                                                    TaskList tl) {
    __shared__ const T *colp[PULL_MAXCH];     // child column holding front column j
    __shared__ const int32_t *rowm[PULL_MAXCH];
    __shared__ int nsrc;
    const int2 tk = tl.items[blockIdx.x];
    const FrontDesc d = fd[tk.x];
    const int j = tk.y, m = d.m;
    if (threadIdx.x == 0) {
        int n = 0;
        for (int q = 0; q < d.nchild; q++) {
            const int32_t *pm = pullmap + d.pmoff + (int64_t)q * m;
            const int32_t cj = pm[j];
            if (cj < 0) continue;
            const FrontDesc c = fd[child_ids[d.child0 + q]];
            colp[n] = arena + c.off + (int64_t)(c.p + cj) * c.m + c.p;
            rowm[n] = pm;
            n++;
        }
        nsrc = n;
    }
    __syncthreads();
    const int ns = nsrc;
    T *out = arena + d.off + (int64_t)j * m;
    constexpr int U = 4;                      // rows per lane in flight
    for (int i0 = threadIdx.x; i0 < m; i0 += U * blockDim.x) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = T(0);
        for (int q = 0; q < ns; q++) {
            int32_t ci[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int i = i0 + u * blockDim.x;
                ci[u] = i < m ? rowm[q][i] : -1;
            }
            T x[U];
#pragma unroll
            for (int u = 0; u < U; u++) x[u] = ci[u] >= 0 ? colp[q][ci[u]] : T(0);
#pragma unroll
            for (int u = 0; u < U; u++) v[u] += x[u];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int i = i0 + u * blockDim.x;
            if (i < m) out[i] = v[u];
        }
    }
}

template <class T>
__global__ void k_front_assemble(T *arena, const FrontDesc *__restrict__ fd, int64_t count,
                                 const int32_t *__restrict__ efront,
                                 const int32_t *__restrict__ epos,
                                 const int32_t *__restrict__ esrc,
                                 const double *__restrict__ diag, double sigma, double offv) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    int32_t src = esrc[e];
    double v = (src >= 0) ? diag[src] - sigma : offv;
    T *F = arena + fd[efront[e]].off;
    F[epos[e]] += (T)v;
}

// max of v over the 64 lanes of a wave by DPP lane moves (quad swaps, row
// mirrors, row broadcasts): a few cycles per step instead of an LDS round
// trip; the result is valid in lane 63.  Lanes a row mask leaves out keep
// their own value.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_step_max(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    return fmax(v, __hiloint2double(hi2, lo2));
}
__device__ __forceinline__ double wave_max(double v) {
    v = dpp_step_max<0xB1, 0xF>(v);     // quad_perm [1, 0, 3, 2]
    v = dpp_step_max<0x4E, 0xF>(v);     // quad_perm [2, 3, 0, 1]
    v = dpp_step_max<0x141, 0xF>(v);    // row_half_mirror
    v = dpp_step_max<0x140, 0xF>(v);    // row_mirror: every lane of a row holds its max
    v = dpp_step_max<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_step_max<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

// LU with partial pivoting of panel t (one workgroup per front): the pivot
// of column j is the largest |entry| among all rows of its pivot window at or
// below row j (rows [k0 + j, K1), K1 = piv_window_end), not only the rows of
// the 64 x 64 diagonal block, which keeps the element growth of the
// restricted pivoting small.  The candidate rows (at most PIV_WIN x FNB) are
// factored in LDS: the U rows of the panel, and the
// multipliers of every other candidate row, which are final L entries.  Plus
// U_tt^-1 for the L-column solves of the rows below K1 (stored once per front
// in uinv, FNB x FNB column major, identity beyond kb).  The multipliers of
// column j are used as D[i][j] / pivot_j in the updates and the column is
// scaled at the end (the scaling of a row commutes with the later
// interchanges).  Thread (column c = tid % 64, row group g = tid / 64) updates
// rows i = g (mod 4) of its column.  ipiv[first + k0 + j] = the candidate row
// (relative to k0, in [j, K1 - k0)) swapped with row j.
template <class T>
__global__ __launch_bounds__(256) void k_panel(T *arena, const FrontDesc *__restrict__ fd,
                                               int32_t *__restrict__ ipiv,
                                               int32_t *__restrict__ nperturbed, TaskList tl,
                                               int t, const double *__restrict__ thresh,
                                               double *__restrict__ uinv) {
    constexpr int H = FNB / 2;
    constexpr int LD = FNB + 1;
    // the candidate rows; after they are written back, the same space holds
    // U_tt^-1 (FNB x LD doubles) and a scratch block (H x (H + 1) doubles)
    constexpr size_t ROWS_B = (size_t)PIV_WIN * LD * sizeof(T);
    constexpr size_t INV_B = (size_t)FNB * LD * sizeof(T) + (FNB * LD + H * (H + 1)) * sizeof(double);
    __shared__ __align__(16) unsigned char smem[ROWS_B > INV_B ? ROWS_B : INV_B];
    __shared__ int piv[FNB];
    __shared__ T rpv[FNB];
    __shared__ double wmx[4];
    __shared__ int wrow[4];
    T (*D)[LD] = reinterpret_cast<T (*)[LD]>(smem);
    double (*Ui)[LD] = reinterpret_cast<double (*)[LD]>(smem + FNB * LD * sizeof(T));
    double (*Tm)[H + 1] = reinterpret_cast<double (*)[H + 1]>(smem + FNB * LD * sizeof(T) +
                                                              FNB * LD * sizeof(double));
    const int f = tl.fronts[blockIdx.x];
    const FrontDesc d = fd[f];
    const int k0 = t * FNB, kb = min(FNB, d.p - k0), m = d.m;
    const int R = piv_window_end(k0, d.p) - k0;       // candidate rows: kb <= R <= PIV_WIN
    T *F = arena + d.off;
    const int c = threadIdx.x % FNB, g = threadIdx.x / FNB, lane = threadIdx.x % 64;
    for (int i = g; i < R; i += 4)
        D[i][c] = (c < kb) ? F[(int64_t)(k0 + i) + (int64_t)(k0 + c) * m] : T(0);
    for (int i = R + g; i < FNB; i += 4) D[i][c] = T(0);
    __syncthreads();
    const T th = (T)thresh[d.seg];                   // the static-pivot threshold of its problem
    for (int j = 0; j < kb; j++) {
        // pivot: argmax over rows i in [j, R) of |D[i][j]|, the lowest row on
        // ties: per wave (64 rows) the DPP maximum and the lowest lane holding
        // it, then across the four waves in order
        {
            const int i = threadIdx.x;
            const double v = (i >= j && i < R) ? (double)fabs(D[i][j]) : -1.0;
            const double mx = __shfl(wave_max(v), 63);
            const uint64_t hit = __ballot(v == mx && v >= 0.0);
            if (lane == 0) {
                wmx[g] = hit ? mx : -1.0;
                wrow[g] = hit ? g * 64 + (__ffsll((unsigned long long)hit) - 1) : -1;
            }
        }
        __syncthreads();
        int r = j;
        {
            double best = -1.0;
            for (int w = 0; w < 4; w++)
                if (wrow[w] >= 0 && wmx[w] > best) { best = wmx[w]; r = wrow[w]; }
            r = (r >= j && r < R) ? r : j;
        }
        if (g == 0 && r != j && c < kb) {            // interchange rows j and r of column c
            T x = D[j][c];
            D[j][c] = D[r][c];
            D[r][c] = x;
        }
        if (threadIdx.x == 0) piv[j] = r;
        __syncthreads();
        T pv = D[j][j];
        const bool pert = fabs(pv) < th;
        if (pert) pv = (pv >= T(0)) ? th : -th;
        const T rp = T(1) / pv;
        if (c > j && c < kb) {                       // trailing update of column c
            const T ujc = D[j][c];
            // four rows at a time, all loads before the stores, so that the
            // LDS round trips of a thread overlap
            int i = j + 1 + g;
            for (; i + 12 < R; i += 16) {
                const T l0 = D[i][j], l1 = D[i + 4][j], l2 = D[i + 8][j], l3 = D[i + 12][j];
                const T a0 = D[i][c], a1 = D[i + 4][c], a2 = D[i + 8][c], a3 = D[i + 12][c];
                D[i][c] = a0 - (l0 * rp) * ujc;
                D[i + 4][c] = a1 - (l1 * rp) * ujc;
                D[i + 8][c] = a2 - (l2 * rp) * ujc;
                D[i + 12][c] = a3 - (l3 * rp) * ujc;
            }
            for (; i < R; i += 4) D[i][c] -= (D[i][j] * rp) * ujc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            D[j][j] = pv;
            rpv[j] = rp;
            if (pert) atomicAdd(nperturbed + d.seg, 1);   // per problem of a batch
        }
    }
    __syncthreads();
    if (c < kb)
        for (int i = c + 1 + g; i < R; i += 4) D[i][c] *= rpv[c];       // column c of L
    for (int i = g; i < FNB; i += 4)
        if (i >= kb && i == c) D[i][c] = T(1);                           // identity padding
    __syncthreads();
    if (c < kb)
        for (int i = g; i < R; i += 4) F[(int64_t)(k0 + i) + (int64_t)(k0 + c) * m] = D[i][c];
    if (g == 0 && c < kb) ipiv[d.first + k0 + c] = piv[c];
    __syncthreads();                                 // rows >= FNB of D are reused below
    // U^-1 by 32 x 32 blocks: the two diagonal inverses (one column per lane of
    // waves 0 and 1), then Ui12 = -Ui11 (U12 Ui22)
    if (g < 2 && c < H) {
        const int o = g * H;                         // block origin
        double x[H];
#pragma unroll
        for (int i = H - 1; i >= 0; i--) {
            double sum = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int q = i + 1; q < H; q++) sum -= (double)D[o + i][o + q] * x[q];
            x[i] = (i <= c) ? sum / (double)D[o + i][o + i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < H; i++) {
            Ui[o + i][o + c] = x[i];
            Ui[(1 - g) * H + i][o + c] = 0.0;        // the block below (g = 0) / left of U22 rows
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < H * H; e += 256) {             // Tm = U12 Ui22
        int i = e % H, jj = e / H;
        double acc = 0.0;
        for (int q = 0; q <= jj; q++) acc += (double)D[i][H + q] * Ui[H + q][H + jj];
        Tm[i][jj] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < H * H; e += 256) {             // Ui12 = -Ui11 Tm
        int i = e % H, jj = e / H;
        double acc = 0.0;
        for (int q = i; q < H; q++) acc += Ui[i][q] * Tm[q][jj];
        Ui[i][H + jj] = -acc;
    }
    __syncthreads();
    double *u = uinv + (int64_t)f * FNB * FNB;
    for (int e = threadIdx.x; e < FNB * FNB; e += 256) u[e] = Ui[e % FNB][e / FNB];
}

// Row interchanges of panel t applied to every column outside the panel (so
// that P A = L U holds with one row permutation per front), and the U rows of
// panel t: the permuted block rows right of the panel solved with the unit
// lower L_tt.  One thread per column.  The interchanges move rows inside the
// candidate window [k0, K1): position i of the window receives the row that
// was at src[i].  Every row moved below the panel (i >= kb) comes from one of
// the panel's own rows (src[i] < kb): a row leaves position j only through
// interchange j, and what position j holds then is one of the first kb rows.
// So a column's new panel rows are loaded first, then the moved rows below
// are written (their sources, panel rows, are still unwritten), then the
// panel rows.
template <class T>
__device__ __forceinline__ void trsm_u_item(T *arena, const FrontDesc *__restrict__ fd,
                                            const int32_t *__restrict__ ipiv, int2 tk, int t,
                                            T (*Ls)[FNB + 1], int *src, int *mrow, int *nmoved) {
    FrontDesc d = fd[tk.x];
    int chunk = tk.y;
    int k0 = t * FNB, kb = min(FNB, d.p - k0), k1 = k0 + kb, m = d.m;
    const int R = piv_window_end(k0, d.p) - k0;
    int nleft = (k0 + TRSM_U_COLS - 1) / TRSM_U_COLS;
    T *F = arena + d.off;
    for (int e = threadIdx.x; e < FNB * FNB; e += blockDim.x) {
        int i = e % FNB, j = e / FNB;
        Ls[i][j] = (i < kb && j < i) ? F[(int64_t)(k0 + i) + (int64_t)(k0 + j) * m] : T(0);
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < R; i++) src[i] = i;
        for (int j = 0; j < kb; j++) {
            int r = ipiv[d.first + k0 + j];
            r = (r >= j && r < R) ? r : j;
            int a = src[j]; src[j] = src[r]; src[r] = a;
        }
        int nm = 0;                                  // the rows moved below the panel
        for (int i = kb; i < R; i++)
            if (src[i] != i) mrow[nm++] = i;
        *nmoved = nm;
    }
    __syncthreads();
    int col, lim;
    bool solve = false;
    if (chunk < nleft) { col = chunk * TRSM_U_COLS; lim = k0; }
    else { col = k1 + (chunk - nleft) * TRSM_U_COLS; lim = m; solve = true; }
    col += threadIdx.x;
    if (col >= lim) return;
    T *Fc = F + (int64_t)col * m + k0;
    T x[FNB];
#pragma unroll
    for (int i = 0; i < FNB; i++) x[i] = (i < kb) ? Fc[src[i]] : T(0);
    // the rows moved below the panel, from panel rows not yet overwritten
    const int nm = *nmoved;
    for (int q0 = 0; q0 < nm; q0 += 8) {
        T y[8];
#pragma unroll
        for (int q = 0; q < 8; q++) y[q] = (q0 + q < nm) ? Fc[src[mrow[q0 + q]]] : T(0);
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (q0 + q < nm) Fc[mrow[q0 + q]] = y[q];
    }
    if (solve) {
#pragma unroll
        for (int i = 1; i < FNB; i++) {
            T s = x[i];
#pragma unroll
            for (int j = 0; j < i; j++) s -= Ls[i][j] * x[j];
            x[i] = s;
        }
    }
#pragma unroll
    for (int i = 0; i < FNB; i++)
        if (i < kb) Fc[i] = x[i];
}

// In-place inverses of the SB x SB diagonal blocks of L11 (unit lower) and
// U11 (upper) of every front, after its factorisation, so that each diagonal
// block of the triangular solves is a dense matrix-vector product instead of
// a sequential substitution; plus the composite row permutation of the block
// (prow: final position -> front-local row before the interchanges).
// Blocked by 32 x 32 sub-blocks:  Linv_ij = -Linv_ii sum_{k=j..i-1} L_ik Linv_kj
// (i > j, by ascending j), Uinv_ij = -Uinv_ii sum_{k=i+1..j} U_ik Uinv_kj
// (i < j, by descending j).  Arithmetic in FP64 whatever T is.
constexpr int ISB = 32;

template <class T>
__global__ __launch_bounds__(256) void k_invert_diag(T *arena, const FrontDesc *__restrict__ fd,
                                                     const int32_t *__restrict__ ipiv,
                                                     int32_t *__restrict__ prow, TaskList tl,
                                                     int mode, int fixed_blk) {
    __shared__ double tmp[ISB][ISB + 1];
    const int2 tk = tl.items[blockIdx.x];
    FrontDesc d = fd[tk.x];
    int blk = fixed_blk >= 0 ? fixed_blk : tk.y;
    const bool doL = mode & 1, doU = mode & 2;
    int b0 = blk * SB, sz = min(SB, d.p - b0), m = d.m;
    T *F = arena + d.off + (int64_t)b0 * m + b0;     // block origin, leading dimension m
    int nsb = (sz + ISB - 1) / ISB;
    int tid = threadIdx.x;
    // composite row permutation of the panels inside this block (their
    // interchanges stay inside the block's rows)
    __shared__ int src[SB];
    if (doU && tid == 0) {
        for (int i = 0; i < sz; i++) src[i] = i;
        for (int q0 = 0; q0 < sz; q0 += FNB) {
            const int kb = min(FNB, sz - q0);
            for (int j = 0; j < kb; j++) {
                int r = ipiv[d.first + b0 + q0 + j];
                r = (r >= j && q0 + r < sz) ? r : j;
                int a = src[q0 + j]; src[q0 + j] = src[q0 + r]; src[q0 + r] = a;
            }
        }
        for (int i = 0; i < sz; i++) prow[d.first + b0 + i] = b0 + src[i];
    }
    auto at = [&](int r, int c) -> T & { return F[(int64_t)r + (int64_t)c * m]; };
    // phase 1: diagonal 32 x 32 sub-blocks (thread = sub-block i, column j)
    {
        int i = tid / ISB, j = tid % ISB;
        int r0 = i * ISB, ns = min(ISB, sz - r0);
        double xl[ISB], xu[ISB];
        bool act = i < nsb && j < ns;
        // every read below stays inside the ns x ns sub-block (rows, columns < ns)
#pragma unroll
        for (int r = 0; r < ISB; r++) {              // L: unit lower, column j
            double v = (r == j) ? 1.0 : 0.0;
            if (act && r < ns && r > j) {
#pragma unroll
                for (int q = 0; q < r; q++) v -= (double)at(r0 + r, r0 + q) * xl[q];
            }
            xl[r] = (act && r >= j && r < ns) ? v : 0.0;
        }
#pragma unroll
        for (int r = ISB - 1; r >= 0; r--) {         // U: upper, column j
            double v = 0.0;
            if (act && r <= j) {
                v = (r == j) ? 1.0 : 0.0;
#pragma unroll
                for (int q = r + 1; q < ISB; q++)
                    if (q < ns) v -= (double)at(r0 + r, r0 + q) * xu[q];
                v /= (double)at(r0 + r, r0 + r);
            }
            xu[r] = v;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ISB; r++)
            if (act && r < ns && (r > j ? doL : doU)) at(r0 + r, r0 + j) = (T)(r > j ? xl[r] : xu[r]);
        __syncthreads();
    }
    int tc = tid % ISB, tr = tid / ISB;              // tile coordinates: 8 row groups
    // phase 2: L off-diagonal sub-blocks
    for (int i = 1; doL && i < nsb; i++) {
        int ri = i * ISB, ni = min(ISB, sz - ri);
        for (int j = 0; j < i; j++) {
            int cj = j * ISB;
            // tmp = sum_{k=j}^{i-1} L_ik Linv_kj   (Linv_jj unit lower)
            for (int q = 0; q < 4; q++) {
                int r = tr + 8 * q;
                double acc = 0.0;
                if (r < ni) {
                    for (int kk = j; kk < i; kk++) {
                        int ck = kk * ISB;
                        for (int c2 = 0; c2 < ISB; c2++) {
                            int row_k = ck + c2;           // row inside block kk
                            double lin;                    // Linv_{kk,j}(c2, tc)
                            if (kk == j) lin = (c2 == tc) ? 1.0 : (c2 > tc ? (double)at(row_k, cj + tc) : 0.0);
                            else lin = (double)at(row_k, cj + tc);
                            acc += (double)at(ri + r, ck + c2) * lin;
                        }
                    }
                }
                tmp[r][tc] = acc;
            }
            __syncthreads();
            // Linv_ij = -Linv_ii tmp
            double out[4];
            for (int q = 0; q < 4; q++) {
                int r = tr + 8 * q;
                double acc = 0.0;
                if (r < ni) {
                    acc = tmp[r][tc];
                    for (int c2 = 0; c2 < r; c2++) acc += (double)at(ri + r, ri + c2) * tmp[c2][tc];
                }
                out[q] = -acc;
            }
            __syncthreads();
            for (int q = 0; q < 4; q++) {
                int r = tr + 8 * q;
                if (r < ni) at(ri + r, cj + tc) = (T)out[q];
            }
            __syncthreads();
        }
    }
    // phase 3: U off-diagonal sub-blocks
    for (int i = nsb - 2; doU && i >= 0; i--) {
        int ri = i * ISB;
        for (int j = nsb - 1; j > i; j--) {
            int cj = j * ISB, nj = min(ISB, sz - cj);
            // tmp = sum_{k=i+1}^{j} U_ik Uinv_kj
            for (int q = 0; q < 4; q++) {
                int r = tr + 8 * q;
                double acc = 0.0;
                if (tc < nj) {
                    for (int kk = i + 1; kk <= j; kk++) {
                        int ck = kk * ISB, nk = min(ISB, sz - ck);
                        for (int c2 = 0; c2 < nk; c2++) {
                            double uin;                    // Uinv_{kk,j}(c2, tc)
                            if (kk == j) uin = (c2 <= tc) ? (double)at(ck + c2, cj + tc) : 0.0;
                            else uin = (double)at(ck + c2, cj + tc);
                            acc += (double)at(ri + r, ck + c2) * uin;
                        }
                    }
                }
                tmp[r][tc] = acc;
            }
            __syncthreads();
            double out[4];
            for (int q = 0; q < 4; q++) {
                int r = tr + 8 * q;
                double acc = 0.0;
                if (tc < nj)
                    for (int c2 = r; c2 < ISB; c2++) acc += (double)at(ri + r, ri + c2) * tmp[c2][tc];
                out[q] = -acc;
            }
            __syncthreads();
            for (int q = 0; q < 4; q++) {
                int r = tr + 8 * q;
                if (tc < nj) at(ri + r, cj + tc) = (T)out[q];
            }
            __syncthreads();
        }
    }
}

// L21 of panel t: every row below the panel times U_tt^-1 (computed once per
// front by k_panel); each workgroup multiplies its 64 rows by the inverse.
// As[k][i]: row i of the chunk, panel column k.
template <class T>
__device__ __forceinline__ void trsm_l_item(T *arena, const FrontDesc *__restrict__ fd, int2 tk,
                                            int t, const double *__restrict__ uinv,
                                            double (*Ui)[FNB + 1], double (*As)[FNB + 1]) {
    FrontDesc d = fd[tk.x];
    int chunk = tk.y;
    int k0 = t * FNB, kb = min(FNB, d.p - k0), m = d.m;
    // the rows of the candidate window got their multipliers in k_panel
    const int K1 = piv_window_end(k0, d.p);
    int r0 = K1 + chunk * TRSM_L_ROWS, nr = min(TRSM_L_ROWS, m - r0);
    T *F = arena + d.off;
    const double *u = uinv + (int64_t)tk.x * FNB * FNB;
    for (int e = threadIdx.x; e < FNB * FNB; e += blockDim.x) {
        int i = e % FNB, j = e / FNB;
        Ui[i][j] = u[e];
        As[j][i] = (i < nr && j < kb) ? (double)F[(int64_t)(r0 + i) + (int64_t)(k0 + j) * m] : 0.0;
    }
    __syncthreads();
    int i = threadIdx.x % TRSM_L_ROWS, jb = (threadIdx.x / TRSM_L_ROWS) * 16;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; q++) acc[q] = 0.0;
    for (int kk = 0; kk < kb; kk++) {
        double a = As[kk][i];
#pragma unroll
        for (int q = 0; q < 16; q++) acc[q] += a * Ui[kk][jb + q];
    }
    if (i < nr)
#pragma unroll
        for (int q = 0; q < 16; q++)
            if (jb + q < kb) F[(int64_t)(r0 + i) + (int64_t)(k0 + jb + q) * m] = (T)acc[q];
}

// The U-row and L-column solves of panel t in one launch (they are
// independent once the panel is factored): the first tu.total workgroups take
// U-row items, the rest L-column items.
template <class T>
__global__ __launch_bounds__(256) void k_trsm(T *arena, const FrontDesc *__restrict__ fd,
                                              const int32_t *__restrict__ ipiv, TaskList tu,
                                              TaskList tlo, int t,
                                              const double *__restrict__ uinv) {
    static_assert(TRSM_U_COLS == 256 && TRSM_L_ROWS == 64, "one thread per column / row quarter");
    __shared__ double smem[2][FNB][FNB + 1];
    __shared__ int src[SB], mrow[SB], nmoved;
    if ((int64_t)blockIdx.x < tu.total)
        trsm_u_item<T>(arena, fd, ipiv, tu.items[blockIdx.x], t,
                       reinterpret_cast<T (*)[FNB + 1]>(&smem[0][0][0]), src, mrow, &nmoved);
    else
        trsm_l_item<T>(arena, fd, tlo.items[blockIdx.x - tu.total], t, uinv, smem[0], smem[1]);
}

// trailing update F[k1:m, k1:m] -= F[k1:m, k0:k1] F[k0:k1, k1:m] on the matrix
// cores: 128 x 128 output tile per workgroup of eight waves, each wave a
// 64 x 32 strip as 4 x 2 MFMA 16x16x4 blocks (FP64 or FP32 by T), the A and B
// panels staged in LDS k-major.  Eight waves with 64 accumulators each leave
// four waves per SIMD (two workgroups per CU): one wave issues the FP64
// instruction at most every other slot of its SIMD's matrix core, so the
// core stays busy while any two of the four have operands ready, which two
// waves of 128 accumulators (a 64 x 64 quarter each) could not ensure.
template <class T> struct MfmaAcc;
// Operand layout of both 16x16x4 instructions: lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Result element v of lane l is row_of(l/16, v), column l%16
// (checked on gfx950: FP32 packs four consecutive rows per lane group, FP64
// strides them by four).
template <> struct MfmaAcc<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row_of(int lk, int v) { return lk + 4 * v; }
};
template <> struct MfmaAcc<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row_of(int lk, int v) { return 4 * lk + v; }
};

constexpr int ST = SCHUR_TILE;       // 128
// K columns staged per pass (FP64 half as many, to keep the prefetch, the two
// operand sets and the 32 accumulator elements of a lane inside the register
// budget of four waves per SIMD)
template <class T> struct SchurCfg {
    static constexpr int KC = sizeof(T) == 8 ? 16 : 32;
    static constexpr int PF = ST * KC / SCHUR_THREADS;   // elements of A (and of B) per thread
    // LDS layouts (64 banks of 4 bytes).  A as [k][row], rows padded to 144
    // elements, so the four k-rows one operand read touches sit half the banks
    // apart (FP64) or a quarter apart (FP32).  B as [column][k], as it lies in
    // the front: FP64 unpadded, the 16-byte k-pairs of column c stored at pair
    // slot (k / 2) xor ((c / 2) mod 8), so the 16 columns one operand read
    // touches fall on distinct banks and each 1 KB run of 8 columns can be
    // filled by one direct global-to-LDS load per wave; FP32 with an odd row
    // length (33) for the same effect.
    static constexpr bool SWZ = sizeof(T) == 8;
    static constexpr int SPA = ST + 16;
    static constexpr int SPB = SWZ ? KC : KC + 1;
    static constexpr int ABUF = KC * SPA, BBUF = ST * SPB;
    static __device__ __forceinline__ int bpos(int c, int k) {
        return SWZ ? c * SPB + ((((k >> 1) ^ ((c >> 1) & 7))) << 1) + (k & 1) : c * SPB + k;
    }
};

static_assert(SCHUR_THREADS == 512 && ST == 128,
              "eight waves, as two rows of 64 and four columns of 32, cover the 128 x 128 tile");
static_assert((ST * SchurCfg<double>::KC) % SCHUR_THREADS == 0 &&
                  (ST * SchurCfg<float>::KC) % SCHUR_THREADS == 0 && SchurCfg<double>::KC % 8 == 0,
              "a K chunk splits evenly over the threads, and its k-rows over the eight waves");

// BIG = 0: update after panel t inside its outer SB block, K = the panel's kb
//          columns: the first tiles cover the rows below the panel and the
//          columns up to the end of the outer block, the rest the remaining
//          rows of the outer block and every column right of it;
// BIG = 1: trailing update (everything right of and below, including the
//          contribution block) after outer block t: for even t, K = block t's
//          (up to SB) columns; for odd t, K = blocks t - 1 and t together;
// BIG = 5: after even outer block t whose successor exists, K = block t's SB
//          columns applied only to the strips block t + 1 = [K1, K2) reads:
//          rows [K1, m) x columns [K1, K2), then rows [K1, K2) x columns [K2, m);
// BIG = 2, 3: merge of the inverted, folded blocks b1 = [a, a + SB) and
//          b2 = [a + SB, e) (a = t SSB) into one solve block: with the folded
//          panels L~ = L Linv and U~ = U Uinv, the rows below e need
//          L~[., b1] -= L~[., b2] L~[b2, b1]   (BIG = 2: K = b2),
//          the rows above a need U~[., b2] -= U~[., b1] U~[b1, b2]  (BIG = 3: K = b1).
// The next K chunk is fetched from HBM into registers while the current one
// feeds the matrix cores from LDS.
template <class T, int BIG>
__global__ __launch_bounds__(SCHUR_THREADS, 4) void k_schur(T *arena, const FrontDesc *__restrict__ fd,
                                                  TaskList tl, int t) {
    typedef typename MfmaAcc<T>::v4 v4;
    constexpr int KC = SchurCfg<T>::KC, PF = SchurCfg<T>::PF;
    constexpr int SPA = SchurCfg<T>::SPA, SPB = SchurCfg<T>::SPB;
    constexpr int STAGE = SchurCfg<T>::ABUF + SchurCfg<T>::BBUF;
    // two LDS stages of the A and B chunks: the next chunk is stashed into the
    // idle one while the current one is consumed (one barrier per chunk)
    __shared__ T smem[2 * STAGE];
    const int2 tk = tl.items[blockIdx.x];
    FrontDesc d = fd[tk.x];
    int64_t tile = tk.y;
    int m = d.m, kc0, kd, rlo, rhi, clo, chi;
    if (!BIG) {
        kc0 = t * FNB; kd = min(FNB, d.p - kc0);
        int k1 = kc0 + kd, K1 = min(d.p, (kc0 / SB + 1) * SB);
        int n0 = (K1 > k1) ? ((m - k1 + ST - 1) / ST) * ((K1 - k1 + ST - 1) / ST) : 0;
        if (tile < n0) { rlo = k1; rhi = m; clo = k1; chi = K1; }
        else { tile -= n0; rlo = k1; rhi = K1; clo = K1; chi = m; }
    } else if (BIG == 1) {
        kc0 = (t & 1) ? (t - 1) * SB : t * SB;
        kd = min((t & 1) ? 2 * SB : SB, d.p - kc0);
        rlo = kc0 + kd; rhi = m; clo = rlo; chi = m;
    } else if (BIG == 5) {
        kc0 = t * SB; kd = SB;
        const int K1 = kc0 + SB, K2 = min(d.p, K1 + SB);
        const int64_t n1 = (int64_t)((m - K1 + ST - 1) / ST) * ((K2 - K1 + ST - 1) / ST);
        if (tile < n1) { rlo = K1; rhi = m; clo = K1; chi = K2; }
        else { tile -= n1; rlo = K1; rhi = K2; clo = K2; chi = m; }
    } else {
        int a = t * SSB, e = min(d.p, a + SSB);
        if (BIG == 2) { kc0 = a + SB; kd = e - kc0; rlo = e; rhi = m; clo = a; chi = a + SB; }
        else { kc0 = a; kd = SB; rlo = 0; rhi = a; clo = a + SB; chi = e; }
    }
    int ntr = (rhi - rlo + ST - 1) / ST;
    int ti = (int)(tile % ntr), tj = (int)(tile / ntr);
    int r0 = rlo + ti * ST, c0 = clo + tj * ST;
    T *F = arena + d.off;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int wr = (w & 1) * 64, wc = (w >> 1) * 32;
    int li = lane & 15, lk = lane >> 4;
    // global -> register prefetch of one K chunk: A rows i = e % ST (coalesced
    // down the column), B k = e % KC (contiguous k of one column).  Each load
    // is a per-chunk uniform base plus one 32-bit per-lane offset.
    const int tid = threadIdx.x;
    const uint32_t aoff = (uint32_t)((tid % ST) + (tid / ST) * m) * (uint32_t)sizeof(T);
    const uint32_t boff = (uint32_t)((tid % KC) + (tid / KC) * m) * (uint32_t)sizeof(T);
    const bool rok = r0 + tid % ST < rhi;
    T pa[PF], pb[PF];
    auto fetch = [&](int kc) {
        const int kn = min(KC, kd - kc);
        const char *Ab = reinterpret_cast<const char *>(F + r0 + (int64_t)(kc0 + kc) * m);
        const char *Bb = reinterpret_cast<const char *>(F + (kc0 + kc) + (int64_t)c0 * m);
#pragma unroll
        for (int q = 0; q < PF; q++) {
            const int kk = tid / ST + q * (SCHUR_THREADS / ST), j = tid / KC + q * (SCHUR_THREADS / KC);
            pa[q] = (rok && kk < kn)
                        ? *reinterpret_cast<const T *>(Ab + (int64_t)q * (SCHUR_THREADS / ST) * m * sizeof(T) + aoff)
                        : T(0);
            pb[q] = (c0 + j < chi && tid % KC < kn)
                        ? *reinterpret_cast<const T *>(Bb + (int64_t)q * (SCHUR_THREADS / KC) * m * sizeof(T) + boff)
                        : T(0);
        }
    };
    auto stash = [&](int buf) {
        T *As = smem + buf * STAGE, *Bs = As + SchurCfg<T>::ABUF;
#pragma unroll
        for (int q = 0; q < PF; q++) {
            int e = tid + q * SCHUR_THREADS;
            As[(e / ST) * SPA + (e % ST)] = pa[q];
            Bs[SchurCfg<T>::bpos(e / KC, e % KC)] = pb[q];
        }
    };
    // Interior FP64 tiles fill full chunks with direct global-to-LDS loads
    // (16 bytes per lane, lane l at byte 16 l of the wave's 1 KB run): A one
    // k-row of 128 rows per instruction, B 8 columns per instruction with the
    // k-pair slots swizzled as above.  No registers and no stash.
    auto issue = [&](int kc, int buf) {
        T *As = smem + buf * STAGE, *Bs = As + SchurCfg<T>::ABUF;
#pragma unroll
        for (int i = 0; i < KC / 8; i++) {
            const int k = w + 8 * i;
            const T *src = F + r0 + 2 * lane + (int64_t)(kc0 + kc + k) * m;
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (__attribute__((address_space(3))) void *)(As + k * SPA),
                                             16, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < ST / 64; i++) {
            const int ib = w + 8 * i, c = ib * 8 + (lane >> 3), slot = lane & 7;
            const int kp = slot ^ ((c >> 1) & 7);
            const T *src = F + (kc0 + kc + 2 * kp) + (int64_t)(c0 + c) * m;
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (__attribute__((address_space(3))) void *)(Bs + ib * 8 * SPB),
                                             16, 0, 0);
        }
    };
    // operands of one 4-deep k-step: A rows wr + 16 a + li (negated: the tile
    // computes C - A B), B columns wc + 16 b + li, k = 4 ks + lk
    auto operands = [&](int buf, int ks, T (&av)[4], T (&bv)[2]) {
        const T *As = smem + buf * STAGE, *Bs = As + SchurCfg<T>::ABUF;
        const int kk = ks * 4 + lk;
#pragma unroll
        for (int a = 0; a < 4; a++) av[a] = -As[kk * SPA + wr + a * 16 + li];
#pragma unroll
        for (int b = 0; b < 2; b++) bv[b] = Bs[SchurCfg<T>::bpos(wc + b * 16 + li, kk)];
    };
    // The accumulators start from the C tile itself and A enters negated, so
    // the matrix cores leave C - A B in registers: the tile is read once at
    // the start (while the first chunk is in flight) and only written at the
    // end.  Lane (li, lk) holds rows wr + 16 a + row_of(lk, v) and columns
    // wc + 16 b + li.
    v4 acc[4][2];
    auto load_c = [&]() {
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int c = c0 + wc + b * 16 + li;
            const T *Fc = F + (int64_t)min(c, chi - 1) * m;
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int r = r0 + wr + a * 16 + MfmaAcc<T>::row_of(lk, v);
                    acc[a][b][v] = (r < rhi && c < chi) ? Fc[r] : T(0);
                }
        }
    };
    auto mma = [&](const T (&av)[4], const T (&bv)[2]) {
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) acc[a][b] = MfmaAcc<T>::mma(av[a], bv[b], acc[a][b]);
    };
    // all KC / 4 k-steps of the chunk in `buf` (a partial chunk's missing k are
    // zeros), the operands of k-step ks + 1 read while k-step ks runs
    auto steps = [&](int buf) {
        T av0[4], bv0[2], av1[4], bv1[2];
        operands(buf, 0, av0, bv0);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ks += 2) {
            operands(buf, ks + 1, av1, bv1);
            mma(av0, bv0);
            if (ks + 2 < KC / 4) operands(buf, ks + 2, av0, bv0);
            mma(av1, bv1);
        }
    };
    const bool dma = SchurCfg<T>::SWZ && r0 + ST <= rhi && c0 + ST <= chi;
    if (dma) {
        const int nfull = kd / KC;
        if (nfull > 0) issue(0, 0);
        load_c();
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int c = 0; c < nfull; c++) {
            if (c + 1 < nfull) issue((c + 1) * KC, (c + 1) & 1);
            steps(c & 1);
            __builtin_amdgcn_s_waitcnt(0);       // the next chunk's direct loads
            __syncthreads();
        }
        if (nfull * KC < kd) {                   // partial last chunk: masked loads
            fetch(nfull * KC);
            stash(nfull & 1);
            __syncthreads();
            steps(nfull & 1);
        }
    } else {
        fetch(0);
        load_c();
        stash(0);
        __syncthreads();
        if (KC < kd) fetch(KC);
        // Per chunk: the first operands are read, then the next chunk (in
        // flight since the previous one) is stashed into the idle stage and
        // the one after it fetched, while the reads land.
        for (int kc = 0, buf = 0; kc < kd; kc += KC, buf ^= 1) {
            T av0[4], bv0[2], av1[4], bv1[2];
            operands(buf, 0, av0, bv0);
            if (kc + KC < kd) {
                stash(buf ^ 1);
                if (kc + 2 * KC < kd) fetch(kc + 2 * KC);
            }
#pragma unroll
            for (int ks = 0; ks < KC / 4; ks += 2) {
                operands(buf, ks + 1, av1, bv1);
                mma(av0, bv0);
                if (ks + 2 < KC / 4) operands(buf, ks + 2, av0, bv0);
                mma(av1, bv1);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const int c = c0 + wc + b * 16 + li;
        if (c >= chi) continue;
        T *Fc = F + (int64_t)c * m;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = r0 + wr + a * 16 + MfmaAcc<T>::row_of(lk, v);
                if (r < rhi) Fc[r] = acc[a][b][v];
            }
    }
}

// Completes the inverse of every merged solve block [a, e) (a = t SSB) once
// the two products of k_schur<., 2 / 3> have run:
//   lower: Linv = [[I1, 0], [X, I2]],  X = -I2 L~[b2, b1]   (I2 unit lower)
//   upper: Uinv = [[J1, Y], [0, J2]],  Y = -J1 U~[b1, b2]   (J1 upper)
// computed in place over the folded blocks L~[b2, b1] and U~[b1, b2].  Work
// item: 16 columns of one side of one pair (per pair the lower-side chunks
// first, then the upper-side ones); the columns are staged in LDS, then
// thread i forms row i from row i of the triangular factor.
constexpr int MT_COLS = 16;

template <class T>
__global__ __launch_bounds__(256) void k_merge_tri(T *arena, const FrontDesc *__restrict__ fd,
                                                  TaskList tl) {
    __shared__ double vs[MT_COLS][SB + 1];
    const int2 tk = tl.items[blockIdx.x];
    const FrontDesc d = fd[tk.x];
    const int m = d.m;
    int w = tk.y, a = 0, n2 = 0;
    for (a = 0; a + SB < d.p; a += SSB) {            // locate the pair and side
        n2 = min(d.p, a + SSB) - a - SB;
        int nl = SB / MT_COLS, nu = (n2 + MT_COLS - 1) / MT_COLS;
        if (w < nl + nu) break;
        w -= nl + nu;
    }
    if (a + SB >= d.p) return;                       // not reached for valid items
    const int b2 = a + SB;
    T *F = arena + d.off;
    const int i = threadIdx.x;
    if (w < SB / MT_COLS) {
        // lower side: X[:, j] = -(v + sum_{k<i} I2[i][k] v[k]), v = L~[b2 + ., a + j]
        const int j0 = w * MT_COLS;
        for (int e = threadIdx.x; e < MT_COLS * SB; e += 256) {
            int c = e / SB, r = e % SB;
            vs[c][r] = r < n2 ? (double)F[(b2 + r) + (int64_t)(a + j0 + c) * m] : 0.0;
        }
        __syncthreads();
        if (i < n2) {
            double acc[MT_COLS];
#pragma unroll
            for (int c = 0; c < MT_COLS; c++) acc[c] = vs[c][i];
            for (int k = 0; k < i; k++) {
                double coef = (double)F[(b2 + i) + (int64_t)(b2 + k) * m];
#pragma unroll
                for (int c = 0; c < MT_COLS; c++) acc[c] += coef * vs[c][k];
            }
#pragma unroll
            for (int c = 0; c < MT_COLS; c++) F[(b2 + i) + (int64_t)(a + j0 + c) * m] = (T)(-acc[c]);
        }
    } else {
        // upper side: Y[:, j] = -sum_{k>=i} J1[i][k] v[k], v = U~[a + ., b2 + j]
        const int j0 = (w - SB / MT_COLS) * MT_COLS, nc = min(MT_COLS, n2 - j0);
        for (int e = threadIdx.x; e < MT_COLS * SB; e += 256) {
            int c = e / SB, r = e % SB;
            vs[c][r] = c < nc ? (double)F[(a + r) + (int64_t)(b2 + j0 + c) * m] : 0.0;
        }
        __syncthreads();
        double acc[MT_COLS];
#pragma unroll
        for (int c = 0; c < MT_COLS; c++) acc[c] = 0.0;
        for (int k = i; k < SB; k++) {
            double coef = (double)F[(a + i) + (int64_t)(a + k) * m];
#pragma unroll
            for (int c = 0; c < MT_COLS; c++) acc[c] += coef * vs[c][k];
        }
#pragma unroll
        for (int c = 0; c < MT_COLS; c++)
            if (c < nc) F[(a + i) + (int64_t)(b2 + j0 + c) * m] = (T)(-acc[c]);
    }
}

// Once per factorisation, after the diagonal blocks are inverted: fold each
// inverse into the off-diagonal panel of its block column,
//   L~[rows below block t, t] = L[., t] Linv_tt,   U~[rows above, t] = U[., t] Uinv_tt,
// so that a solve step needs only v_t (not Xinv_tt v_t) to update the other
// rows, and the diagonal product runs in the same launch.  Work item: XR = 64
// rows of one panel times the (unit lower or upper) inverse, on the matrix
// cores: wave w owns output columns 64 w .. 64 w + 63 (4 x 4 MFMA 16x16x4
// blocks), K in chunks of XK through LDS.  In place is safe: a workgroup
// reads all of its rows before it writes any, and no other workgroup touches
// them.
constexpr int XR = 64, XK = 8, XAP = XR + 16, XBP = SB + 16;

template <class T>
__global__ __launch_bounds__(256) void k_xform(T *arena, const FrontDesc *__restrict__ fd,
                                              TaskList tl) {
    typedef typename MfmaAcc<T>::v4 v4;
    __shared__ T As[2][XK][XAP];     // A chunk: k-row, panel row
    __shared__ T Bs[2][XK][XBP];     // inverse chunk: k-row, column
    const int2 tk = tl.items[blockIdx.x];
    FrontDesc d = fd[tk.x];
    int64_t w = tk.y;
    int m = d.m, nb = (d.p + SB - 1) / SB;
    // locate (block t, side, chunk): per block first the L chunks, then the U chunks
    int t = 0, side = 0, chunk = 0;
    for (t = 0; t < nb; t++) {
        int t0 = t * SB, tend = min(d.p, t0 + SB);
        int nl = (m - tend + XR - 1) / XR, nu = (t0 + XR - 1) / XR;
        if (w < nl) { side = 0; chunk = (int)w; break; }
        w -= nl;
        if (w < nu) { side = 1; chunk = (int)w; break; }
        w -= nu;
    }
    const int t0 = t * SB, st = min(SB, d.p - t0), tend = t0 + st;
    const int r0 = side == 0 ? tend + chunk * XR : chunk * XR;
    const int rlim = side == 0 ? m : t0;
    const int nr = min(XR, rlim - r0);
    T *F = arena + d.off;
    const T *X = F + t0 + (int64_t)t0 * m;          // the inverted diagonal block
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int li = lane & 15, lk = lane >> 4, wc = wv * 64;
    // staging of one K chunk: A 64 x XK (2 per thread), X XK x 256 (8 per thread)
    T pa[XR * XK / 256], pb[XK * SB / 256];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int q = 0; q < XR * XK / 256; q++) {
            const int e = tid + q * 256, i = e % XR, k = e / XR, kk = kc + k;
            pa[q] = (i < nr && kk < st) ? F[(r0 + i) + (int64_t)(t0 + kk) * m] : T(0);
        }
#pragma unroll
        for (int q = 0; q < XK * SB / 256; q++) {
            const int e = tid + q * 256, k = e % XK, jj = e / XK, kr = kc + k;
            T x = T(0);
            if (kr < st && jj < st) {
                if (side == 0) x = (kr > jj) ? X[kr + (int64_t)jj * m] : (kr == jj ? T(1) : T(0));
                else x = (kr <= jj) ? X[kr + (int64_t)jj * m] : T(0);
            }
            pb[q] = x;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < XR * XK / 256; q++) {
            const int e = tid + q * 256;
            As[buf][e / XR][e % XR] = pa[q];
        }
#pragma unroll
        for (int q = 0; q < XK * SB / 256; q++) {
            const int e = tid + q * 256;
            Bs[buf][e % XK][e / XK] = pb[q];
        }
    };
    v4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = v4{0, 0, 0, 0};
    fetch(0);
    stash(0);
    __syncthreads();
    for (int kc = 0, buf = 0; kc < st; kc += XK, buf ^= 1) {
        if (kc + XK < st) fetch(kc + XK);
#pragma unroll
        for (int ks = 0; ks < XK / 4; ks++) {
            const int kk = ks * 4 + lk;
            T av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; a++) av[a] = As[buf][kk][a * 16 + li];
#pragma unroll
            for (int b = 0; b < 4; b++) bv[b] = Bs[buf][kk][wc + b * 16 + li];
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) acc[a][b] = MfmaAcc<T>::mma(av[a], bv[b], acc[a][b]);
        }
        if (kc + XK < st) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 4; b++) {
        const int c = wc + b * 16 + li;
        if (c >= st) continue;
        T *Fc = F + (int64_t)(t0 + c) * m + r0;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = a * 16 + MfmaAcc<T>::row_of(lk, v);
                if (r < nr) Fc[r] = acc[a][b][v];
            }
    }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

int64_t xform_items(int m, int p) {
    int64_t n = 0;
    for (int t0 = 0; t0 < p; t0 += SB) {
        int tend = std::min(p, t0 + SB);
        n += (m - tend + XR - 1) / XR + (t0 + XR - 1) / XR;
    }
    return n;
}

int64_t schur_tiles(int64_t rest) {
    int64_t nt = (rest + SCHUR_TILE - 1) / SCHUR_TILE;
    return nt * nt;
}

template <class T>
void launch_front_pull(T *arena, const FrontDesc *fd, const int32_t *pullmap,
                       const int32_t *child_ids, TaskList tl, hipStream_t s) {
    if (tl.total == 0) return;
    hipLaunchKernelGGL(k_front_pull<T>, dim3((unsigned)tl.total), dim3(256), 0, s, arena, fd,
                       pullmap, child_ids, tl);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_front_assemble(T *arena, const FrontDesc *fd, int64_t count, const int32_t *efront,
                           const int32_t *epos, const int32_t *esrc, const double *diag,
                           double sigma, double offv, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_front_assemble<T>, dim3(cdiv(count, 256)), dim3(256), 0, s, arena, fd,
                       count, efront, epos, esrc, diag, sigma, offv);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_panel(T *arena, const FrontDesc *fd, int32_t *ipiv, int32_t *nperturbed, TaskList tl,
                  int t, const double *thresh, double *uinv, hipStream_t s) {
    if (tl.n == 0) return;
    k_panel<T><<<dim3(tl.n), dim3(256), 0, s>>>(arena, fd, ipiv, nperturbed, tl, t, thresh, uinv);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_trsm(T *arena, const FrontDesc *fd, const int32_t *ipiv, TaskList tu, TaskList tlo,
                 int t, const double *uinv, hipStream_t s) {
    const int64_t n = tu.total + tlo.total;
    if (n == 0) return;
    k_trsm<T><<<dim3((unsigned)n), dim3(256), 0, s>>>(arena, fd, ipiv, tu, tlo, t, uinv);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_invert_diag(T *arena, const FrontDesc *fd, const int32_t *ipiv, int32_t *prow,
                        TaskList tl, int mode, int fixed_blk, hipStream_t s) {
    if (tl.total == 0) return;
    hipLaunchKernelGGL(k_invert_diag<T>, dim3((unsigned)tl.total), dim3(256), 0, s, arena, fd, ipiv,
                       prow, tl, mode, fixed_blk);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_xform(T *arena, const FrontDesc *fd, TaskList tl, hipStream_t s) {
    if (tl.total == 0) return;
    hipLaunchKernelGGL(k_xform<T>, dim3((unsigned)tl.total), dim3(256), 0, s, arena, fd, tl);
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_schur(T *arena, const FrontDesc *fd, TaskList tl, int t, int kind, hipStream_t s) {
    if (tl.total == 0) return;
    const dim3 g((unsigned)tl.total), b(SCHUR_THREADS);
    switch (kind) {
        case 0: k_schur<T, 0><<<g, b, 0, s>>>(arena, fd, tl, t); break;
        case 1: k_schur<T, 1><<<g, b, 0, s>>>(arena, fd, tl, t); break;
        case 2: k_schur<T, 2><<<g, b, 0, s>>>(arena, fd, tl, t); break;
        case 3: k_schur<T, 3><<<g, b, 0, s>>>(arena, fd, tl, t); break;
        default: k_schur<T, 5><<<g, b, 0, s>>>(arena, fd, tl, t); break;
    }
    MBL_CHECK_LAUNCH();
}

template <class T>
void launch_merge_tri(T *arena, const FrontDesc *fd, TaskList tl, hipStream_t s) {
    if (tl.total == 0) return;
    k_merge_tri<T><<<dim3((unsigned)tl.total), dim3(256), 0, s>>>(arena, fd, tl);
    MBL_CHECK_LAUNCH();
}

int merge_tri_items(int p) {
    int n = 0;
    for (int a = 0; a + SB < p; a += SSB) {
        int n2 = std::min(p, a + SSB) - a - SB;
        n += SB / MT_COLS + (n2 + MT_COLS - 1) / MT_COLS;
    }
    return n;
}


#define MBL_INST_FRONT(T)                                                                       \
    template void launch_front_pull<T>(T *, const FrontDesc *, const int32_t *, const int32_t *, \
                                       TaskList, hipStream_t);                                  \
    template void launch_front_assemble<T>(T *, const FrontDesc *, int64_t, const int32_t *,    \
                                           const int32_t *, const int32_t *, const double *,    \
                                           double, double, hipStream_t);                        \
    template void launch_panel<T>(T *, const FrontDesc *, int32_t *, int32_t *, TaskList, int,  \
                                  const double *, double *, hipStream_t);                       \
    template void launch_trsm<T>(T *, const FrontDesc *, const int32_t *, TaskList, TaskList,    \
                                 int, const double *, hipStream_t);                             \
    template void launch_xform<T>(T *, const FrontDesc *, TaskList, hipStream_t);               \
    template void launch_invert_diag<T>(T *, const FrontDesc *, const int32_t *, int32_t *,      \
                                        TaskList, int, int, hipStream_t);                        \
    template void launch_schur<T>(T *, const FrontDesc *, TaskList, int, int, hipStream_t);     \
    template void launch_merge_tri<T>(T *, const FrontDesc *, TaskList, hipStream_t);

MBL_INST_FRONT(float)
MBL_INST_FRONT(double)

}  // namespace mbl
