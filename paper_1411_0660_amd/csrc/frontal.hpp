// frontal.hpp -- device-side descriptors of the multifrontal LU and the
// launch wrappers of its kernels (factorisation: k_front.hip, solves:
// k_trsv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mbl {

// Panel width of the blocked partial LU of every front; also the block size
// of the triangular solves (the row interchanges of a panel stay inside it).
constexpr int FNB = 64;
// Diagonal block of the triangular solves (a multiple of FNB); these blocks of
// L11 and U11 are stored inverted after the factorisation.
constexpr int SB = 4 * FNB;
constexpr int SSB = 2 * SB;         // solve block: two factorization blocks merged
// Pivot window: the pivot of a panel column is chosen among the rows of its
// aligned PIV_WIN-row window at or below it (inside one outer block, so that
// the interchanges stay inside the block's rows)
constexpr int PIV_WIN = 256;
static_assert(PIV_WIN % FNB == 0 && SB % PIV_WIN == 0, "pivot window inside an outer block");
// end (front-local row) of the pivot window of the panel starting at row k0
__host__ __device__ inline int piv_window_end(int k0, int p) {
    return (k0 / PIV_WIN + 1) * PIV_WIN < p ? (k0 / PIV_WIN + 1) * PIV_WIN : p;
}
// Rows of one work item of a solve step (k_solve_step): 64 / STEP_RW adjacent
// columns per wave load, so small steps still spread over many workgroups.
#ifndef MBL_STEP_RW
#define MBL_STEP_RW 32
#endif
constexpr int STEP_RW = MBL_STEP_RW;
static_assert(STEP_RW == 16 || STEP_RW == 32 || STEP_RW == 64, "rows per solve-step item");

struct FrontDesc {
    int64_t off;      // first element of the dense m x m front (column-major) in the arena
    int64_t voff;     // first element of the front's solve vector block (m x nrhs)
    int32_t m, p;     // order, number of pivots
    int32_t first;    // new index of the first pivot
    int32_t cptr;     // offset of the contribution-row list (new indices)
    int32_t mapoff;   // offset of this front's rows inside its parent (relative map), -1 at roots
    int32_t parent;
    int32_t child0, nchild;  // children in FactorTables::child_ids[child0 .. child0 + nchild)
    int64_t poff;     // offset of the front's L21 / U12 partial products in the level scratch
    int32_t cptr_inv; // offset of the front's inverse relative map (m + 1 row pointers)
    int32_t pmoff;    // offset of the front's pull map: per child, per front row, the
                      // child's update row landing there, or -1 (nchild blocks of m)
    int64_t yoff;     // first element of the front's forward-solution block (p x nrhs, ld p)
    int32_t seg;      // problem of a batch the front belongs to (0 for a lone problem)
};

// A set of fronts processed by one launch and the prefix sums of the work
// items (tiles, columns, rows) each front contributes.
struct TaskList {
    const int32_t *fronts;   // front ids
    const int64_t *prefix;   // prefix[k] = first work item of fronts[k]; prefix[n] = total
    const int2 *items;       // per work item: (front id, item index inside the front)
    int32_t n;
    int64_t total;
    double elems;            // factor entries the launch streams (algorithmic)
    double rows;             // vector rows it reads and writes (per right-hand side)
    double flops;            // multiply-adds x 2 (Schur update)
};

template <class T>
struct FrontArgs {
    T *arena;
    const FrontDesc *fd;
};

// ---- factorisation ----------------------------------------------------------
// every entry of the listed fronts from their children's update blocks (zero
// where none contributes); one work item per front column
constexpr int PULL_MAXCH = 8;       // children per front the pull assembly handles
template <class T>
void launch_front_pull(T *arena, const FrontDesc *fd, const int32_t *pullmap,
                       const int32_t *child_ids, TaskList tl, hipStream_t s);
// original entries: F[pos] += (src >= 0 ? diag[src] - sigma : offv)
template <class T>
void launch_front_assemble(T *arena, const FrontDesc *fd, int64_t count, const int32_t *efront,
                           const int32_t *epos, const int32_t *esrc, const double *diag,
                           double sigma, double offv, hipStream_t s);
// step t of the blocked partial LU on every listed front; pivots below
// thresh[front's problem] are perturbed to it
template <class T>
void launch_panel(T *arena, const FrontDesc *fd, int32_t *ipiv, int32_t *nperturbed, TaskList tl,
                  int t, const double *thresh, double *uinv, hipStream_t s);
// the U rows of panel t (and its row interchanges on the other columns) and
// the L columns below it, in one launch
template <class T>
void launch_trsm(T *arena, const FrontDesc *fd, const int32_t *ipiv, TaskList tu, TaskList tlo,
                 int t, const double *uinv, hipStream_t s);
// inner (panel t, K = 64, inside its outer block) or outer-block trailing
// update; kind 0: inner update after panel t; 1: trailing update after outer
// block t (even t: K = block t; odd t: K = blocks t - 1 and t); 5: after even
// block t, block t's update of the strips of block t + 1 only; 2 and 3: the
// two products that merge the factorization blocks 2t and 2t + 1 into solve
// block t (rows below, then rows above; see k_merge_tri)
template <class T>
void launch_schur(T *arena, const FrontDesc *fd, TaskList tl, int t, int kind, hipStream_t s);
// in-place triangular products that complete the inverse of each merged
// solve block (work items: 16-column chunks, see k_merge_tri)
template <class T>
void launch_merge_tri(T *arena, const FrontDesc *fd, TaskList tl, hipStream_t s);
int merge_tri_items(int p);


// tile sizes used by the work-item counts of the task lists
constexpr int TRSM_U_COLS = 256;   // columns per work item of the U12 solve
constexpr int TRSM_L_ROWS = 64;    // rows per work item of the L21 solve
constexpr int SCHUR_TILE = 128;    // square tile of the Schur update
constexpr int SCHUR_THREADS = 512; // eight waves per Schur tile, each a 64 x 32 strip
int64_t schur_tiles(int64_t rest);

// L~ = L[., t] Linv_tt below each diagonal block, U~ = U[., t] Uinv_tt above it
template <class T>
void launch_xform(T *arena, const FrontDesc *fd, TaskList tl, hipStream_t s);
int64_t xform_items(int m, int p);
// mode bits: 1 invert the unit-lower parts, 2 the upper parts (and write the
// composite row permutation); fixed_blk >= 0 selects one block per front,
// otherwise the items are the blocks
template <class T>
void launch_invert_diag(T *arena, const FrontDesc *fd, const int32_t *ipiv, int32_t *prow,
                        TaskList tl, int mode, int fixed_blk, hipStream_t s);

// ---- triangular solves (vectors FP64, factors T) ------------------------------
// forward right-hand side of every listed front, one thread per row:
// v_f = P([b(pivots); 0] + children's updates), the children's rows found
// through the inverse relative map (inv_ptr / inv_src = (child, child row))
void launch_fwd_gather(const FrontDesc *fd, const int32_t *perm, const int32_t *prow,
                       const int32_t *inv_ptr, const int2 *inv_src, TaskList tl, int nrhs,
                       const double *b, int64_t ldb, double *vec, hipStream_t s);
// Where the backward steps write the solution of the pivot rows: by new index
// (xnew, ld n) and by original index (xout through perm, ld ldx, nrhs columns).
struct BwdIO {
    const int32_t *perm;
    double *xnew;
    double *xout;
    int64_t n, ldx;
    int nrhs;
};
// solve block t of every listed front (forward or backward, see k_trsv.hip)
template <class T>
void launch_solve_step(const T *arena, const FrontDesc *fd, TaskList tl, int t, int nrhs, bool fwd,
                       double *vec, double *yv, BwdIO bio, hipStream_t s);
// backward: partial products U12 x_c over 64 x SB tiles, x_c (the contribution
// rows, pivots of ancestors) read from xnew through the contribution-row
// lists; then their fixed-order sum into the forward solution of the pivots.
// ipw (here and in launch_fwd_l21): tiles per workgroup, 1 or 2 (a launch
// shape only: the results do not depend on it)
template <class T>
void launch_bwd_u12(const T *arena, const FrontDesc *fd, TaskList tl, int nrhs,
                    const int32_t *contrib, const double *xnew, int64_t n, double *part, int ipw,
                    hipStream_t s);
void launch_bwd_u12_reduce(const FrontDesc *fd, TaskList tl, int nrhs, double *yv,
                           const double *part, hipStream_t s);
// forward contribution rows: V[p:m] -= L~21 V[0:p] (tiles into part, then the
// reduction into the solve vectors)
template <class T>
void launch_fwd_l21(const T *arena, const FrontDesc *fd, TaskList tl, int nrhs, const double *vec,
                    double *part, int ipw, hipStream_t s);
void launch_fwd_l21_reduce(const FrontDesc *fd, TaskList tl, int nrhs, double *vec,
                           const double *part, hipStream_t s);

}  // namespace mbl
