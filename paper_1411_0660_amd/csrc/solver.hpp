// solver.hpp -- per-L plans, the numeric multifrontal factor/solve drivers and
// the Krylov-Schur eigensolver that sit between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "frontal.hpp"
#include "obs.hpp"
#include "symbolic.hpp"

namespace mbl {

struct StepTasks {                    // one 64-wide panel of the blocked LU
    TaskList panel, trsm_u, rows_below, schur;
};

// Outer blocks are applied in pairs: after an even block t whose successor
// exists, only the strips block t + 1 reads are updated (strip); after odd
// block t + 1 the trailing matrix takes both blocks at once (schur, K = 2 SB).
// A front whose last block is even takes that block alone (schur, K = SB).
struct OuterTasks {                   // one 256-wide outer block
    TaskList schur, strip;
};

struct LevelTasks {
    int64_t ebegin = 0, ecount = 0;    // original entries of the level
    TaskList all;                      // every front, one item each
    TaskList pull;                     // assembly from the children: one item per front column
    std::vector<StepTasks> steps;
    std::vector<OuterTasks> outer;
    // triangular solves, one list per SB-wide solve block
    std::vector<TaskList> fstep, bstep;
    TaskList fgather;                  // forward right-hand sides, 256-row items
    TaskList u12, u12red;              // U12 x_c tiles and their reduction
    TaskList l21, l21red;              // forward contribution rows: tiles and reduction
    int64_t part_elems = 0;            // level scratch of the L21 / U12 partial products
};

struct Plan {
    int L = 0;
    int nseg = 1;                      // problems of a batch plan (copies of one front tree)
    int64_t dim = 0, nnz = 0;          // of the whole (block-diagonal) matrix
    DevBuf basis, rowptr, col;
    std::vector<int32_t> h_rowptr, h_col;
    bool have_symbolic = false;
    FrontTree tree;
    std::vector<FrontDesc> h_fd;
    int64_t arena_elems = 0, vec_elems = 0;
    std::vector<LevelTasks> levels;
    TaskList inv;                      // SB diagonal blocks of every front (inversion)
    TaskList xform;                    // 16-row panels folded with the inverted blocks
    std::vector<TaskList> fold_lo, fold_up;   // per merged solve block: the two products
    TaskList merge;                    // in-place triangular products of the merge
    int64_t y_elems = 0;               // forward-solution blocks (sum of p x 16)
    int64_t part_elems = 0;            // max over levels
    DevBuf d_fd, d_perm, d_contrib, d_pullmap, d_child_ids, d_tfronts, d_tprefix, d_titems;
    DevBuf d_efront, d_epos, d_esrc, d_inv_ptr, d_inv_src;
    // Launch shapes of the solves chosen by the solve autotuner, per factor
    // precision and right-hand-side count (key sizeof(T) * 100 + nrhs): tiles
    // per workgroup of the L21 and U12 products at every tree level.  Set
    // once, under the plan cache's lock; the results do not depend on them.
    struct SolveTune {
        std::vector<int8_t> l21, u12;
    };
    std::map<int, SolveTune> tune;
};

template <class T>
struct Factor {
    int L = -1;
    int64_t dim = 0;                   // order of the factored (possibly batched) matrix
    DevBuf arena, ipiv, prow, npert, thr;
    DevBuf uinv;                       // per front: U_tt^-1 of the current panel (FNB x FNB)
    bool valid = false;
    double sigma = 0.0;
};

struct SolveStats {
    int ir_iters = 0;
    int n_perturbed = 0;
    std::vector<int> perturbed;        // per problem of a batch plan
    double backward_error = 0.0;
    double t_factor = 0.0, t_solve = 0.0;
    int n_rhs = 0;
    int gmres_inner = 0;               // GMRES iterations of the latest shifted solve
};

// Per-L plans (basis, CSR pattern, symbolic analysis, task lists): read-only
// once built, shared by the contexts of one device (the serving slots).  Only
// the owning context builds plans, so their memory is charged to its budget.
struct PlanCache {
    std::recursive_mutex mu;
    std::map<int, std::unique_ptr<Plan>> plans;
    std::map<int, std::unique_ptr<Plan>> batched;     // key L * 100 + problems
};

class Context {
  public:
    Context(int device, size_t budget, hipStream_t stream);
    // a context on the same device that reads the plans of `owner`
    Context(const Context &owner, size_t budget);
    ~Context();

    int device;
    hipStream_t stream;
    bool own_stream;
    Budget budget;
    std::recursive_mutex mu;

    Plan &plan(int L);                 // basis + CSR on the device (cached)
    void ensure_symbolic(Plan &p);     // ordering + front tables (cached)
    void build_tables(Plan &p);        // front tables of a plan whose tree is set
    Plan &batch_plan(int L, int nseg); // nseg copies of plan(L), solved together (cached)
    // free the per-request work buffers (factors, solve vectors, Krylov bases)
    void trim();

    // realization state: fields + diagonal of H on the device
    void set_realization(Plan &p, double J, const double *fields_host, double h, uint64_t seed,
                         bool use_seed);
    double J = 1.0, offv = 0.5;
    DevBuf d_fields, d_diag;
    std::vector<double> h_fields;

    // y = (H - shift) x; diag: the diagonal of H (nullptr: d_diag)
    void spmv(Plan &p, double shift, int nvec, const double *x, double *y,
              const double *diag = nullptr);
    // extremal eigenvalues by Krylov-Schur on H
    void extremal(Plan &p, double &emin, double &emax, int &napply);
    // the same for the p.nseg problems of a batch plan (diag: their diagonals,
    // packed); emin, emax, napply: one per problem
    void extremal_seg(Plan &p, const double *diag, double *emin, double *emax, int *napply);

    // shifted LU + refined solves
    void factor(Plan &p, int prec, double sigma, double anorm, SolveStats &st);
    // X = (H - sigma)^-1 B (device, original basis order, ld = dim), refined in FP64
    void shift_solve(Plan &p, int prec, int nrhs, const double *B, double *X, SolveStats &st);

    // Batches: the p.nseg problems of a batch plan, each at its own shift.
    // LU of every problem; shifted: their diagonals of H - sigma_s, packed
    void factor_batch(Plan &bp, int prec, const double *shifted, const std::vector<double> &anorm,
                      SolveStats &st);
    struct BatchSolveStats {
        std::vector<int> ir_iters, passes, pass_rhs;   // per problem
        // problems whose lone solve would leave the plain refinement (GMRES,
        // a refinement failure): no longer refined, solved alone afterwards
        std::vector<char> dropped;
        std::vector<uint32_t> hooks;                  // refinement-stall test hooks
        double t_solve = 0.0;
        explicit BatchSolveStats(int nseg)
            : ir_iters(nseg, 0), passes(nseg, 0), pass_rhs(nseg, 0), dropped(nseg, 0),
              hooks(nseg, 0) {}
    };
    // X = (H_s - sigma_s)^-1 B per problem (packed columns, ld = bp.dim), each
    // refined as a lone solve is; problems with skip[s] or bs.dropped[s] get
    // one unrefined pass
    void shift_solve_batch(Plan &bp, int prec, int nrhs, const double *B, double *X,
                           const double *shifted, const std::vector<double> &anorm,
                           const std::vector<char> &skip, BatchSolveStats &bs);
    DevBuf d_bdiag, d_bshift;          // diagonals of a batch's H and H - sigma, packed

    // block Krylov-Schur on an operator; Ritz vectors of the nwant selected
    // values (priority order) land in out (dim x nwant)
    enum class Want { LargestAbs, BothEnds };
    struct KSOut {
        std::vector<double> theta, rho;
        double tmin = 0.0, tmax = 0.0;   // extreme Ritz values of the last Rayleigh-Ritz
        int restarts = 0, napply = 0, nconv = 0;
    };
    // all eigenpairs of count small symmetric matrices (host in, host out;
    // device Jacobi, one workgroup each)
    void small_eig_batch(int count, int m, const std::vector<std::vector<double>> &A,
                         std::vector<std::vector<double>> &w,
                         std::vector<std::vector<double>> &Z, bool general = false);
    // block Krylov-Schur on nseg problems of order n with packed vectors (ld
    // nseg n); conv(problem, theta, rho); seeds[nseg]; out: nseg n x nwant
    // op(X, Y, nb, finished): Y = Op X for nb packed columns; finished[s] != 0
    // marks problems whose result is final (their columns are not used)
    using KSOp = std::function<void(const double *, double *, int, const std::vector<char> &)>;
    void krylov_schur(int64_t n, int nseg, int b, int ncv, int nkeep, int nwant, Want want,
                      const KSOp &op, const std::function<bool(int, double, double)> &conv,
                      int max_restarts, const uint64_t *seeds, double *out,
                      std::vector<KSOut> &result, const std::vector<char> *dropped = nullptr);

    // per-launch timing of one kernel class (mbl_profile_enable)
    struct Prof {
        std::string cls;
        std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
        size_t used = 0;
        int64_t launches = 0;
        double bytes = 0.0, flops = 0.0, seconds = 0.0;
    } prof;
    bool prof_on(const char *cls) const { return !prof.cls.empty() && prof.cls == cls; }
    void prof_begin();
    void prof_end(double bytes, double flops);
    void prof_collect();

    ObsWork obs;
    DevBuf d_psi, d_psi2, d_hpsi, d_e, d_cpart, d_obs, d_r_out, d_se;
    uint32_t hooks = 0;                // MBL_HOOK_* of the request being solved
    double anorm_ = 1.0;               // ||H - sigma|| estimate of the current factor
    // Backward error each shifted solve is refined to.  Standalone solves and
    // FP32 factors: SOLVE_TARGET.  FP64 factors inside the eigensolver:
    // 0.05 tol (5e-12 at the default tol = 1e-10): the Krylov test accepts a
    // Ritz pair at a relative residual of 0.1 tol, and an operator backward
    // error be adds about 2 be to it (||H - sigma|| <= 2 ||H|| for sigma
    // inside the spectrum).  An FP64 first solve either meets that or a sweep
    // takes it far below; refinement of FP32 factors contracts slowly and
    // would stop just under the target, at the limit of what the Krylov test
    // tolerates, so it keeps the tighter one.
    static constexpr double SOLVE_TARGET = 1e-13;
    static double eig_refine_target(double tol) { return std::min(SOLVE_TARGET * 50.0, 0.05 * tol); }
    double refine_target = SOLVE_TARGET;
    double hnorm_ = 1.0;
    // passes of right-hand-side blocks through the factors, and the vectors
    // they carried (forward plus backward sweep each), since creation
    int64_t lu_passes = 0, lu_pass_rhs = 0;

  private:
    std::shared_ptr<PlanCache> plans_;
    bool owns_plans_ = true;
    Factor<float> f32_;
    Factor<double> f64_;
    Factor<double> fb64_;              // factors of a batch of problems (one replicated plan)
    Factor<float> fb32_;
    DevBuf d_on;                       // per problem of a batch: still refining
    DevBuf d_vec, d_yv, d_upart, d_xnew, d_r, d_d, d_part, d_V, d_V2, d_W, d_small, d_ritz, d_tnpart;
    DevBuf d_gV, d_gZ, d_gpart, d_gcoef;   // GMRES refinement: bases, partials, coefficients
    DevBuf d_stage;                        // Krylov coefficients, R factors, flags per restart cycle
    PinnedBuf h_stage;                     // their copy in page-locked memory
    PinnedBuf h_ritz;                      // Rayleigh-Ritz matrices and their eigenpairs
    PinnedBuf h_coef;                      // restart coefficients of every problem
    // LU of the plan's matrix with diagonal diag - sigma; thresh: static-pivot
    // threshold of each problem of the plan
    template <class T> void factor_t(Plan &p, Factor<T> &f, const double *diag, double sigma,
                                     const std::vector<double> &thresh, SolveStats &st);
    template <class T> void lu_apply_seq(Plan &p, Factor<T> &f, int nrhs, const double *b,
                                         int64_t ldb, double *x, int64_t ldx,
                                         const Plan::SolveTune &tn);
    // the solve launch shapes of (plan, precision, nrhs), timed on this factor
    // at first use: every level's L21 and U12 products with one and with two
    // tiles per workgroup (their outputs are scratch partial sums), the faster
    // kept (MBL_NO_TUNE: one tile everywhere)
    template <class T> Plan::SolveTune solve_tune(Plan &p, Factor<T> &f, int nrhs);
    // captured launch sequences of lu_apply (see lu_apply)
    struct GraphKey {
        const Plan *plan;              // lone and batch plans of one L differ
        int L, tsize, nrhs;
        const void *bufs[8];
        bool operator<(const GraphKey &o) const {
            if (plan != o.plan) return std::less<const Plan *>()(plan, o.plan);
            if (L != o.L) return L < o.L;
            if (tsize != o.tsize) return tsize < o.tsize;
            if (nrhs != o.nrhs) return nrhs < o.nrhs;
            for (int i = 0; i < 8; i++)
                if (bufs[i] != o.bufs[i]) return bufs[i] < o.bufs[i];
            return false;
        }
    };
    std::map<GraphKey, hipGraphExec_t> graphs_;
    bool use_graphs_ = true;
    DevBuf d_gin, d_gout;              // staging vectors of the captured sequences
    void clear_graphs();
    template <class T> void lu_apply(Plan &p, Factor<T> &f, int nrhs, const double *b,
                                     int64_t ldb, double *x, int64_t ldx);
    template <class T> void gmres_refine(Plan &p, Factor<T> &f, int nrhs, const double *B,
                                         double *X, double target, SolveStats &st);
    template <class T> void refine(Plan &p, Factor<T> &f, int nrhs, const double *B, double *X,
                                   SolveStats &st);
    template <class T> void refine_batch(Plan &p, Factor<T> &f, int nrhs, const double *B,
                                         double *X, const double *shifted,
                                         const std::vector<double> &anorm,
                                         const std::vector<char> &skip, BatchSolveStats &bs);
};

// Block size of the shift-invert Krylov iteration (right-hand sides per pass
// through the factors) when the problem does not set one: 8 from sector
// dimension 1e5 (L = 20), 4 from 128 (L = 10), single vectors below.
inline int default_block(int64_t n) { return n >= 100000 ? 8 : (n >= 128 ? 4 : 1); }

// extremal: optional {E_min, E_max} of this realization, computed earlier
// (energy sweeps reuse them); nullptr computes them.
void solve_problem(Context &ctx, const mbl_problem &prob, mbl_result &res,
                   const double *extremal = nullptr);

// Whether count problems can be solved as one batch: one chain length (sector
// of dimension >= 128), J, nev, precision, tolerance and Krylov settings, no
// test hooks but the refinement-stall ones, 2 <= count <= 16.
bool batchable(const mbl_problem *probs, int count);
// Solves a batchable set on the batch plan of nseg = count copies: every
// problem's arithmetic is that of solve_problem (results bitwise the same),
// the launches are shared.  A problem whose lone solve takes a path the batch
// cannot follow (GMRES refinement of an FP32 factor, a refinement failure)
// leaves the batch and is solved alone after it.  status[k]: that problem's
// status (MBL_ENOTCONV results are still written).  Returns false, with
// nothing valid written, when the set is not batchable or the batch does not
// fit in memory: then the caller solves the problems one at a time.
bool solve_batch(Context &ctx, int count, const mbl_problem *probs, mbl_result *res, int *status);

}  // namespace mbl
