/*
 * mbl.h -- C ABI of libmbl, an MI355X (gfx950) shift-invert eigensolver for the
 * periodic random-field Heisenberg chain
 *
 *     H = J sum_{i=1..L} S_i . S_{i+1} + sum_i h_i S^z_i ,   S_{L+1} = S_1,
 *
 * (Eq. (1) of Luitz, Laflorencie, Alet, "Many-body localization edge in the
 * random-field Heisenberg chain", 2014), restricted to the S^z = 0 sector for
 * even L and to the S^z = +1/2 sector for odd L (the paper's odd sizes; the
 * smallest |S^z| an odd chain has).
 * For one disorder realization (L, h, seed) and an energy-density target eps
 * it computes the nev eigenpairs nearest sigma = E_min + eps (E_max - E_min)
 * with a sparse LU of (H - sigma) driving a Krylov method on (H - sigma)^-1,
 * and the eigenvector observables (section "Numerical method" and section
 * "Characterization of ergodic and localized regimes").
 *
 * Conventions shared by every entry point:
 *   - Return value: int status, MBL_OK (0) or a negative MBL_E* code; nothing
 *     else crosses the ABI on failure (no exceptions).  mbl_strerror() names a
 *     code; mbl_last_error() gives a message for the last failure on the
 *     calling thread.
 *   - Basis order: the sector is the set of L-bit words with nup = (L + 1) / 2
 *     bits set (integer division: L/2 for even L), in ascending integer
 *     order; bit i is site i+1, bit set = spin up.  Every vector of length
 *     dim = C(L, nup) is in this order.  The half chain A of the observables is
 *     sites 1..L/2 (integer division: the low L/2 bits).
 *   - Fields: h_i = h (2 u_i - 1), u_i = (z_i >> 11) 2^-53 where z_i is the
 *     i-th output of SplitMix64 (Steele, Lea, Flood 2014) started from state
 *     = seed (uniform distribution on [-h, h], the sentence after Eq. (1)).
 *   - Pointers named *_host are host memory owned by the caller; pointers
 *     named *_dev are device memory on the context's device, owned by the
 *     caller.  The library owns all device memory it allocates itself and
 *     releases it in mbl_destroy().
 *   - All work runs on the context's HIP stream; calls returning host results
 *     synchronise that stream before returning.
 *   - A context is not safe for concurrent calls from several threads except
 *     for mbl_submit / mbl_poll / mbl_wait, which are.
 */
#ifndef MBL_H
#define MBL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define MBL_OK        0
#define MBL_EINVAL   -1   /* bad argument: L out of range, nev > dim, eps not in [0,1], NULL */
#define MBL_ENOMEM   -2   /* device allocation failed or footprint above the context budget */
#define MBL_ENOTCONV -3   /* fewer than nev pairs reached the tolerance; partial results are valid */
#define MBL_ENUMERIC -4   /* shifted solve could not be refined to the target backward error */
#define MBL_EDEVICE  -5   /* HIP runtime error */
#define MBL_EBUSY    -6   /* request queue full */
#define MBL_ENOTFOUND -7  /* unknown ticket */

#define MBL_L_MAX 22      /* largest L with a 32-bit sector word and int32 indices */

/* ---- precision of the sparse LU ------------------------------------------ */
typedef enum {
    MBL_FP64 = 0,        /* LU factors in FP64 ("plain" shift-invert) */
    MBL_FP32_IR64 = 1    /* LU factors in FP32 on MFMA, every solve refined in FP64 */
} mbl_precision;

/* ---- request flags -------------------------------------------------------- */
#define MBL_WANT_VECTORS  1u  /* copy eigenvectors to result.evecs */
#define MBL_WANT_OBS      2u  /* compute r, S_1, S_E into result (default on in mbl_problem_init) */
#define MBL_WANT_OBS_EXTRA 4u /* also S_2, F, f and KL (result.s2, .fluct, .dynfrac, .kl) */
/* Test hooks: each forces one failure path of the request so that its
 * documented outcome can be checked; the context stays usable afterwards. */
#define MBL_HOOK_IR_STALL32 0x100u /* refinement with FP32 factors reports stagnation at its
                                      first sweep: the request refactors in FP64 and goes on
                                      (result.fallback = 1, MBL_OK) */
#define MBL_HOOK_IR_STALL64 0x200u /* refinement with FP64 factors reports stagnation at its
                                      first sweep: MBL_ENUMERIC (no wider precision to fall
                                      back to) */
#define MBL_HOOK_NO_CONV    0x400u /* the Krylov convergence test never passes: the iteration
                                      stops after max_restarts restarts and the request ends
                                      with MBL_ENOTCONV and its partial results */

/* One shift-invert eigenproblem (section "Numerical method"). */
typedef struct {
    int L;                 /* 2 <= L <= MBL_L_MAX; odd L: the S^z = +1/2 sector */
    double J;              /* exchange coupling (1.0 in the paper's model); 0 allowed */
    double h;              /* disorder strength: h_i uniform in [-h, h] */
    uint64_t seed;         /* SplitMix64 seed of the fields */
    const double *fields;  /* optional host array[L]; when non-NULL it replaces (h, seed) */
    double eps;            /* energy-density target in [0, 1]; sigma = E_min + eps (E_max - E_min) */
    double sigma;          /* NaN: derive from eps; finite: use this shift directly */
    int nev;               /* eigenpairs wanted, 1 <= nev <= dim */
    int prec;              /* mbl_precision */
    double tol;            /* residual target ||H psi - E psi|| <= tol ||H||_2; 0 -> 1e-10 */
    uint32_t flags;        /* MBL_WANT_* */
    int block;             /* Krylov block size b (right-hand sides per LU pass); 0 -> default */
    int ncv;               /* Krylov basis size; 0 -> default from nev and block */
    int max_restarts;      /* 0 -> default */
    size_t fail_alloc_bytes; /* test hook: 0 = off; otherwise every device allocation of this
                              request fails (MBL_ENOMEM) once the request has allocated this many
                              bytes in total; the context stays usable */
} mbl_problem;

/* Results; every pointer is a caller-owned host buffer or NULL (not wanted). */
typedef struct {
    double *evals;         /* [nev] ascending */
    double *evecs;         /* [nev * dim], eigenvector j at evecs + j*dim (basis order) */
    double *resid;         /* [nev] ||H psi - E psi||_2 / ||H||_2, FP64 SpMV */
    double *r;             /* [nev - 2] gap ratios of the consecutive levels (item (i)) */
    double *s1;            /* [nev] participation entropy S_1 (item (iii)) */
    double *se;            /* [nev] half-chain entanglement entropy, A = sites 1..L/2 (item (ii)) */
    double *s2;            /* [nev] participation entropy S_2         (MBL_WANT_OBS_EXTRA) */
    double *fluct;         /* [nev] bipartite fluctuations of S^z_A  (MBL_WANT_OBS_EXTRA) */
    double *dynfrac;       /* [nev] dynamical spin fraction f          (MBL_WANT_OBS_EXTRA) */
    double *kl;            /* [nev - 1] KL divergence of neighbours    (MBL_WANT_OBS_EXTRA) */
    /* outputs */
    double emin, emax, sigma, hnorm; /* extremal energies, shift, ||H||_2 = max(|E_min|, |E_max|) */
    double r_mean;         /* mean of the finite r values */
    double max_resid;      /* max of resid[] */
    int nconv;             /* pairs that met tol (== nev on success) */
    int n_restarts;        /* Krylov restarts */
    int n_opapply;         /* right-hand sides pushed through the shifted solve */
    int n_passes;          /* passes through the LU factors (forward and backward sweep of a
                              block of right-hand sides), refinement included */
    int n_pass_rhs;        /* right-hand sides those passes carried in total */
    int ir_iters_max;      /* largest number of refinement sweeps of one solve */
    int n_perturbed;       /* pivots replaced by the static-pivot threshold */
    int fallback;          /* 0 none; 1 FP32 refinement stalled -> FP64 LU used */
    double t_phase[8];     /* seconds: 0 assemble, 1 extremal, 2 symbolic, 3 factor,
                              4 Krylov (solves + orthogonalisation), 5 observables,
                              6 total, 7 of which shifted solves */
    double t_submit, t_start, t_done; /* requests (mbl_submit): seconds since the server
                              started at submission, admission and completion */
    int batch;             /* problems solved in one batch with this one (1: alone) */
} mbl_result;

/* Statistics of the per-L symbolic analysis (fill-reducing nested dissection,
 * assembly tree of dense fronts). */
typedef struct {
    int64_t dim, nnz_h;    /* sector dimension, nonzeros of H */
    int64_t n_fronts, n_levels;
    int64_t max_front, max_pivots;   /* largest front order m = p + c, largest p */
    int64_t nnz_factor;    /* entries of L and U (p^2 + 2 p c summed over fronts) */
    int64_t front_entries; /* sum of m^2 (storage of all dense fronts) */
    double flops_factor;   /* sum over fronts of (2/3) p^3 + 2 p^2 c + 2 p c^2 (LU) */
    double seconds;        /* host time of the analysis */
} mbl_symbolic_info;

/* Diagnostics of one shifted solve. */
typedef struct {
    int ir_iters;          /* refinement sweeps of the worst right-hand side */
    int n_perturbed;       /* perturbed pivots in the factorisation */
    double backward_error; /* max_k ||b - (H - sigma) x|| / (||H - sigma|| ||x|| + ||b||) */
    double t_factor, t_solve;
} mbl_solve_info;

/* ---- context ------------------------------------------------------------- */
typedef struct mbl_ctx mbl_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory the context may hold (0 = 90% of the free memory).  hip_stream is a
 * hipStream_t to run on (NULL = the context creates its own). */
int mbl_create(int device, size_t hbm_budget_bytes, void *hip_stream, mbl_ctx **out);
int mbl_destroy(mbl_ctx *ctx);
const char *mbl_strerror(int code);
const char *mbl_last_error(void);
void mbl_problem_init(mbl_problem *p);   /* defaults: J = 1, sigma = NaN, prec FP64, MBL_WANT_OBS */

/* ---- single steps (parity hooks; each runs the same kernels as mbl_solve) -- */
int64_t mbl_sector_dim(int L);                        /* C(L, (L + 1) / 2), or -1 out of range */
int mbl_fields(int L, double h, uint64_t seed, double *out_host); /* SplitMix64 fields */
/* Sector words in basis order, enumerated on the device. */
int mbl_basis(mbl_ctx *ctx, int L, uint32_t *out_host);
/* Index of each word in the sector (-1 for a word outside it), on the device. */
int mbl_rank(mbl_ctx *ctx, int L, const uint32_t *words_host, int64_t count, int64_t *ranks_host);
/* CSR of H assembled on the device: rowptr[dim+1], col[nnz], val[nnz] (diagonal
 * included, columns ascending).  Any output may be NULL; *nnz_out gets nnz. */
int mbl_hamiltonian(mbl_ctx *ctx, int L, double J, const double *fields_host,
                    int32_t *rowptr_host, int32_t *col_host, double *val_host, int64_t *nnz_out);
/* y = H x for nvec vectors (column-major dim x nvec), FP64, on the device. */
int mbl_spmv(mbl_ctx *ctx, int L, double J, const double *fields_host, int nvec,
             const double *x_host, double *y_host);
/* Extremal eigenvalues by Lanczos on H. */
int mbl_extremal(mbl_ctx *ctx, int L, double J, const double *fields_host,
                 double *emin, double *emax);
/* Eigenpairs of `count` dense symmetric matrices of order m (1 <= m <= 1024),
 * the Rayleigh-Ritz step of the shift-invert Krylov iteration (section
 * "Numerical method": the projected matrix), by the cyclic Jacobi method on the
 * device, one workgroup per matrix.  A_host: count column-major m x m
 * matrices, back to back (only the values are read; symmetry is assumed).
 * Outputs: w_host[count * m], each matrix's eigenvalues ascending;
 * Z_host[count * m * m], column j of matrix k's block = the unit eigenvector
 * of w_host[k * m + j].  flags: 0, or MBL_EIG_GENERAL to run the kernel of
 * orders above 128 also at smaller orders (it gives the same bits: a check of
 * the two kernels).  MBL_ENUMERIC if a matrix needs more than 40 sweeps. */
#define MBL_EIG_GENERAL 1
int mbl_ritz_eig(mbl_ctx *ctx, int count, int m, const double *A_host, double *w_host,
                 double *Z_host, int flags);
/* Fill-reducing ordering and front tree for L (cached in the context). */
int mbl_symbolic(mbl_ctx *ctx, int L, mbl_symbolic_info *info);
/* Fill-reducing permutation: perm_host[k] = basis index eliminated k-th. */
int mbl_ordering(mbl_ctx *ctx, int L, int32_t *perm_host);
/* The assembly tree of dense fronts behind mbl_symbolic (test and inspection
 * hook).  Front f (post-order: children before parents) eliminates the
 * permuted indices first[f] .. first[f] + npiv[f] - 1 and passes an update to
 * the ncontrib[f] contribution rows contrib[cptr[f] .. cptr[f] + ncontrib[f] - 1]
 * (permuted indices, ascending) on to front parent[f] (-1 for a root).  Call
 * with NULL arrays to get *n_fronts and *n_contrib, then again with host arrays
 * of those lengths (first, npiv, ncontrib, parent: n_fronts int32; cptr:
 * n_fronts int64; contrib: n_contrib int32).  Either size pointer may be NULL
 * on the second call. */
int mbl_front_tree(mbl_ctx *ctx, int L, int32_t *first, int32_t *npiv, int32_t *ncontrib,
                   int32_t *parent, int64_t *cptr, int32_t *contrib, int64_t *n_fronts,
                   int64_t *n_contrib);
/* x = (H - sigma)^-1 b for nrhs right-hand sides (column-major dim x nrhs):
 * multifrontal LU of H - sigma in precision prec, then forward/back solves
 * with FP64 iterative refinement. */
int mbl_shift_solve(mbl_ctx *ctx, int L, double J, const double *fields_host, double sigma,
                    int prec, int nrhs, const double *b_host, double *x_host,
                    mbl_solve_info *info);
/* Observables of given unit vectors (nev columns of length dim, ascending
 * energies evals[nev]): r[nev-2], s1[nev], se[nev]; NULL outputs are skipped. */
int mbl_observables(mbl_ctx *ctx, int L, int nev, const double *evals_host,
                    const double *evecs_host, double *r_host, double *s1_host, double *se_host);
/* S_2, F, f, KL of given vectors (the remaining indicators of the paper). */
int mbl_observables_extra(mbl_ctx *ctx, int L, int nev, const double *evecs_host,
                          double *s2_host, double *fluct_host, double *dynfrac_host,
                          double *kl_host);

/* ---- allocation-free observables -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It computes
 * what mbl_observables computes (gap ratios, S_1, S_E of nev given unit
 * vectors), with the same kernels, but the inputs and outputs are device
 * buffers the caller owns on the calling thread's current HIP device, and the
 * work buffers are one fixed array of MBL_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends.  No call
 * allocates or frees device memory.
 *   evals_dev  [nev] ascending energies (read only when r_dev is not NULL)
 *   evecs_dev  column-major dim x nev, leading dimension ld >= dim (basis order)
 *   r_dev [nev - 2], s1_dev [nev], se_dev [nev]; a NULL output is skipped
 *   hip_stream a hipStream_t of the current device (NULL = the null stream);
 *              the call only enqueues work on it and returns, so results are
 *              ready once the stream is synchronised.
 * Limits: nev <= MBL_NOALLOC_MAX_NEV; S_E is computed in chunks of as many
 * vectors as the array holds (one at L = 22); a size beyond the array returns
 * MBL_EINVAL with a message.  The first call on a device looks up the array's
 * device address and loads small constant tables, so it should not be the
 * call that is captured.  Every call on one device shares that device's
 * array and leaves its contents behind: calls that overlap in time on one
 * device (several streams or threads) race and must be serialised by the
 * caller. */
#define MBL_NOALLOC_SCRATCH_BYTES (32u << 20)
#define MBL_NOALLOC_MAX_NEV 256
int mbl_observables_noalloc(int L, int nev, const double *evals_dev, const double *evecs_dev,
                            int64_t ld, double *r_dev, double *s1_dev, double *se_dev,
                            void *hip_stream);

/* ---- the whole path ------------------------------------------------------ */
/* Fields -> assembly -> E_min/E_max -> sigma -> LU of H - sigma -> block
 * Krylov-Schur on (H - sigma)^-1 -> nev pairs nearest sigma -> observables. */
int mbl_solve(mbl_ctx *ctx, const mbl_problem *prob, mbl_result *res);
/* Several disorder realizations or targets solved together (batching): the
 * `count` problems (1..16) are factored, solved and iterated in shared launches
 * on a block-diagonal plan whose front tree is `count` copies of the lone one,
 * and each problem's arithmetic is exactly that of mbl_solve (its results are
 * bitwise the same as a separate call).  Problems batch when they share L
 * (sector dimension >= 128), J, nev, prec, tol, block, ncv and max_restarts
 * and set no test hook other than MBL_HOOK_IR_STALL32/64; otherwise, or when
 * the batch does not fit in memory, they are solved one after another.  A
 * problem whose lone solve takes a path the batch cannot follow (GMRES
 * refinement or an FP64 fallback of an FP32 factor, a refinement failure)
 * leaves the batch and is solved alone after it.  probs[k] -> results[k] (the mbl_result buffers as for
 * mbl_solve); status[k] = that problem's mbl status.  t_phase of batched
 * problems are the batch's.  Returns MBL_OK, or the first nonzero status. */
int mbl_solve_batch(mbl_ctx *ctx, int count, const mbl_problem *probs, mbl_result *results,
                    int *status);
/* Predicted device bytes of one request (factor fronts + Krylov basis + work). */
int mbl_footprint(mbl_ctx *ctx, int L, int prec, int nev, int block, size_t *bytes);

/* ---- measurement ---------------------------------------------------------- */
/* Per-launch timing of one kernel class with HIP events on the context's
 * stream, plus the algorithmic bytes and flops of the timed launches (what the
 * method must move or compute, not what the hardware counters report).
 * Classes: "schur" (trailing update of the frontal LU), "fwd_update",
 * "bwd_update" (diagonal-block products of the solves), "l21" and "u12" (the
 * off-diagonal block products L21 y and U12 x of the solves), "spmv". */
typedef struct {
    int64_t launches;      /* launches timed since mbl_profile_enable */
    double seconds;        /* sum of their durations */
    double bytes;          /* algorithmic HBM bytes of those launches */
    double flops;          /* algorithmic flops of those launches */
} mbl_kernel_profile;
/* Start timing `kernel_class` (NULL or "" stops timing); clears the counters. */
int mbl_profile_enable(mbl_ctx *ctx, const char *kernel_class);
/* Synchronises the stream and returns the counters. */
int mbl_profile_read(mbl_ctx *ctx, mbl_kernel_profile *out);

/* ---- energy sweep of one realization, disorder averages ------------------
 * The paper's protocol ("Numerical method" section): for each disorder
 * realization the extremal energies are computed once and then the eigenpairs
 * nearest every target of an energy-density grid (eps = 0.05, 0.1, ..., 0.95);
 * observables are first averaged over the eigenstates of one realization (one
 * bin per realization and target, since eigenstates of one sample are
 * correlated) and then over realizations, with the standard error taken over
 * the bins.  sigma_E, the standard deviation of the entanglement entropy, is
 * the quantity the entanglement discussion of the paper follows across the
 * transition. */
#define MBL_NBIN 10
enum {
    MBL_BIN_R = 0,      /* mean of the finite gap ratios r_n (item (i)) */
    MBL_BIN_S1 = 1,     /* mean participation entropy S_1 */
    MBL_BIN_S2 = 2,     /* mean participation entropy S_2 */
    MBL_BIN_SE = 3,     /* mean half-chain entanglement entropy S_E */
    MBL_BIN_SE2 = 4,    /* mean of S_E^2 (for sigma_E) */
    MBL_BIN_FLUCT = 5,  /* mean bipartite fluctuation F */
    MBL_BIN_DYNFRAC = 6,/* mean dynamical spin fraction f */
    MBL_BIN_KL = 7,     /* mean of the finite KL divergences of neighbours (NaN if none) */
    MBL_BIN_EDENS = 8,  /* mean energy density (E - E_min) / (E_max - E_min) of the states */
    MBL_BIN_NCONV = 9   /* converged pairs */
};
/* Solves the realization of `base` (L, J, h, seed or fields, nev, prec, tol,
 * block, ncv, max_restarts; base->eps, base->sigma and MBL_WANT_VECTORS are
 * ignored) at each eps[k], k < n_eps, reusing its fields, H, the symbolic
 * analysis and E_min / E_max (computed once, by the first target), and writes
 * that target's bin to bins[k * MBL_NBIN + q] (host, n_eps * MBL_NBIN doubles;
 * NaN where a target failed) and its mbl status to status[k] (host, n_eps
 * ints; MBL_ENOTCONV bins come from the partial results).  Each target's
 * arithmetic is that of mbl_solve with the same problem, so its results are
 * identical to a separate call.  Returns MBL_OK, the status of the first target
 * that did not converge (the others are still solved), or an argument or device
 * error (then later targets keep MBL_EBUSY: not attempted). */
int mbl_sweep(mbl_ctx *ctx, const mbl_problem *base, const double *eps, int n_eps,
              double *bins, int *status);
/* Disorder average of one target's bins over n_real realizations
 * (bins[i * MBL_NBIN + q], host): mean[q] over the realizations whose bin q is
 * finite, sem[q] = sqrt(sum_i (b_i - mean)^2 / (k (k - 1))) over those k bins
 * (NaN for k < 2), and, if sigma_e is not NULL, *sigma_e = the standard
 * deviation of S_E over all eigenstates of all realizations (each realization
 * weighted equally), sqrt(max(0, mean[SE2] - mean[SE]^2)).  Host arithmetic
 * only; mean and sem are MBL_NBIN doubles. */
int mbl_disorder_average(const double *bins, int n_real, double *mean, double *sem,
                         double *sigma_e);

/* ---- serving: continuous batching of solve requests ----------------------
 * The paper's workload is many independent solves (disorder realizations x
 * energy targets, "Numerical method" section).  Requests of mixed sizes are
 * taken in arrival order and admitted to one of `slots` solver slots (each its
 * own HIP stream and host thread, so their work overlaps on the device) when a
 * slot is idle and the device bytes all slots hold, plus the request's
 * predicted footprint (mbl_footprint; an FP32 request also counts the FP64
 * factor of its fallback), fit `budget_bytes`; while it runs, a slot's
 * allocations are capped at the footprint it was admitted with.  A request that does not fit
 * lets later ones pass, at most 2 x slots times.  The per-L plans are built
 * once by the context and shared.  Queued requests that can share launches
 * are admitted to one slot together and solved as a batch (mbl_solve_batch,
 * mbl_serve_batch_limit).  A request's arithmetic does not depend on its slot,
 * its batch or the other requests: its result is the same alone and in the
 * mix (bitwise, given the same device).  Requests whose footprint exceeds the
 * budget complete with MBL_ENOMEM. */
typedef struct {
    int slots;
    size_t budget_bytes;
    size_t held_bytes;          /* bytes the slots may hold now (largest admitted each) */
    int64_t submitted, admitted, completed;
    int64_t running, queued;    /* now */
    int64_t max_running;        /* largest number of requests on the device at once */
    int64_t bypasses;           /* admissions ahead of an earlier request */
    int64_t trims;              /* idle slots that gave their buffers back */
    int64_t retries;            /* requests run again after their slot gave back buffers
                                   kept from earlier requests to stay within its admission */
    size_t max_slot_peak;       /* largest device bytes one slot has held; a slot may hold
                                   no more than the footprint it was admitted with */
    int64_t batches;            /* admissions of two or more requests solved together */
    int64_t batched;            /* requests admitted in those */
} mbl_serve_info;

/* Start the server with `slots` (1..16; 0 = 4) slots and a budget (0 = the
 * context's budget).  Optional: mbl_submit starts it with the defaults.
 * MBL_EBUSY if it is already running. */
int mbl_serve_start(mbl_ctx *ctx, int slots, size_t budget_bytes);
/* Queued requests that mbl_solve_batch would batch (one L, the same J, nev,
 * precision, tolerance and Krylov settings) are admitted together, up to
 * max_batch (1..16; default 16; 1 = every request alone) per slot; a batch is
 * admitted with the footprints of all its requests.  Applies to the running
 * server, or to the next one started. */
int mbl_serve_batch_limit(mbl_ctx *ctx, int max_batch);
/* Queue one request; `prob` is copied, but prob->fields (if set), `res` and the
 * buffers it points to must stay valid until mbl_wait returns for the ticket.
 * Errors of the solve itself are reported by mbl_wait's status. */
int mbl_submit(mbl_ctx *ctx, const mbl_problem *prob, mbl_result *res, uint64_t *ticket);
/* done = 1 once the result is written. MBL_ENOTFOUND for unknown tickets. */
int mbl_poll(mbl_ctx *ctx, uint64_t ticket, int *done);
/* Block until the request completes; *status = its mbl status.  The ticket is
 * released. */
int mbl_wait(mbl_ctx *ctx, uint64_t ticket, int *status);
int mbl_serve_stats(mbl_ctx *ctx, mbl_serve_info *out);

#ifdef __cplusplus
}
#endif
#endif /* MBL_H */
