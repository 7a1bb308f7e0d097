// api.cpp -- the extern "C" boundary of libmbl: argument checks, error codes,
// host <-> device marshalling.  Every numerical step runs in the kernels
// behind mbl::Context.
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/mbl.h"
#include "common.hpp"
#include "kernels.hpp"
#include "serve.hpp"
#include "solver.hpp"

namespace mbl {
static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }
}  // namespace mbl

struct mbl_ctx {
    mbl::Context *c;
    mbl::Server *srv;
    std::mutex srv_mu;
    int max_batch = mbl::MBL_SEG_MAX;   // of the server (mbl_serve_batch_limit)
};

using namespace mbl;

namespace {

template <class F>
int guarded(F &&f) {
    try {
        f();
        return MBL_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return MBL_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return MBL_EDEVICE;
    }
}

void check_L(int L) {
    MBL_REQUIRE(L >= 2 && L <= MBL_L_MAX, MBL_EINVAL, "L must satisfy 2 <= L <= 22");
}

}  // namespace

extern "C" {

const char *mbl_strerror(int code) {
    switch (code) {
        case MBL_OK: return "ok";
        case MBL_EINVAL: return "invalid argument";
        case MBL_ENOMEM: return "out of device memory or above the context budget";
        case MBL_ENOTCONV: return "not all eigenpairs converged";
        case MBL_ENUMERIC: return "shifted solve failed to refine";
        case MBL_EDEVICE: return "HIP device error";
        case MBL_EBUSY: return "request queue full";
        case MBL_ENOTFOUND: return "unknown ticket";
        default: return "unknown status";
    }
}

const char *mbl_last_error(void) { return g_last_error.c_str(); }

void mbl_problem_init(mbl_problem *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->L = 12;
    p->J = 1.0;
    p->h = 1.0;
    p->eps = 0.5;
    p->sigma = NAN;
    p->nev = 20;
    p->prec = MBL_FP64;
    p->flags = MBL_WANT_OBS;
}

int mbl_create(int device, size_t hbm_budget_bytes, void *hip_stream, mbl_ctx **out) {
    if (!out) return MBL_EINVAL;
    *out = nullptr;
    return guarded([&] {
        int n = 0;
        MBL_HIP(hipGetDeviceCount(&n));
        MBL_REQUIRE(device >= 0 && device < n, MBL_EINVAL, "no such HIP device");
        mbl_ctx *c = new mbl_ctx;
        c->c = new Context(device, hbm_budget_bytes, static_cast<hipStream_t>(hip_stream));
        c->srv = nullptr;
        *out = c;
    });
}

int mbl_destroy(mbl_ctx *ctx) {
    if (!ctx) return MBL_EINVAL;
    return guarded([&] {
        if (ctx->srv) { delete ctx->srv; ctx->srv = nullptr; }
        (void)hipSetDevice(ctx->c->device);
        delete ctx->c;
        delete ctx;
    });
}

int64_t mbl_sector_dim(int L) {
    if (L < 2 || L > MBL_L_MAX) return -1;
    return binom(L, sector_nup(L));
}

int mbl_fields(int L, double h, uint64_t seed, double *out_host) {
    if (!out_host || L < 1 || L > 32) return MBL_EINVAL;
    uint64_t st = seed;
    for (int i = 0; i < L; i++) {
        uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        out_host[i] = h * (2.0 * u - 1.0);
    }
    return MBL_OK;
}

int mbl_basis(mbl_ctx *ctx, int L, uint32_t *out_host) {
    if (!ctx || !out_host) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        MBL_HIP(hipSetDevice(ctx->c->device));
        Plan &p = ctx->c->plan(L);
        d2h(out_host, p.basis.ptr<uint32_t>(), p.dim, ctx->c->stream);
        MBL_HIP(hipStreamSynchronize(ctx->c->stream));
    });
}

int mbl_rank(mbl_ctx *ctx, int L, const uint32_t *words_host, int64_t count, int64_t *ranks_host) {
    if (!ctx || (count > 0 && (!words_host || !ranks_host)) || count < 0) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        MBL_HIP(hipSetDevice(ctx->c->device));
        if (count == 0) return;
        DevBuf w, r;
        w.alloc(sizeof(uint32_t) * count, &ctx->c->budget);
        r.alloc(sizeof(int64_t) * count, &ctx->c->budget);
        h2d(w.ptr<uint32_t>(), words_host, count, ctx->c->stream);
        launch_rank(L, w.ptr<uint32_t>(), count, r.ptr<int64_t>(), ctx->c->stream);
        d2h(ranks_host, r.ptr<int64_t>(), count, ctx->c->stream);
        MBL_HIP(hipStreamSynchronize(ctx->c->stream));
    });
}

int mbl_hamiltonian(mbl_ctx *ctx, int L, double J, const double *fields_host, int32_t *rowptr_host,
                    int32_t *col_host, double *val_host, int64_t *nnz_out) {
    if (!ctx || !fields_host) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.set_realization(p, J, fields_host, 0.0, 0, false);
        if (nnz_out) *nnz_out = p.nnz;
        if (rowptr_host) std::memcpy(rowptr_host, p.h_rowptr.data(), sizeof(int32_t) * (p.dim + 1));
        if (col_host) std::memcpy(col_host, p.h_col.data(), sizeof(int32_t) * p.nnz);
        if (val_host) {
            std::vector<double> diag(p.dim);
            d2h(diag.data(), c.d_diag.ptr<double>(), p.dim, c.stream);
            MBL_HIP(hipStreamSynchronize(c.stream));
            for (int64_t k = 0; k < p.dim; k++)
                for (int32_t e = p.h_rowptr[k]; e < p.h_rowptr[k + 1]; e++)
                    val_host[e] = (p.h_col[e] == k) ? diag[k] : c.offv;
        }
    });
}

int mbl_spmv(mbl_ctx *ctx, int L, double J, const double *fields_host, int nvec,
             const double *x_host, double *y_host) {
    if (!ctx || !fields_host || !x_host || !y_host || nvec < 1) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.set_realization(p, J, fields_host, 0.0, 0, false);
        DevBuf x, y;
        x.alloc(sizeof(double) * p.dim * nvec, &c.budget);
        y.alloc(sizeof(double) * p.dim * nvec, &c.budget);
        h2d(x.ptr<double>(), x_host, p.dim * nvec, c.stream);
        c.spmv(p, 0.0, nvec, x.ptr<double>(), y.ptr<double>());
        d2h(y_host, y.ptr<double>(), p.dim * nvec, c.stream);
        MBL_HIP(hipStreamSynchronize(c.stream));
    });
}

int mbl_extremal(mbl_ctx *ctx, int L, double J, const double *fields_host, double *emin,
                 double *emax) {
    if (!ctx || !fields_host || !emin || !emax) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.set_realization(p, J, fields_host, 0.0, 0, false);
        int nap = 0;
        c.extremal(p, *emin, *emax, nap);
    });
}

int mbl_ritz_eig(mbl_ctx *ctx, int count, int m, const double *A_host, double *w_host,
                 double *Z_host, int flags) {
    if (!ctx || count < 0 || m < 1 || m > 1024 || (flags & ~MBL_EIG_GENERAL)) return MBL_EINVAL;
    if (count > 0 && (!A_host || !w_host || !Z_host)) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        if (count == 0) return;
        const size_t mm = (size_t)m * m;
        std::vector<std::vector<double>> A(count), w, Z;
        for (int k = 0; k < count; k++) A[k].assign(A_host + mm * k, A_host + mm * (k + 1));
        c.small_eig_batch(count, m, A, w, Z, (flags & MBL_EIG_GENERAL) != 0);
        for (int k = 0; k < count; k++) {
            std::copy(w[k].begin(), w[k].end(), w_host + (size_t)m * k);
            std::copy(Z[k].begin(), Z[k].end(), Z_host + mm * k);
        }
    });
}

int mbl_symbolic(mbl_ctx *ctx, int L, mbl_symbolic_info *info) {
    if (!ctx) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.ensure_symbolic(p);
        if (info) {
            const FrontTree &t = p.tree;
            info->dim = p.dim;
            info->nnz_h = p.nnz;
            info->n_fronts = (int64_t)t.fronts.size();
            info->n_levels = t.n_levels;
            info->max_front = t.max_m;
            info->max_pivots = t.max_p;
            info->nnz_factor = t.nnz_factor;
            info->front_entries = t.front_entries;
            info->flops_factor = t.flops;
            info->seconds = t.seconds;
        }
    });
}

int mbl_ordering(mbl_ctx *ctx, int L, int32_t *perm_host) {
    if (!ctx || !perm_host) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.ensure_symbolic(p);
        std::memcpy(perm_host, p.tree.perm.data(), sizeof(int32_t) * p.dim);
    });
}

int mbl_front_tree(mbl_ctx *ctx, int L, int32_t *first, int32_t *npiv, int32_t *ncontrib,
                   int32_t *parent, int64_t *cptr, int32_t *contrib, int64_t *n_fronts,
                   int64_t *n_contrib) {
    if (!ctx) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.ensure_symbolic(p);
        const FrontTree &t = p.tree;
        if (n_fronts) *n_fronts = (int64_t)t.fronts.size();
        if (n_contrib) *n_contrib = (int64_t)t.contrib.size();
        for (size_t f = 0; f < t.fronts.size(); f++) {
            const Front &F = t.fronts[f];
            if (first) first[f] = F.first;
            if (npiv) npiv[f] = F.p;
            if (ncontrib) ncontrib[f] = F.c;
            if (parent) parent[f] = F.parent;
            if (cptr) cptr[f] = F.cptr;
        }
        if (contrib) std::memcpy(contrib, t.contrib.data(), sizeof(int32_t) * t.contrib.size());
    });
}

int mbl_shift_solve(mbl_ctx *ctx, int L, double J, const double *fields_host, double sigma,
                    int prec, int nrhs, const double *b_host, double *x_host,
                    mbl_solve_info *info) {
    if (!ctx || !fields_host || !b_host || !x_host || nrhs < 1 || !std::isfinite(sigma))
        return MBL_EINVAL;
    if (prec != MBL_FP64 && prec != MBL_FP32_IR64) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.set_realization(p, J, fields_host, 0.0, 0, false);
        // ||H - sigma|| bound from the Gershgorin discs of H
        std::vector<double> diag(p.dim);
        d2h(diag.data(), c.d_diag.ptr<double>(), p.dim, c.stream);
        MBL_HIP(hipStreamSynchronize(c.stream));
        double g = 0.0;
        for (int64_t k = 0; k < p.dim; k++) {
            double r = std::fabs(diag[k] - sigma) +
                       std::fabs(c.offv) * (double)(p.h_rowptr[k + 1] - p.h_rowptr[k] - 1);
            g = std::max(g, r);
        }
        SolveStats st;
        c.factor(p, prec, sigma, g > 0 ? g : 1.0, st);
        DevBuf b, x;
        b.alloc(sizeof(double) * p.dim * nrhs, &c.budget);
        x.alloc(sizeof(double) * p.dim * nrhs, &c.budget);
        h2d(b.ptr<double>(), b_host, p.dim * nrhs, c.stream);
        c.shift_solve(p, prec, nrhs, b.ptr<double>(), x.ptr<double>(), st);
        d2h(x_host, x.ptr<double>(), p.dim * nrhs, c.stream);
        MBL_HIP(hipStreamSynchronize(c.stream));
        if (info) {
            info->ir_iters = st.ir_iters;
            info->n_perturbed = st.n_perturbed;
            info->backward_error = st.backward_error;
            info->t_factor = st.t_factor;
            info->t_solve = st.t_solve;
        }
    });
}

static int observables_impl(mbl_ctx *ctx, int L, int nev, const double *evals_host,
                            const double *evecs_host, double *r_host, double *s1_host,
                            double *se_host, double *s2_host, double *fl_host, double *df_host,
                            double *kl_host) {
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        int64_t n = p.dim;
        MBL_REQUIRE(nev >= 1 && nev <= 4096, MBL_EINVAL, "nev out of range");
        DevBuf psi, e, q, r, se;
        psi.alloc(sizeof(double) * n * nev, &c.budget);
        h2d(psi.ptr<double>(), evecs_host, n * nev, c.stream);
        c.obs.prepare(L, p.basis.ptr<uint32_t>(), n, nev, &c.budget, c.stream);
        q.alloc(sizeof(double) * OBS_NQ * nev, &c.budget);
        c.obs.vector_sums(p.basis.ptr<uint32_t>(), psi.ptr<double>(), n, nev, q.ptr<double>(),
                          c.stream);
        std::vector<double> qh((size_t)OBS_NQ * nev);
        if (r_host && evals_host && nev >= 3) {
            e.alloc(sizeof(double) * nev, &c.budget);
            r.alloc(sizeof(double) * nev, &c.budget);
            h2d(e.ptr<double>(), evals_host, nev, c.stream);
            c.obs.gap_ratios(nev, e.ptr<double>(), r.ptr<double>(), c.stream);
            d2h(r_host, r.ptr<double>(), nev - 2, c.stream);
        }
        if (se_host) {
            se.alloc(sizeof(double) * nev, &c.budget);
            c.obs.entanglement(psi.ptr<double>(), n, nev, c.obs.norms_dev(), se.ptr<double>(),
                               c.stream);
            d2h(se_host, se.ptr<double>(), nev, c.stream);
        }
        d2h(qh.data(), q.ptr<double>(), qh.size(), c.stream);
        MBL_HIP(hipStreamSynchronize(c.stream));
        if (se_host)
            for (int j = 0; j < nev; j++)
                if (!std::isfinite(se_host[j]))
                    throw Error(MBL_ENUMERIC, "entanglement: non-finite result");
        for (int j = 0; j < nev; j++) {
            const double *v = &qh[(size_t)j * OBS_NQ];
            if (s1_host) s1_host[j] = v[1];
            if (s2_host) s2_host[j] = -std::log(v[2]);
            if (fl_host) fl_host[j] = v[4] - v[3] * v[3];
            if (df_host) df_host[j] = 1.0 - (v[5] * v[5] + v[6] * v[6]) / v[7];
            if (kl_host && j + 1 < nev) kl_host[j] = v[8];
        }
    });
}

int mbl_observables_noalloc(int L, int nev, const double *evals_dev, const double *evecs_dev,
                            int64_t ld, double *r_dev, double *s1_dev, double *se_dev,
                            void *hip_stream) {
    return guarded([&] {
        observables_noalloc(L, nev, evals_dev, evecs_dev, ld, r_dev, s1_dev, se_dev,
                            static_cast<hipStream_t>(hip_stream));
    });
}

int mbl_observables(mbl_ctx *ctx, int L, int nev, const double *evals_host,
                    const double *evecs_host, double *r_host, double *s1_host, double *se_host) {
    if (!ctx || !evecs_host) return MBL_EINVAL;
    return observables_impl(ctx, L, nev, evals_host, evecs_host, r_host, s1_host, se_host, nullptr,
                            nullptr, nullptr, nullptr);
}

int mbl_observables_extra(mbl_ctx *ctx, int L, int nev, const double *evecs_host, double *s2_host,
                          double *fluct_host, double *dynfrac_host, double *kl_host) {
    if (!ctx || !evecs_host) return MBL_EINVAL;
    return observables_impl(ctx, L, nev, nullptr, evecs_host, nullptr, nullptr, nullptr, s2_host,
                            fluct_host, dynfrac_host, kl_host);
}

int mbl_solve(mbl_ctx *ctx, const mbl_problem *prob, mbl_result *res) {
    if (!ctx || !prob || !res) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        MBL_HIP(hipSetDevice(ctx->c->device));
        solve_problem(*ctx->c, *prob, *res);
    });
}

int mbl_solve_batch(mbl_ctx *ctx, int count, const mbl_problem *probs, mbl_result *results,
                    int *status) {
    if (!ctx || !probs || !results || !status || count < 1 || count > MBL_SEG_MAX)
        return MBL_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
    for (int k = 0; k < count; k++) status[k] = MBL_EBUSY;
    bool done = false;
    int rc = guarded([&] {
        MBL_HIP(hipSetDevice(ctx->c->device));
        done = solve_batch(*ctx->c, count, probs, results, status);
    });
    if (rc == MBL_EDEVICE) {
        for (int k = 0; k < count; k++) status[k] = rc;
        return rc;
    }
    // any other failure of the batch as a whole (an invalid problem, extremal
    // energies of one problem not converging): each problem gets the status
    // of its lone solve
    if (rc != MBL_OK) done = false;
    if (!done)
        for (int k = 0; k < count; k++)
            status[k] = guarded([&] {
                MBL_HIP(hipSetDevice(ctx->c->device));
                solve_problem(*ctx->c, probs[k], results[k]);
            });
    for (int k = 0; k < count; k++)
        if (status[k] != MBL_OK) return status[k];
    return MBL_OK;
}

namespace {
// One realization's bin for one target: averages over its nev eigenstates
// (the per-sample binning of the "Numerical method" section).
void realization_bins(const mbl_result &r, int nev, const std::vector<double> &E,
                      const std::vector<double> &rv, const std::vector<double> &s1,
                      const std::vector<double> &s2, const std::vector<double> &se,
                      const std::vector<double> &fl, const std::vector<double> &df,
                      const std::vector<double> &kl, double *bin) {
    auto mean = [](const std::vector<double> &v, size_t count) {
        double sum = 0.0;
        size_t k = 0;
        for (size_t j = 0; j < count; j++)
            if (std::isfinite(v[j])) { sum += v[j]; k++; }
        return k ? sum / (double)k : NAN;
    };
    const size_t n = (size_t)nev;
    bin[MBL_BIN_R] = nev >= 3 ? mean(rv, n - 2) : NAN;
    bin[MBL_BIN_S1] = mean(s1, n);
    bin[MBL_BIN_S2] = mean(s2, n);
    bin[MBL_BIN_SE] = mean(se, n);
    double q = 0.0;
    for (size_t j = 0; j < n; j++) q += se[j] * se[j];
    bin[MBL_BIN_SE2] = q / (double)n;
    bin[MBL_BIN_FLUCT] = mean(fl, n);
    bin[MBL_BIN_DYNFRAC] = mean(df, n);
    bin[MBL_BIN_KL] = nev >= 2 ? mean(kl, n - 1) : NAN;
    double w = r.emax - r.emin, ed = 0.0;
    for (size_t j = 0; j < n; j++) ed += w > 0 ? (E[j] - r.emin) / w : 0.0;
    bin[MBL_BIN_EDENS] = ed / (double)n;
    bin[MBL_BIN_NCONV] = (double)r.nconv;
}
}  // namespace

int mbl_sweep(mbl_ctx *ctx, const mbl_problem *base, const double *eps, int n_eps,
              double *bins, int *status) {
    if (!ctx || !base || !eps || !bins || !status || n_eps < 1) return MBL_EINVAL;
    for (int k = 0; k < n_eps; k++)
        if (!(eps[k] >= 0.0 && eps[k] <= 1.0)) return MBL_EINVAL;
    for (int k = 0; k < n_eps; k++) status[k] = MBL_EBUSY;   // not reached yet
    for (int k = 0; k < n_eps * MBL_NBIN; k++) bins[k] = NAN;
    const int nev = base->nev;
    if (nev < 1 || nev > 256) return MBL_EINVAL;
    std::vector<double> E(nev), rv(std::max(1, nev - 2)), s1(nev), s2(nev), se(nev), fl(nev),
        df(nev), kl(std::max(1, nev - 1)), rs(nev);
    double ext[2] = {0.0, 0.0};
    bool have_ext = false;
    int first_err = MBL_OK;
    for (int k = 0; k < n_eps; k++) {
        mbl_problem pr = *base;
        pr.eps = eps[k];
        pr.sigma = NAN;
        pr.flags = (base->flags | MBL_WANT_OBS | MBL_WANT_OBS_EXTRA) & ~MBL_WANT_VECTORS;
        mbl_result res;
        std::memset(&res, 0, sizeof res);
        res.evals = E.data(); res.resid = rs.data(); res.r = rv.data(); res.s1 = s1.data();
        res.se = se.data(); res.s2 = s2.data(); res.fluct = fl.data(); res.dynfrac = df.data();
        res.kl = kl.data();
        int code = guarded([&] {
            std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
            MBL_HIP(hipSetDevice(ctx->c->device));
            solve_problem(*ctx->c, pr, res, have_ext ? ext : nullptr);
        });
        status[k] = code;
        if (code == MBL_OK || code == MBL_ENOTCONV) {
            if (!have_ext) { ext[0] = res.emin; ext[1] = res.emax; have_ext = true; }
            realization_bins(res, nev, E, rv, s1, s2, se, fl, df, kl, bins + (size_t)k * MBL_NBIN);
        }
        if (code != MBL_OK && first_err == MBL_OK) first_err = code;
        if (code != MBL_OK && code != MBL_ENOTCONV && code != MBL_ENUMERIC) return code;
    }
    return first_err;
}

int mbl_disorder_average(const double *bins, int n_real, double *mean, double *sem,
                         double *sigma_e) {
    if (!bins || n_real < 1 || !mean || !sem) return MBL_EINVAL;
    for (int q = 0; q < MBL_NBIN; q++) {
        double sum = 0.0;
        int k = 0;
        for (int i = 0; i < n_real; i++) {
            double b = bins[(size_t)i * MBL_NBIN + q];
            if (std::isfinite(b)) { sum += b; k++; }
        }
        double m = k ? sum / k : NAN, ss = 0.0;
        for (int i = 0; i < n_real; i++) {
            double b = bins[(size_t)i * MBL_NBIN + q];
            if (std::isfinite(b)) ss += (b - m) * (b - m);
        }
        mean[q] = m;
        sem[q] = k >= 2 ? std::sqrt(ss / ((double)k * (k - 1))) : NAN;
    }
    if (sigma_e) {
        double v = mean[MBL_BIN_SE2] - mean[MBL_BIN_SE] * mean[MBL_BIN_SE];
        *sigma_e = std::sqrt(std::max(0.0, v));
    }
    return MBL_OK;
}

int mbl_footprint(mbl_ctx *ctx, int L, int prec, int nev, int block, size_t *bytes) {
    if (!ctx || !bytes) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        check_L(L);
        Context &c = *ctx->c;
        MBL_HIP(hipSetDevice(c.device));
        Plan &p = c.plan(L);
        c.ensure_symbolic(p);
        *bytes = footprint_bytes(p, prec, nev, block);
    });
}

int mbl_profile_enable(mbl_ctx *ctx, const char *kernel_class) {
    if (!ctx) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        Context &c = *ctx->c;
        c.prof_collect();
        c.prof.cls = kernel_class ? kernel_class : "";
        c.prof.launches = 0;
        c.prof.bytes = c.prof.flops = c.prof.seconds = 0.0;
    });
}

int mbl_profile_read(mbl_ctx *ctx, mbl_kernel_profile *out) {
    if (!ctx || !out) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::recursive_mutex> lk(ctx->c->mu);
        Context &c = *ctx->c;
        c.prof_collect();
        out->launches = c.prof.launches;
        out->seconds = c.prof.seconds;
        out->bytes = c.prof.bytes;
        out->flops = c.prof.flops;
    });
}

int mbl_serve_start(mbl_ctx *ctx, int slots, size_t budget_bytes) {
    if (!ctx || slots < 0 || slots > 16) return MBL_EINVAL;
    return guarded([&] {
        std::lock_guard<std::mutex> lk(ctx->srv_mu);
        MBL_REQUIRE(!ctx->srv, MBL_EBUSY, "server already running");
        MBL_HIP(hipSetDevice(ctx->c->device));
        ctx->srv = new Server(ctx->c, slots ? slots : 4,
                              budget_bytes ? budget_bytes : ctx->c->budget.limit, ctx->max_batch);
    });
}

int mbl_serve_batch_limit(mbl_ctx *ctx, int max_batch) {
    if (!ctx || max_batch < 1 || max_batch > MBL_SEG_MAX) return MBL_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->srv_mu);
    ctx->max_batch = max_batch;
    if (ctx->srv) ctx->srv->set_max_batch(max_batch);
    return MBL_OK;
}

int mbl_submit(mbl_ctx *ctx, const mbl_problem *prob, mbl_result *res, uint64_t *ticket) {
    if (!ctx || !prob || !res || !ticket) return MBL_EINVAL;
    return guarded([&] {
        {
            std::lock_guard<std::mutex> lk(ctx->srv_mu);
            if (!ctx->srv) {
                MBL_HIP(hipSetDevice(ctx->c->device));
                ctx->srv = new Server(ctx->c, 4, ctx->c->budget.limit, ctx->max_batch);
            }
        }
        *ticket = ctx->srv->submit(*prob, res);
    });
}

int mbl_serve_stats(mbl_ctx *ctx, mbl_serve_info *out) {
    if (!ctx || !out) return MBL_EINVAL;
    if (!ctx->srv) return MBL_ENOTFOUND;
    return guarded([&] { ctx->srv->info(out); });
}

int mbl_poll(mbl_ctx *ctx, uint64_t ticket, int *done) {
    if (!ctx || !done) return MBL_EINVAL;
    if (!ctx->srv) return MBL_ENOTFOUND;
    return ctx->srv->poll(ticket, done);
}

int mbl_wait(mbl_ctx *ctx, uint64_t ticket, int *status) {
    if (!ctx) return MBL_EINVAL;
    if (!ctx->srv) return MBL_ENOTFOUND;
    return ctx->srv->wait(ticket, status);
}

}  // extern "C"
