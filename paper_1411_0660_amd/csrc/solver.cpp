// solver.cpp -- plans, multifrontal factor/solve drivers with FP64 iterative
// refinement, block Krylov-Schur, and the whole shift-invert solve of one
// (L, h, seed, eps) problem (section "Numerical method").
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "kernels.hpp"
#include "smalleig.hpp"

namespace mbl {

int debug_level() {
    static int lvl = [] {
        const char *e = std::getenv("MBL_DEBUG");
        return e ? std::atoi(e) : 0;
    }();
    return lvl;
}

double wall_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

namespace {
constexpr int MAXRHS = 16;       // right-hand sides per pass through the factors
constexpr int RES_PARTS = 256;   // blocks of the residual reduction

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Builder of TaskLists: offsets first, device pointers once uploaded.
struct TaskBuilder {
    std::vector<int32_t> fr;
    std::vector<int64_t> pre;
    std::vector<int2> its;
    std::vector<TaskList *> lists;
    struct Offs { int64_t fr, pre, its; };
    std::vector<Offs> offs;
    void add(TaskList &tl, const std::vector<int32_t> &fronts, const std::vector<int64_t> &items) {
        tl.n = (int32_t)fronts.size();
        Offs o{(int64_t)fr.size(), (int64_t)pre.size(), (int64_t)its.size()};
        int64_t acc = 0;
        fr.insert(fr.end(), fronts.begin(), fronts.end());
        for (size_t k = 0; k < items.size(); k++) {
            pre.push_back(acc);
            acc += items[k];
            MBL_REQUIRE(items[k] < INT32_MAX, MBL_EINVAL, "task list: too many items per front");
            for (int64_t j = 0; j < items[k]; j++) its.push_back(make_int2(fronts[k], (int)j));
        }
        pre.push_back(acc);
        if (fronts.empty()) fr.push_back(0);    // keep pointers valid
        tl.total = acc;
        lists.push_back(&tl);
        offs.push_back(o);
    }
};
}  // namespace

Context::Context(int dev, size_t budget_bytes, hipStream_t s)
    : device(dev), plans_(std::make_shared<PlanCache>()) {
    MBL_HIP(hipSetDevice(dev));
    if (s) { stream = s; own_stream = false; }
    else { MBL_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)); own_stream = true; }
    size_t fr = 0, tot = 0;
    MBL_HIP(hipMemGetInfo(&fr, &tot));
    budget.limit = budget_bytes ? budget_bytes : (size_t)(0.92 * (double)fr);
    use_graphs_ = std::getenv("MBL_NO_GRAPH") == nullptr;
}

Context::Context(const Context &owner, size_t budget_bytes)
    : device(owner.device), plans_(owner.plans_), owns_plans_(false) {
    MBL_HIP(hipSetDevice(device));
    MBL_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    own_stream = true;
    budget.limit = budget_bytes;
    use_graphs_ = std::getenv("MBL_NO_GRAPH") == nullptr;
}

void Context::trim() {
    MBL_HIP(hipStreamSynchronize(stream));
    clear_graphs();
    for (DevBuf *b : {&f32_.arena, &f32_.ipiv, &f32_.prow, &f32_.npert, &f64_.arena, &f64_.ipiv,
                      &f64_.prow, &f64_.npert, &d_vec, &d_yv, &d_upart, &d_xnew, &d_r, &d_d,
                      &d_part, &d_V, &d_V2, &d_W, &d_small, &d_ritz, &d_tnpart, &d_stage, &d_gV, &d_gZ, &d_gpart,
                      &d_gcoef, &d_psi, &d_psi2, &d_hpsi, &d_e, &d_cpart, &d_obs, &d_r_out,
                      &d_se})
        b->reset();
    for (DevBuf *b : {&f32_.uinv, &f64_.uinv, &f32_.thr, &f64_.thr, &fb64_.arena, &fb64_.ipiv,
                      &fb64_.prow, &fb64_.npert, &fb64_.uinv, &fb64_.thr, &fb32_.arena,
                      &fb32_.ipiv, &fb32_.prow, &fb32_.npert, &fb32_.uinv, &fb32_.thr, &d_on,
                      &d_bdiag, &d_bshift})
        b->reset();
    obs.release();
    fb64_.valid = false;
    fb64_.L = -1;
    fb32_.valid = false;
    fb32_.L = -1;
    f32_.valid = false;
    f64_.valid = false;
    f32_.L = -1;                       // buffers freed: the next factorization reallocates
    f64_.L = -1;
}

Context::~Context() {
    (void)hipStreamSynchronize(stream);
    clear_graphs();
    for (auto &e : prof.pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    if (owns_plans_) {
        std::lock_guard<std::recursive_mutex> lk(plans_->mu);
        plans_->batched.clear();
        plans_->plans.clear();
    }
    if (own_stream) (void)hipStreamDestroy(stream);
}

void Context::prof_begin() {
    if (prof.used == prof.pool.size()) {
        hipEvent_t a, b;
        MBL_HIP(hipEventCreate(&a));
        MBL_HIP(hipEventCreate(&b));
        prof.pool.push_back({a, b});
    }
    MBL_HIP(hipEventRecord(prof.pool[prof.used].first, stream));
}

void Context::prof_end(double bytes, double flops) {
    MBL_HIP(hipEventRecord(prof.pool[prof.used].second, stream));
    prof.used++;
    prof.launches++;
    prof.bytes += bytes;
    prof.flops += flops;
    if (prof.used >= 4096) prof_collect();
}

void Context::prof_collect() {
    if (prof.used == 0) return;
    MBL_HIP(hipStreamSynchronize(stream));
    for (size_t i = 0; i < prof.used; i++) {
        float ms = 0.0f;
        MBL_HIP(hipEventElapsedTime(&ms, prof.pool[i].first, prof.pool[i].second));
        prof.seconds += 1e-3 * (double)ms;
    }
    prof.used = 0;
}

Plan &Context::plan(int L) {
    std::lock_guard<std::recursive_mutex> lk(plans_->mu);
    auto it = plans_->plans.find(L);
    if (it != plans_->plans.end()) return *it->second;
    MBL_REQUIRE(owns_plans_, MBL_EINVAL, "plan for this L not prepared by the owning context");
    std::unique_ptr<Plan> p(new Plan);
    p->L = L;
    p->dim = binom(L, sector_nup(L));
    int64_t n = p->dim;
    p->basis.alloc(sizeof(uint32_t) * n, &budget);
    launch_basis(L, n, p->basis.ptr<uint32_t>(), stream);
    DevBuf scratch;
    scratch.alloc(scan_scratch_bytes(n), &budget);
    p->rowptr.alloc(sizeof(int32_t) * (n + 1), &budget);
    launch_row_ptr(L, n, p->basis.ptr<uint32_t>(), p->rowptr.ptr<int32_t>(), scratch.ptr<void>(),
                   stream);
    p->h_rowptr.resize(n + 1);
    d2h(p->h_rowptr.data(), p->rowptr.ptr<int32_t>(), n + 1, stream);
    MBL_HIP(hipStreamSynchronize(stream));
    p->nnz = p->h_rowptr[n];
    p->col.alloc(sizeof(int32_t) * p->nnz, &budget);
    launch_fill_csr(L, n, p->basis.ptr<uint32_t>(), p->rowptr.ptr<int32_t>(), p->col.ptr<int32_t>(),
                    stream);
    p->h_col.resize(p->nnz);
    d2h(p->h_col.data(), p->col.ptr<int32_t>(), p->nnz, stream);
    MBL_HIP(hipStreamSynchronize(stream));
    Plan &ref = *p;
    plans_->plans[L] = std::move(p);
    return ref;
}

void Context::ensure_symbolic(Plan &p) {
    std::lock_guard<std::recursive_mutex> lk(plans_->mu);
    if (p.have_symbolic) return;
    MBL_REQUIRE(owns_plans_, MBL_EINVAL, "symbolic analysis not prepared by the owning context");
    Pattern A;
    A.n = p.dim;
    A.rowptr = p.h_rowptr;
    A.col = p.h_col;
    NdOptions opt;
    p.tree = build_front_tree(A, opt);
    build_tables(p);
}

// Device tables of a plan from its front tree and CSR pattern: front
// descriptors, the maps of the extend-add and of the solves, the original
// entries of every front, and the per-level task lists.  A batch plan's tree
// is nseg copies of one tree, so every launch covers all its problems.
void Context::build_tables(Plan &p) {
    FrontTree &t = p.tree;
    int nf = (int)t.fronts.size();
    const int nf1 = nf / std::max(1, p.nseg);         // fronts per problem
    MBL_REQUIRE(t.max_m < 46340, MBL_EINVAL, "front too large for 32-bit local positions");
    MBL_REQUIRE((int64_t)t.contrib.size() < INT32_MAX, MBL_EINVAL, "contribution lists too long");

    // fronts by level
    std::vector<std::vector<int32_t>> bylev(t.n_levels);
    for (int f = 0; f < nf; f++) bylev[t.fronts[f].level].push_back(f);
    p.h_fd.assign(nf, FrontDesc{});
    std::vector<int32_t> child_ids, relmap;
    int64_t off = 0, voff = 0;
    p.levels.assign(t.n_levels, LevelTasks{});
    std::vector<int32_t> efront, epos, esrc;
    std::vector<int32_t> mp;
    for (int l = 0; l < t.n_levels; l++) {
        LevelTasks &lv = p.levels[l];
        lv.ebegin = (int64_t)efront.size();
        int64_t poff = 0;
        for (int f : bylev[l]) {
            const Front &F = t.fronts[f];
            FrontDesc &d = p.h_fd[f];
            d.off = off;
            d.voff = voff;
            d.m = F.m();
            d.p = F.p;
            d.first = F.first;
            d.cptr = (int32_t)F.cptr;
            d.parent = F.parent;
            d.child0 = (int32_t)child_ids.size();
            d.nchild = (int32_t)F.children.size();
            d.seg = nf1 > 0 ? f / nf1 : 0;
            for (int c : F.children) child_ids.push_back(c);
            off += (int64_t)d.m * d.m;
            voff += (int64_t)d.m * MAXRHS;
            d.poff = poff;
            poff += std::max(cdiv64(d.m - d.p, SB) * (int64_t)d.p,    // U12 (backward) or
                             cdiv64(d.p, SB) * (int64_t)(d.m - d.p))    // L21 (forward) partials
                    * MAXRHS;
            d.yoff = p.y_elems;
            p.y_elems += (int64_t)d.p * MAXRHS;
            // original entries of H - sigma owned by this front
            const int32_t *cr = t.contrib.data() + F.cptr;
            auto local = [&](int32_t i) -> int32_t {
                if (i < F.first + F.p) return i - F.first;
                return F.p + (int32_t)(std::lower_bound(cr, cr + F.c, i) - cr);
            };
            for (int32_t j = F.first; j < F.first + F.p; j++) {
                int32_t old = t.perm[j];
                int32_t lj = j - F.first;
                for (int32_t e = p.h_rowptr[old]; e < p.h_rowptr[old + 1]; e++) {
                    int32_t i = t.iperm[p.h_col[e]];
                    if (i < F.first) continue;
                    int32_t li = local(i);
                    efront.push_back(f);
                    epos.push_back(li + lj * d.m);
                    esrc.push_back(i == j ? old : -1);
                    if (li >= F.p) {
                        efront.push_back(f);
                        epos.push_back(lj + li * d.m);
                        esrc.push_back(-1);
                    }
                }
            }
        }
        lv.ecount = (int64_t)efront.size() - lv.ebegin;
        lv.part_elems = poff;
        p.part_elems = std::max(p.part_elems, poff);
    }
    for (int f = 0; f < nf; f++) {
        if (t.fronts[f].parent < 0) { p.h_fd[f].mapoff = -1; continue; }
        child_relative_map(t, f, mp);
        p.h_fd[f].mapoff = (int32_t)relmap.size();
        relmap.insert(relmap.end(), mp.begin(), mp.end());
    }
    // pull maps: for every front with children, per child and front row, the
    // child's update row that lands on that row (or -1)
    std::vector<int32_t> pullmap;
    for (int f = 0; f < nf; f++) {
        FrontDesc &d = p.h_fd[f];
        MBL_REQUIRE(d.nchild <= PULL_MAXCH, MBL_EINVAL, "front with too many children");
        d.pmoff = (int32_t)pullmap.size();
        pullmap.resize(pullmap.size() + (size_t)d.nchild * d.m, -1);
        for (int q = 0; q < d.nchild; q++) {
            const FrontDesc &cd = p.h_fd[child_ids[d.child0 + q]];
            int32_t *pm = pullmap.data() + d.pmoff + (int64_t)q * d.m;
            for (int32_t k = 0; k < cd.m - cd.p; k++) {
                const int32_t r = relmap[cd.mapoff + k];
                MBL_REQUIRE(r >= 0 && r < d.m, MBL_EINVAL, "relative map entry outside the parent front");
                pm[r] = k;
            }
        }
        MBL_REQUIRE(pullmap.size() < (size_t)INT32_MAX, MBL_EINVAL, "pull maps too long");
    }
    p.arena_elems = off;
    p.vec_elems = voff;
    // inverse relative map: for every front row, the (child, child row) pairs
    // whose update lands on it
    std::vector<int32_t> inv_ptr;
    std::vector<int32_t> inv_src;   // pairs (element of the child's update row in the solve
                                    // vectors, the child's order = stride between right-hand sides)
    MBL_REQUIRE(p.vec_elems < (int64_t)INT32_MAX, MBL_EINVAL, "solve vectors too long");
    {
        std::vector<std::vector<std::pair<int32_t, int32_t>>> rows;
        for (int f = 0; f < nf; f++) {
            FrontDesc &d = p.h_fd[f];
            rows.assign(d.m, {});
            for (int q = 0; q < d.nchild; q++) {
                int c = child_ids[d.child0 + q];
                const FrontDesc &cd = p.h_fd[c];
                for (int32_t k = 0; k < cd.m - cd.p; k++) rows[relmap[cd.mapoff + k]].push_back({c, k});
            }
            d.cptr_inv = (int32_t)inv_ptr.size();
            int32_t acc = (int32_t)(inv_src.size() / 2);
            for (int32_t i = 0; i < d.m; i++) {
                inv_ptr.push_back(acc);
                for (auto &pr : rows[i]) {
                    const FrontDesc &cd = p.h_fd[pr.first];
                    inv_src.push_back((int32_t)(cd.voff + cd.p + pr.second));
                    inv_src.push_back(cd.m);
                    acc++;
                }
            }
            inv_ptr.push_back(acc);
            MBL_REQUIRE(inv_ptr.size() < (size_t)INT32_MAX, MBL_EINVAL, "inverse map too long");
        }
    }
    // bounds of every index the kernels will follow
    {
        std::vector<char> seen(p.dim, 0);
        for (int32_t v : t.perm) {
            MBL_REQUIRE(v >= 0 && v < p.dim && !seen[v], MBL_EINVAL, "ordering is not a permutation");
            seen[v] = 1;
        }
        for (int f = 0; f < nf; f++) {
            const FrontDesc &d = p.h_fd[f];
            MBL_REQUIRE(d.p >= 0 && d.m >= d.p && d.first >= 0 && d.first + d.p <= p.dim,
                        MBL_EINVAL, "front descriptor out of range");
            for (int32_t k = 0; k < d.m - d.p; k++) {
                int32_t x = t.contrib[d.cptr + k];
                MBL_REQUIRE(x >= d.first + d.p && x < p.dim, MBL_EINVAL, "contribution row out of range");
            }
            if (d.parent >= 0) {
                const FrontDesc &P = p.h_fd[d.parent];
                MBL_REQUIRE(d.mapoff >= 0 && d.mapoff + (d.m - d.p) <= (int64_t)relmap.size(),
                            MBL_EINVAL, "relative map out of range");
                for (int32_t k = 0; k < d.m - d.p; k++)
                    MBL_REQUIRE(relmap[d.mapoff + k] >= 0 && relmap[d.mapoff + k] < P.m, MBL_EINVAL,
                                "relative map entry outside the parent front");
            }
        }
        for (size_t e = 0; e < efront.size(); e++) {
            const FrontDesc &d = p.h_fd[efront[e]];
            MBL_REQUIRE(epos[e] >= 0 && (int64_t)epos[e] < (int64_t)d.m * d.m && esrc[e] < p.dim,
                        MBL_EINVAL, "original entry outside its front");
        }
    }

    TaskBuilder tb;
    {
        std::vector<int32_t> all;
        std::vector<int64_t> nb;
        for (int f = 0; f < nf; f++)
            if (p.h_fd[f].p > 0) { all.push_back(f); nb.push_back(cdiv64(p.h_fd[f].p, SB)); }
        tb.add(p.inv, all, nb);
        std::vector<int64_t> xi;
        for (int f : all) xi.push_back(xform_items(p.h_fd[f].m, p.h_fd[f].p));
        tb.add(p.xform, all, xi);
        // merging factorization blocks 2t, 2t + 1 into solve block t
        int maxpairs = 0;
        for (int f : all) maxpairs = std::max<int>(maxpairs, (int)cdiv64(p.h_fd[f].p, SSB));
        p.fold_lo.assign(maxpairs, TaskList{});
        p.fold_up.assign(maxpairs, TaskList{});
        for (int tp = 0; tp < maxpairs; tp++) {
            std::vector<int32_t> flo, fup;
            std::vector<int64_t> nlo, nup;
            for (int f : all) {
                const FrontDesc &d = p.h_fd[f];
                int a = tp * SSB, e = std::min(d.p, a + SSB);
                if (e <= a + SB) continue;           // no second block to merge
                if (d.m > e) { flo.push_back(f); nlo.push_back(cdiv64(d.m - e, SCHUR_TILE) * cdiv64(SB, SCHUR_TILE)); }
                if (a > 0) { fup.push_back(f); nup.push_back(cdiv64(a, SCHUR_TILE) * cdiv64(e - a - SB, SCHUR_TILE)); }
            }
            tb.add(p.fold_lo[tp], flo, nlo);
            tb.add(p.fold_up[tp], fup, nup);
        }
        std::vector<int32_t> mf;
        std::vector<int64_t> mi;
        for (int f : all)
            if (p.h_fd[f].p > SB) { mf.push_back(f); mi.push_back(merge_tri_items(p.h_fd[f].p)); }
        tb.add(p.merge, mf, mi);
    }
    for (int l = 0; l < t.n_levels; l++) {
        LevelTasks &lv = p.levels[l];
        const std::vector<int32_t> &fl = bylev[l];
        std::vector<int64_t> one(fl.size(), 1);
        std::vector<int32_t> ut, ur, lt, lr;
        std::vector<int64_t> uti, uri, lti, lri;
        int maxsteps = 0, maxsb = 0;
        for (int f : fl) {
            const FrontDesc &d = p.h_fd[f];
            if (d.p > 0) {
                ur.push_back(f);
                uri.push_back(cdiv64(d.p, 256));
                if (d.m > d.p) { ut.push_back(f); uti.push_back(cdiv64(d.p, 64) * cdiv64(d.m - d.p, SB)); }
                if (d.m > d.p) {
                    lt.push_back(f);
                    lti.push_back(cdiv64(d.m - d.p, 64) * cdiv64(d.p, SB));
                    lr.push_back(f);
                    lri.push_back(cdiv64(d.m - d.p, 256));
                }
            }
            maxsteps = std::max<int>(maxsteps, (int)cdiv64(d.p, FNB));
            maxsb = std::max<int>(maxsb, (int)cdiv64(d.p, SB));
        }
        tb.add(lv.all, fl, one);
        tb.add(lv.u12, ut, uti);
        tb.add(lv.u12red, ur, uri);
        tb.add(lv.l21, lt, lti);
        tb.add(lv.l21red, lr, lri);
        for (int f : ut) {        // each streams its p x (m - p) block once
            const FrontDesc &d = p.h_fd[f];
            lv.u12.elems += (double)d.p * (d.m - d.p);
            lv.u12.rows += d.m;
            lv.l21.elems += (double)d.p * (d.m - d.p);
            lv.l21.rows += d.m;
        }
        {
            std::vector<int64_t> cols;
            for (int f : fl) cols.push_back(p.h_fd[f].m);
            tb.add(lv.pull, fl, cols);
        }
        lv.steps.assign(maxsteps, StepTasks{});
        for (int st = 0; st < maxsteps; st++) {
            std::vector<int32_t> act;
            std::vector<int64_t> o1, tu, rb, sh;
            for (int f : fl) {
                const FrontDesc &d = p.h_fd[f];
                int k0 = st * FNB;
                if (d.p <= k0) continue;
                int kb = std::min(FNB, d.p - k0), k1 = k0 + kb;
                int K1 = std::min(d.p, (k0 / SB + 1) * SB);
                act.push_back(f);
                o1.push_back(1);
                tu.push_back(cdiv64(k0, TRSM_U_COLS) + cdiv64(d.m - k1, TRSM_U_COLS));
                rb.push_back(cdiv64(d.m - piv_window_end(k0, d.p), TRSM_L_ROWS));   // below the pivot window
                sh.push_back((K1 > k1 ? cdiv64(d.m - k1, SCHUR_TILE) * cdiv64(K1 - k1, SCHUR_TILE) : 0) +
                             cdiv64(K1 - k1, SCHUR_TILE) * cdiv64(d.m - K1, SCHUR_TILE));
            }
            StepTasks &S = lv.steps[st];
            tb.add(S.panel, act, o1);
            tb.add(S.trsm_u, act, tu);
            tb.add(S.rows_below, act, rb);
            tb.add(S.schur, act, sh);
            for (int f : act) {
                const FrontDesc &d = p.h_fd[f];
                double k0 = st * FNB, kb = std::min(FNB, d.p - st * FNB);
                double K1 = std::min(d.p, (st * FNB / SB + 1) * SB);
                double rows = d.m - k0 - kb, cols = K1 - k0 - kb, strip = d.m - K1;
                S.schur.flops += 2.0 * (rows * cols + cols * strip) * kb;
                S.schur.elems += 2.0 * (rows * cols + cols * strip) + (rows + cols + strip) * kb;
            }
        }
        lv.outer.assign(maxsb, OuterTasks{});
        for (int T = 0; T < maxsb; T++) {
            std::vector<int32_t> act, sact;
            std::vector<int64_t> sh, ss;
            for (int f : fl) {
                const FrontDesc &d = p.h_fd[f];
                int K0 = T * SB;
                if (d.p <= K0) continue;
                int K1 = std::min(d.p, K0 + SB);
                if (T % 2 == 0 && d.p > K1) {         // successor exists: strips only
                    int K2 = std::min(d.p, K1 + SB);
                    sact.push_back(f);
                    ss.push_back(cdiv64(d.m - K1, SCHUR_TILE) * cdiv64(K2 - K1, SCHUR_TILE) +
                                 cdiv64(K2 - K1, SCHUR_TILE) * cdiv64(d.m - K2, SCHUR_TILE));
                    continue;
                }
                act.push_back(f);
                sh.push_back(cdiv64(d.m - K1, SCHUR_TILE) * cdiv64(d.m - K1, SCHUR_TILE));
            }
            OuterTasks &O = lv.outer[T];
            tb.add(O.schur, act, sh);
            tb.add(O.strip, sact, ss);
            for (int f : act) {
                const FrontDesc &d = p.h_fd[f];
                double K0 = (T % 2 ? T - 1 : T) * SB, kd = std::min(d.p - K0, (T % 2 ? 2.0 : 1.0) * SB);
                double rest = d.m - K0 - kd;
                O.schur.flops += 2.0 * rest * rest * kd;
                O.schur.elems += 2.0 * rest * rest + 2.0 * rest * kd;
            }
            for (int f : sact) {
                const FrontDesc &d = p.h_fd[f];
                double K1 = (T + 1.0) * SB, K2 = std::min<double>(d.p, K1 + SB), w = K2 - K1;
                double area = (d.m - K1) * w + w * (d.m - K2);
                O.strip.flops += 2.0 * area * SB;
                O.strip.elems += 2.0 * area + SB * (2.0 * d.m - K1 - K2 + 2.0 * w);
            }
        }
        {
            std::vector<int64_t> gi;
            for (int f : fl) gi.push_back(cdiv64(p.h_fd[f].m, 256));
            tb.add(lv.fgather, fl, gi);
        }
        const int maxssb = (int)cdiv64((int64_t)maxsb * SB, SSB);   // solve blocks of SSB columns
        lv.fstep.assign(maxssb, TaskList{});
        lv.bstep.assign(maxssb, TaskList{});
        for (int st = 0; st < maxssb; st++) {
            std::vector<int32_t> act;
            std::vector<int64_t> fi, bi;
            for (int f : fl) {
                const FrontDesc &d = p.h_fd[f];
                int t0 = st * SSB;
                if (d.p <= t0) continue;
                int tend = std::min(d.p, t0 + SSB);
                int64_t na = cdiv64(tend - t0, STEP_RW);
                act.push_back(f);
                fi.push_back(na + cdiv64(d.p - tend, STEP_RW));
                bi.push_back(na + cdiv64(t0, STEP_RW));
            }
            tb.add(lv.fstep[st], act, fi);
            tb.add(lv.bstep[st], act, bi);
            for (int f : act) {
                const FrontDesc &d = p.h_fd[f];
                double t0 = st * SSB, sw = std::min(SSB, d.p - st * SSB), tend = t0 + sw;
                lv.fstep[st].elems += 0.5 * sw * (sw + 1) + (d.p - tend) * sw;
                lv.fstep[st].rows += 2.0 * sw + (d.p - tend);
                lv.bstep[st].elems += 0.5 * sw * (sw + 1) + t0 * sw;
                lv.bstep[st].rows += 2.0 * sw + t0;
            }
        }
    }
    // upload
    hipStream_t s = stream;
    p.d_fd.alloc(sizeof(FrontDesc) * nf, &budget);
    h2d(p.d_fd.ptr<FrontDesc>(), p.h_fd.data(), nf, s);
    p.d_perm.alloc(sizeof(int32_t) * p.dim, &budget);
    h2d(p.d_perm.ptr<int32_t>(), t.perm.data(), p.dim, s);
    p.d_contrib.alloc(sizeof(int32_t) * std::max<size_t>(1, t.contrib.size()), &budget);
    h2d(p.d_contrib.ptr<int32_t>(), t.contrib.data(), t.contrib.size(), s);
    p.d_pullmap.alloc(sizeof(int32_t) * std::max<size_t>(1, pullmap.size()), &budget);
    h2d(p.d_pullmap.ptr<int32_t>(), pullmap.data(), pullmap.size(), s);
    p.d_child_ids.alloc(sizeof(int32_t) * std::max<size_t>(1, child_ids.size()), &budget);
    h2d(p.d_child_ids.ptr<int32_t>(), child_ids.data(), child_ids.size(), s);
    p.d_tfronts.alloc(sizeof(int32_t) * std::max<size_t>(1, tb.fr.size()), &budget);
    h2d(p.d_tfronts.ptr<int32_t>(), tb.fr.data(), tb.fr.size(), s);
    p.d_tprefix.alloc(sizeof(int64_t) * std::max<size_t>(1, tb.pre.size()), &budget);
    h2d(p.d_tprefix.ptr<int64_t>(), tb.pre.data(), tb.pre.size(), s);
    if (tb.its.empty()) tb.its.push_back(make_int2(0, 0));
    p.d_titems.alloc(sizeof(int2) * tb.its.size(), &budget);
    h2d(p.d_titems.ptr<int2>(), tb.its.data(), tb.its.size(), s);
    for (size_t i = 0; i < tb.lists.size(); i++) {
        tb.lists[i]->fronts = p.d_tfronts.ptr<int32_t>() + tb.offs[i].fr;
        tb.lists[i]->prefix = p.d_tprefix.ptr<int64_t>() + tb.offs[i].pre;
        tb.lists[i]->items = p.d_titems.ptr<int2>() + tb.offs[i].its;
    }
    p.d_inv_ptr.alloc(sizeof(int32_t) * std::max<size_t>(1, inv_ptr.size()), &budget);
    h2d(p.d_inv_ptr.ptr<int32_t>(), inv_ptr.data(), inv_ptr.size(), s);
    p.d_inv_src.alloc(sizeof(int32_t) * std::max<size_t>(2, inv_src.size()), &budget);
    h2d(p.d_inv_src.ptr<int32_t>(), inv_src.data(), inv_src.size(), s);
    size_t ne = std::max<size_t>(1, efront.size());
    p.d_efront.alloc(sizeof(int32_t) * ne, &budget);
    p.d_epos.alloc(sizeof(int32_t) * ne, &budget);
    p.d_esrc.alloc(sizeof(int32_t) * ne, &budget);
    h2d(p.d_efront.ptr<int32_t>(), efront.data(), efront.size(), s);
    h2d(p.d_epos.ptr<int32_t>(), epos.data(), epos.size(), s);
    h2d(p.d_esrc.ptr<int32_t>(), esrc.data(), esrc.size(), s);
    MBL_HIP(hipStreamSynchronize(s));
    MBL_HIP(hipStreamSynchronize(s));   // uploads complete before other streams read them
    p.have_symbolic = true;
}

// The plan of nseg problems of one chain length solved together: the
// block-diagonal matrix of nseg copies of the sector Hamiltonian, its front
// tree nseg copies of the lone problem's (so each problem is factored and
// solved with exactly its lone arithmetic), built once per (L, nseg).
Plan &Context::batch_plan(int L, int nseg) {
    MBL_REQUIRE(nseg >= 1 && nseg <= MBL_SEG_MAX, MBL_EINVAL, "batch of 1..16 problems");
    std::lock_guard<std::recursive_mutex> lk(plans_->mu);
    Plan &base = plan(L);
    if (nseg == 1) return base;
    ensure_symbolic(base);
    const int key = L * 100 + nseg;
    auto it = plans_->batched.find(key);
    if (it != plans_->batched.end()) return *it->second;
    MBL_REQUIRE(owns_plans_, MBL_EINVAL, "batch plan not prepared by the owning context");
    std::unique_ptr<Plan> bp(new Plan);
    const int64_t n = base.dim, nz = base.nnz;
    bp->L = L;
    bp->nseg = nseg;
    bp->dim = n * nseg;
    bp->nnz = nz * nseg;
    MBL_REQUIRE(bp->nnz < INT32_MAX, MBL_EINVAL, "batch too large for 32-bit indices");
    bp->h_rowptr.resize(bp->dim + 1);
    bp->h_col.resize(bp->nnz);
    for (int sg = 0; sg < nseg; sg++) {
        for (int64_t i = 0; i < n; i++) bp->h_rowptr[sg * n + i] = base.h_rowptr[i] + (int32_t)(sg * nz);
        for (int64_t e = 0; e < nz; e++) bp->h_col[sg * nz + e] = base.h_col[e] + (int32_t)(sg * n);
    }
    bp->h_rowptr[bp->dim] = (int32_t)bp->nnz;
    bp->rowptr.alloc(sizeof(int32_t) * (bp->dim + 1), &budget);
    bp->col.alloc(sizeof(int32_t) * bp->nnz, &budget);
    h2d(bp->rowptr.ptr<int32_t>(), bp->h_rowptr.data(), bp->h_rowptr.size(), stream);
    h2d(bp->col.ptr<int32_t>(), bp->h_col.data(), bp->h_col.size(), stream);
    // the front tree, nseg times
    const FrontTree &t = base.tree;
    FrontTree &T = bp->tree;
    const int nf = (int)t.fronts.size();
    const int64_t nc = (int64_t)t.contrib.size();
    T.n = bp->dim;
    T.perm.resize(bp->dim);
    T.iperm.resize(bp->dim);
    T.fronts.resize((size_t)nf * nseg);
    T.contrib.resize((size_t)nc * nseg);
    for (int sg = 0; sg < nseg; sg++) {
        for (int64_t i = 0; i < n; i++) {
            T.perm[sg * n + i] = t.perm[i] + (int32_t)(sg * n);
            T.iperm[sg * n + i] = t.iperm[i] + (int32_t)(sg * n);
        }
        for (int64_t e = 0; e < nc; e++) T.contrib[sg * nc + e] = t.contrib[e] + (int32_t)(sg * n);
        for (int f = 0; f < nf; f++) {
            Front F = t.fronts[f];
            F.first += (int32_t)(sg * n);
            F.cptr += sg * nc;
            if (F.parent >= 0) F.parent += sg * nf;
            for (auto &c : F.children) c += sg * nf;
            T.fronts[(size_t)sg * nf + f] = F;
        }
    }
    T.n_levels = t.n_levels;
    T.nnz_factor = t.nnz_factor * nseg;
    T.front_entries = t.front_entries * nseg;
    T.max_m = t.max_m;
    T.max_p = t.max_p;
    T.flops = t.flops * nseg;
    build_tables(*bp);
    Plan &ref = *bp;
    plans_->batched[key] = std::move(bp);
    return ref;
}

void Context::set_realization(Plan &p, double J_, const double *fields_host, double h,
                              uint64_t seed, bool use_seed) {
    J = J_;
    offv = (p.L == 2) ? J : 0.5 * J;
    d_fields.ensure(sizeof(double) * 32, &budget);
    if (use_seed) {
        launch_fields(p.L, h, seed, d_fields.ptr<double>(), stream);
        h_fields.resize(p.L);
        d2h(h_fields.data(), d_fields.ptr<double>(), p.L, stream);
    } else {
        h_fields.assign(fields_host, fields_host + p.L);
        h2d(d_fields.ptr<double>(), h_fields.data(), p.L, stream);
    }
    d_diag.ensure(sizeof(double) * p.dim, &budget);
    launch_diag(p.L, J, d_fields.ptr<double>(), p.dim, p.basis.ptr<uint32_t>(),
                d_diag.ptr<double>(), stream);
    MBL_HIP(hipStreamSynchronize(stream));
}

void Context::spmv(Plan &p, double shift, int nvec, const double *x, double *y,
                   const double *diag) {
    bool pr = prof_on("spmv");
    if (pr) prof_begin();
    launch_spmv(p.dim, p.rowptr.ptr<int32_t>(), p.col.ptr<int32_t>(),
                diag ? diag : d_diag.ptr<double>(), offv, shift, nvec, x, y, stream);
    // per vector: columns (4 B/nnz), rowptr, diagonal, x gathered, y written
    if (pr) prof_end(4.0 * p.nnz + 4.0 * p.dim + 8.0 * p.dim + nvec * 16.0 * p.dim,
                     2.0 * nvec * (double)p.nnz);
}

// ---------------------------------------------------------------- factor

template <class T>
void Context::factor_t(Plan &p, Factor<T> &f, const double *diag, double sigma,
                       const std::vector<double> &thresh, SolveStats &st) {
    hipStream_t s = stream;
    MBL_REQUIRE((int)thresh.size() == p.nseg, MBL_EINVAL, "factor: one threshold per problem");
    if (f.L != p.L || f.dim != p.dim) {
        // invalid until every buffer is in place: an allocation that throws
        // part way must not leave buffers of another size behind a valid L
        f.L = -1;
        f.valid = false;
        f.arena.reset();
        f.arena.alloc(sizeof(T) * p.arena_elems, &budget);
        f.ipiv.alloc(sizeof(int32_t) * std::max<int64_t>(1, p.dim), &budget);
        f.prow.alloc(sizeof(int32_t) * std::max<int64_t>(1, p.dim), &budget);
        f.npert.alloc(sizeof(int32_t) * MBL_SEG_MAX, &budget);
        f.uinv.alloc(sizeof(double) * FNB * FNB * std::max<size_t>(1, p.h_fd.size()), &budget);
        f.thr.alloc(sizeof(double) * MBL_SEG_MAX, &budget);
        f.L = p.L;
        f.dim = p.dim;
    }
    f.valid = false;
    MBL_HIP(hipMemsetAsync(f.npert.template ptr<int32_t>(), 0, sizeof(int32_t) * p.nseg, s));
    T *A = f.arena.template ptr<T>();
    const FrontDesc *fd = p.d_fd.ptr<FrontDesc>();
    h2d(f.thr.template ptr<double>(), thresh.data(), thresh.size(), s);
    for (size_t l = 0; l < p.levels.size(); l++) {
        LevelTasks &lv = p.levels[l];
        launch_front_pull<T>(A, fd, p.d_pullmap.ptr<int32_t>(), p.d_child_ids.ptr<int32_t>(),
                             lv.pull, s);
        launch_front_assemble<T>(A, fd, lv.ecount, p.d_efront.ptr<int32_t>() + lv.ebegin,
                                 p.d_epos.ptr<int32_t>() + lv.ebegin,
                                 p.d_esrc.ptr<int32_t>() + lv.ebegin, diag, sigma, offv, s);
        for (size_t t = 0; t < lv.steps.size(); t++) {
            StepTasks &S = lv.steps[t];
            launch_panel<T>(A, fd, f.ipiv.template ptr<int32_t>(), f.npert.template ptr<int32_t>(),
                            S.panel, (int)t, f.thr.template ptr<double>(),
                            f.uinv.template ptr<double>(), s);
            launch_trsm<T>(A, fd, f.ipiv.template ptr<int32_t>(), S.trsm_u, S.rows_below, (int)t,
                           f.uinv.template ptr<double>(), s);
            launch_schur<T>(A, fd, S.schur, (int)t, 0, s);
            // end of an outer block (for every front whose block ends here or earlier)
            int ob = (int)t / (SB / FNB);
            bool last = ((int)t % (SB / FNB) == SB / FNB - 1) || t + 1 == lv.steps.size();
            if (last && ob < (int)lv.outer.size()) {
                OuterTasks &O = lv.outer[ob];
                launch_schur<T>(A, fd, O.strip, ob, 5, s);
                bool pr = prof_on("schur") && O.schur.total > 0;
                if (pr) prof_begin();
                launch_schur<T>(A, fd, O.schur, ob, 1, s);
                if (pr) prof_end(O.schur.elems * sizeof(T), O.schur.flops);
            }
        }
    }
    launch_invert_diag<T>(A, fd, f.ipiv.template ptr<int32_t>(), f.prow.template ptr<int32_t>(),
                          p.inv, 3, -1, s);
    launch_xform<T>(A, fd, p.xform, s);
    for (size_t tp = 0; tp < p.fold_lo.size(); tp++) {
        launch_schur<T>(A, fd, p.fold_lo[tp], (int)tp, 2, s);
        launch_schur<T>(A, fd, p.fold_up[tp], (int)tp, 3, s);
    }
    launch_merge_tri<T>(A, fd, p.merge, s);
    st.perturbed.assign(p.nseg, 0);
    d2h(st.perturbed.data(), f.npert.template ptr<int32_t>(), p.nseg, s);
    MBL_HIP(hipStreamSynchronize(s));
    st.n_perturbed = 0;
    for (int v : st.perturbed) st.n_perturbed += v;
    f.valid = true;
    f.sigma = sigma;
}

void Context::factor(Plan &p, int prec, double sigma, double anorm, SolveStats &st) {
    ensure_symbolic(p);
    anorm_ = anorm;
    double t0 = wall_seconds();
    // static pivots: below 1e-7 ||A|| (FP32 factors) or 1e-14 ||A|| (FP64)
    if (prec == MBL_FP32_IR64) factor_t<float>(p, f32_, d_diag.ptr<double>(), sigma, {1e-7 * anorm}, st);
    else factor_t<double>(p, f64_, d_diag.ptr<double>(), sigma, {1e-14 * anorm}, st);
    st.t_factor = wall_seconds() - t0;
}

template <class T>
void Context::lu_apply(Plan &p, Factor<T> &f, int nrhs, const double *b, int64_t ldb, double *x,
                       int64_t ldx) {
    const int64_t n = p.dim;
    lu_passes++;
    lu_pass_rhs += nrhs;
    // timing a class of the solve launches needs events between them: eager
    const bool timed = prof_on("fwd_update") || prof_on("bwd_update") || prof_on("l21") ||
                       prof_on("u12");
    // work buffers of the solve (before the autotuner, which launches into them)
    d_vec.ensure(sizeof(double) * std::max<int64_t>(1, p.vec_elems), &budget);
    d_yv.ensure(sizeof(double) * std::max<int64_t>(1, p.y_elems), &budget);
    d_upart.ensure(sizeof(double) * std::max<int64_t>(1, p.part_elems), &budget);
    d_xnew.ensure(sizeof(double) * n * MAXRHS, &budget);
    const Plan::SolveTune tn = solve_tune<T>(p, f, nrhs);
    if (!use_graphs_ || timed || ldb != n || ldx != n) {
        lu_apply_seq<T>(p, f, nrhs, b, ldb, x, ldx, tn);
        return;
    }
    // The launch sequence of one application is the same every time for a
    // given plan, factor, right-hand-side count and work buffers: it is
    // captured once as a graph between fixed staging vectors and replayed.
    d_gin.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_gout.ensure(sizeof(double) * n * MAXRHS, &budget);
    GraphKey key{&p, p.L, (int)sizeof(T), nrhs,
                 {f.arena.template ptr<void>(), f.prow.template ptr<void>(), d_vec.ptr<void>(),
                  d_yv.ptr<void>(),
                  d_upart.ptr<void>(), d_xnew.ptr<void>(), d_gin.ptr<void>(), d_gout.ptr<void>()}};
    auto it = graphs_.find(key);
    if (it == graphs_.end()) {
        if (graphs_.size() >= 32) clear_graphs();
        hipGraph_t g = nullptr;
        MBL_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            lu_apply_seq<T>(p, f, nrhs, d_gin.ptr<double>(), n, d_gout.ptr<double>(), n, tn);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(stream, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            throw;
        }
        MBL_HIP(hipStreamEndCapture(stream, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        MBL_HIP(e);
        it = graphs_.emplace(key, ex).first;
    }
    launch_copy(n * nrhs, b, d_gin.ptr<double>(), stream);
    MBL_HIP(hipGraphLaunch(it->second, stream));
    launch_copy(n * nrhs, d_gout.ptr<double>(), x, stream);
}

void Context::clear_graphs() {
    for (auto &kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    graphs_.clear();
}

template <class T>
Plan::SolveTune Context::solve_tune(Plan &p, Factor<T> &f, int nrhs) {
    const int key = (int)sizeof(T) * 100 + nrhs;
    {
        std::lock_guard<std::recursive_mutex> lk(plans_->mu);
        auto it = p.tune.find(key);
        if (it != p.tune.end()) return it->second;
    }
    const size_t nl = p.levels.size();
    Plan::SolveTune tn;
    tn.l21.assign(nl, 1);
    tn.u12.assign(nl, 1);
    if (std::getenv("MBL_NO_TUNE") == nullptr) {
        hipStream_t s = stream;
        const T *A = f.arena.template ptr<T>();
        const FrontDesc *fd = p.d_fd.ptr<FrontDesc>();
        double *part = d_upart.ptr<double>();
        hipEvent_t e0 = nullptr, e1 = nullptr;
        MBL_HIP(hipEventCreate(&e0));
        MBL_HIP(hipEventCreate(&e1));
        try {
            auto timed = [&](const std::function<void(int)> &run, int ipw) {
                run(ipw);                              // warm
                MBL_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < 3; r++) run(ipw);
                MBL_HIP(hipEventRecord(e1, s));
                MBL_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                MBL_HIP(hipEventElapsedTime(&ms, e0, e1));
                return ms;
            };
            auto pick = [&](const std::function<void(int)> &run) -> int8_t {
                const float t1 = timed(run, 1), t2 = timed(run, 2);
                return (t2 < 0.97f * t1) ? 2 : 1;     // two tiles only when clearly faster
            };
            for (size_t l = 0; l < nl; l++) {
                LevelTasks &lv = p.levels[l];
                if (lv.l21.total > 0)
                    tn.l21[l] = pick([&](int ipw) {
                        launch_fwd_l21<T>(A, fd, lv.l21, nrhs, d_vec.ptr<double>(), part, ipw, s);
                    });
                if (lv.u12.total > 0)
                    tn.u12[l] = pick([&](int ipw) {
                        launch_bwd_u12<T>(A, fd, lv.u12, nrhs, p.d_contrib.ptr<int32_t>(),
                                          d_xnew.ptr<double>(), p.dim, part, ipw, s);
                    });
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (debug_level() > 0) {
            int n2 = 0;
            for (size_t l = 0; l < nl; l++) n2 += (tn.l21[l] == 2) + (tn.u12[l] == 2);
            std::fprintf(stderr, "[mbl] solve tune L=%d x%d %s nrhs=%d: %d of %zu products with 2 tiles\n",
                         p.L, p.nseg, sizeof(T) == 4 ? "fp32" : "fp64", nrhs, n2, 2 * nl);
        }
    }
    std::lock_guard<std::recursive_mutex> lk(plans_->mu);
    return p.tune.emplace(key, tn).first->second;      // another context may have tuned it first
}

template <class T>
void Context::lu_apply_seq(Plan &p, Factor<T> &f, int nrhs, const double *b, int64_t ldb,
                           double *x, int64_t ldx, const Plan::SolveTune &tn) {
    hipStream_t s = stream;
    const T *A = f.arena.template ptr<T>();
    const FrontDesc *fd = p.d_fd.ptr<FrontDesc>();
    d_vec.ensure(sizeof(double) * std::max<int64_t>(1, p.vec_elems), &budget);
    d_yv.ensure(sizeof(double) * std::max<int64_t>(1, p.y_elems), &budget);
    d_upart.ensure(sizeof(double) * std::max<int64_t>(1, p.part_elems), &budget);
    d_xnew.ensure(sizeof(double) * p.dim * MAXRHS, &budget);
    double *vec = d_vec.ptr<double>(), *yv = d_yv.ptr<double>();
    double *part = d_upart.ptr<double>(), *xnew = d_xnew.ptr<double>();
    const int2 *isrc = reinterpret_cast<const int2 *>(p.d_inv_src.ptr<int32_t>());
    const BwdIO bio{p.d_perm.ptr<int32_t>(), xnew, x, p.dim, ldx, nrhs};
    auto step = [&](TaskList &tl, int t, bool fwd) {
        const char *cls = fwd ? "fwd_update" : "bwd_update";
        bool pr = prof_on(cls) && tl.total > 0;
        if (pr) prof_begin();
        launch_solve_step<T>(A, fd, tl, t, nrhs, fwd, vec, yv, bio, s);
        if (pr) prof_end(tl.elems * sizeof(T) + 16.0 * nrhs * tl.rows, 2.0 * nrhs * tl.elems);
    };
    for (size_t l = 0; l < p.levels.size(); l++) {
        LevelTasks &lv = p.levels[l];
        launch_fwd_gather(fd, p.d_perm.ptr<int32_t>(), f.prow.template ptr<int32_t>(),
                          p.d_inv_ptr.ptr<int32_t>(), isrc, lv.fgather, nrhs, b, ldb, vec, s);
        for (size_t t = 0; t < lv.fstep.size(); t++) step(lv.fstep[t], (int)t, true);
        bool pr = prof_on("l21") && lv.l21.total > 0;
        if (pr) prof_begin();
        launch_fwd_l21<T>(A, fd, lv.l21, nrhs, vec, part, tn.l21[l], s);
        if (pr) prof_end(lv.l21.elems * sizeof(T) + 8.0 * nrhs * lv.l21.rows, 2.0 * nrhs * lv.l21.elems);
        launch_fwd_l21_reduce(fd, lv.l21red, nrhs, vec, part, s);
    }
    for (size_t l = p.levels.size(); l-- > 0;) {
        LevelTasks &lv = p.levels[l];
        bool pr = prof_on("u12") && lv.u12.total > 0;
        if (pr) prof_begin();
        launch_bwd_u12<T>(A, fd, lv.u12, nrhs, p.d_contrib.ptr<int32_t>(), xnew, p.dim, part,
                          tn.u12[l], s);
        if (pr) prof_end(lv.u12.elems * sizeof(T) + 8.0 * nrhs * lv.u12.rows, 2.0 * nrhs * lv.u12.elems);
        launch_bwd_u12_reduce(fd, lv.u12red, nrhs, yv, part, s);
        for (size_t t = lv.bstep.size(); t-- > 0;) step(lv.bstep[t], (int)t, false);
    }
}

// Refinement for single-precision factors: each outer sweep forms the FP64
// residual r = B - (H - sigma) X and solves (H - sigma) D = r by restarted
// flexible GMRES in FP64, right-preconditioned by the FP32 LU (one Arnoldi
// basis per right-hand side, classical Gram-Schmidt applied twice, Givens
// rotations on the host), then X += D.  Unlike plain refinement, whose
// contraction is |I - A M^-1| and stalls once kappa(A) u_32 is not small,
// GMRES only needs the preconditioned spectrum to be clustered.
template <class T>
void Context::gmres_refine(Plan &p, Factor<T> &f, int nrhs, const double *B, double *X,
                           double target, SolveStats &st) {
    hipStream_t s = stream;
    const int64_t n = p.dim;
    constexpr int KM = 30;                   // Arnoldi steps per cycle (<= 31 blocks for bdot)
    const double inner_tol = 1e-6;           // relative residual reduction per cycle
    const int64_t bs = n * (int64_t)nrhs;    // stride between basis blocks
    d_r.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_d.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_part.ensure(sizeof(double) * RES_PARTS * MAXRHS * 3, &budget);
    d_gV.ensure(sizeof(double) * (size_t)bs * (KM + 1), &budget);
    d_gZ.ensure(sizeof(double) * (size_t)bs * KM, &budget);
    const int nparts = gemm_tn_parts(n);
    d_gpart.ensure(sizeof(double) * (size_t)nparts * (KM + 1) * nrhs, &budget);
    d_gcoef.ensure(sizeof(double) * (size_t)(KM + 1) * nrhs * 2, &budget);
    double *r = d_r.ptr<double>(), *w = d_d.ptr<double>();
    double *V = d_gV.ptr<double>(), *Z = d_gZ.ptr<double>();
    double *gp = d_gpart.ptr<double>(), *co = d_gcoef.ptr<double>(), *co2 = co + (KM + 1) * nrhs;
    std::vector<double> part((size_t)RES_PARTS * nrhs * 3);
    std::vector<double> beta0(nrhs), hc((size_t)(KM + 1) * nrhs), hc2((size_t)(KM + 1) * nrhs);
    std::vector<double> Hm((size_t)(KM + 1) * KM * nrhs), cs((size_t)KM * nrhs), sn((size_t)KM * nrhs);
    std::vector<double> g((size_t)(KM + 1) * nrhs), y((size_t)KM * nrhs);
    std::vector<int> kconv(nrhs);
    std::vector<double> scal(nrhs), nn(nrhs);
    auto Hat = [&](int i, int k, int j) -> double & { return Hm[((size_t)j * KM + k) * (KM + 1) + i]; };
    double be = 1e300;
    int sweeps = 0, inner_total = 0;
    for (;; sweeps++) {
        launch_residual(n, p.rowptr.ptr<int32_t>(), p.col.ptr<int32_t>(), d_diag.ptr<double>(),
                        offv, f.sigma, nrhs, B, X, r, d_part.ptr<double>(), RES_PARTS, s);
        d2h(part.data(), d_part.ptr<double>(), part.size(), s);
        MBL_HIP(hipStreamSynchronize(s));
        be = 0.0;
        for (int v = 0; v < nrhs; v++) {
            double sr = 0, sx = 0, sb = 0;
            for (int q = 0; q < RES_PARTS; q++) {
                const double *pp = &part[((size_t)q * nrhs + v) * 3];
                sr += pp[0]; sx += pp[1]; sb += pp[2];
            }
            double den = anorm_ * std::sqrt(sx) + std::sqrt(sb);
            be = std::max(be, den > 0 ? std::sqrt(sr) / den : 0.0);
            beta0[v] = std::sqrt(sr);
        }
        if (debug_level() > 0)
            std::fprintf(stderr, "[mbl] gmres-ir L=%d sweep=%d be=%.3e nrhs=%d inner=%d\n", p.L,
                         sweeps, be, nrhs, inner_total);
        if (be <= target || sweeps >= 6) break;
        // V_0 = r / |r| per column
        for (int v = 0; v < nrhs; v++) scal[v] = beta0[v] > 0 ? 1.0 / beta0[v] : 0.0;
        h2d(co, scal.data(), (size_t)nrhs, s);
        launch_bcomb(n, 1, nrhs, r, bs, co, 1.0, 0.0, V, s);
        std::fill(Hm.begin(), Hm.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        for (int v = 0; v < nrhs; v++) { g[(size_t)v * (KM + 1)] = beta0[v]; kconv[v] = -1; }
        int k = 0;
        for (; k < KM; k++) {
            double *Vk = V + (int64_t)k * bs, *Zk = Z + (int64_t)k * bs;
            lu_apply<T>(p, f, nrhs, Vk, n, Zk, n);
            launch_spmv(n, p.rowptr.ptr<int32_t>(), p.col.ptr<int32_t>(), d_diag.ptr<double>(), offv,
                        f.sigma, nrhs, Zk, w, s);
            for (int pass = 0; pass < 2; pass++) {
                launch_bdot(n, k + 1, nrhs, V, bs, w, co, gp, nparts, s);
                launch_bcomb(n, k + 1, nrhs, V, bs, co, -1.0, 1.0, w, s);
                d2h(pass == 0 ? hc.data() : hc2.data(), co, (size_t)(k + 1) * nrhs, s);
            }
            launch_bdot(n, 1, nrhs, w, bs, w, co2, gp, nparts, s);
            d2h(nn.data(), co2, (size_t)nrhs, s);
            MBL_HIP(hipStreamSynchronize(s));
            bool all = true;
            for (int v = 0; v < nrhs; v++) {
                double hn = std::sqrt(std::max(0.0, nn[v]));
                for (int i = 0; i <= k; i++)
                    Hat(i, k, v) = hc[(size_t)v * (k + 1) + i] + hc2[(size_t)v * (k + 1) + i];
                Hat(k + 1, k, v) = hn;
                scal[v] = hn > 1e-300 ? 1.0 / hn : 0.0;   // scaling of the next basis vector
                if (kconv[v] >= 0) continue;
                // apply the previous rotations of this column, then a new one
                for (int i = 0; i < k; i++) {
                    double a = Hat(i, k, v), b2 = Hat(i + 1, k, v);
                    Hat(i, k, v) = cs[(size_t)v * KM + i] * a + sn[(size_t)v * KM + i] * b2;
                    Hat(i + 1, k, v) = -sn[(size_t)v * KM + i] * a + cs[(size_t)v * KM + i] * b2;
                }
                double a = Hat(k, k, v), b2 = Hat(k + 1, k, v);
                double rr = std::hypot(a, b2);
                double c = rr > 0 ? a / rr : 1.0, sgn = rr > 0 ? b2 / rr : 0.0;
                cs[(size_t)v * KM + k] = c;
                sn[(size_t)v * KM + k] = sgn;
                Hat(k, k, v) = rr;
                Hat(k + 1, k, v) = 0.0;
                double gk = g[(size_t)v * (KM + 1) + k];
                g[(size_t)v * (KM + 1) + k] = c * gk;
                g[(size_t)v * (KM + 1) + k + 1] = -sgn * gk;
                if (std::fabs(g[(size_t)v * (KM + 1) + k + 1]) <= inner_tol * beta0[v] || hn <= 1e-300)
                    kconv[v] = k + 1;
                else
                    all = false;
            }
            inner_total++;
            if (all || k + 1 == KM) { k++; break; }
            h2d(co, scal.data(), (size_t)nrhs, s);
            launch_bcomb(n, 1, nrhs, w, bs, co, 1.0, 0.0, V + (int64_t)(k + 1) * bs, s);
        }
        // least-squares solutions (upper triangular) and D = Z y, X += D
        std::fill(y.begin(), y.end(), 0.0);
        for (int v = 0; v < nrhs; v++) {
            int kv = kconv[v] >= 0 ? kconv[v] : k;
            for (int i = kv - 1; i >= 0; i--) {
                double acc = g[(size_t)v * (KM + 1) + i];
                for (int q = i + 1; q < kv; q++) acc -= Hat(i, q, v) * y[(size_t)v * k + q];
                y[(size_t)v * k + i] = Hat(i, i, v) != 0.0 ? acc / Hat(i, i, v) : 0.0;
            }
        }
        h2d(co, y.data(), (size_t)k * nrhs, s);
        launch_bcomb(n, k, nrhs, Z, bs, co, 1.0, 1.0, X, s);
    }
    st.backward_error = be;
    st.ir_iters = std::max(st.ir_iters, sweeps);
    st.gmres_inner += inner_total;
    if (be > 1e-10) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "shifted solve: backward error %.3e after %d GMRES sweeps",
                      be, sweeps);
        throw Error(MBL_ENUMERIC, msg);
    }
}

template <class T>
void Context::refine(Plan &p, Factor<T> &f, int nrhs, const double *B, double *X,
                     SolveStats &st) {
    hipStream_t s = stream;
    int64_t n = p.dim;
    d_r.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_d.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_part.ensure(sizeof(double) * RES_PARTS * MAXRHS * 3, &budget);
    double *r = d_r.ptr<double>(), *dd = d_d.ptr<double>();
    lu_apply<T>(p, f, nrhs, B, n, X, n);
    std::vector<double> part((size_t)RES_PARTS * nrhs * 3);
    const double target = sizeof(T) == 8 ? refine_target : SOLVE_TARGET;

    double prev = 1e300;
    int it = 0;
    for (;; it++) {
        launch_residual(n, p.rowptr.ptr<int32_t>(), p.col.ptr<int32_t>(), d_diag.ptr<double>(),
                        offv, f.sigma, nrhs, B, X, r, d_part.ptr<double>(), RES_PARTS, s);
        d2h(part.data(), d_part.ptr<double>(), part.size(), s);
        MBL_HIP(hipStreamSynchronize(s));
        double be = 0.0;
        for (int v = 0; v < nrhs; v++) {
            double sr = 0, sx = 0, sb = 0;
            for (int q = 0; q < RES_PARTS; q++) {
                const double *pp = &part[((size_t)q * nrhs + v) * 3];
                sr += pp[0]; sx += pp[1]; sb += pp[2];
            }
            double den = anorm_ * std::sqrt(sx) + std::sqrt(sb);
            double e = den > 0 ? std::sqrt(sr) / den : 0.0;
            be = std::max(be, e);
        }
        st.backward_error = be;
        if (debug_level() > 0)
            std::fprintf(stderr, "[mbl] refine L=%d prec=%s it=%d be=%.3e nrhs=%d npert=%d\n", p.L,
                         sizeof(T) == 4 ? "fp32" : "fp64", it, be, nrhs, st.n_perturbed);
        if (hooks & (sizeof(T) == 4 ? MBL_HOOK_IR_STALL32 : MBL_HOOK_IR_STALL64))
            throw Error(MBL_ENUMERIC, "shifted solve: refinement stagnation forced by a test hook");
        if (be <= target || it >= 12) break;
        if (sizeof(T) == 4 && it >= 1 && be > 0.25 * prev) {
            // single-precision factors contracting slowly (kappa u_32 not small):
            // continue from the current X with GMRES-based refinement
            st.ir_iters = std::max(st.ir_iters, it);
            gmres_refine<T>(p, f, nrhs, B, X, target, st);
            return;
        }
        if (be > 0.5 * prev && it >= 3) break;    // stagnation
        prev = be;
        lu_apply<T>(p, f, nrhs, r, n, dd, n);
        launch_axpy(n * nrhs, 1.0, dd, X, s);
    }
    st.ir_iters = std::max(st.ir_iters, it);
    if (st.backward_error > 1e-10) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "shifted solve: backward error %.3e after %d refinement sweeps",
                      st.backward_error, it);
        throw Error(MBL_ENUMERIC, msg);
    }
}

void Context::shift_solve(Plan &p, int prec, int nrhs, const double *B, double *X,
                          SolveStats &st) {
    double t0 = wall_seconds();
    st.gmres_inner = 0;
    for (int c = 0; c < nrhs; c += MAXRHS) {
        int nb = std::min(MAXRHS, nrhs - c);
        if (prec == MBL_FP32_IR64) refine<float>(p, f32_, nb, B + (int64_t)c * p.dim, X + (int64_t)c * p.dim, st);
        else refine<double>(p, f64_, nb, B + (int64_t)c * p.dim, X + (int64_t)c * p.dim, st);
    }
    st.n_rhs += nrhs;
    st.t_solve += wall_seconds() - t0;
}

// ---------------------------------------------------------------- batches

void Context::factor_batch(Plan &bp, int prec, const double *shifted,
                           const std::vector<double> &anorm, SolveStats &st) {
    MBL_REQUIRE((int)anorm.size() == bp.nseg, MBL_EINVAL, "factor_batch: one norm per problem");
    double t0 = wall_seconds();
    // the static-pivot thresholds of lone factors, per problem; the diagonals
    // arrive shifted, so the assembly subtracts zero
    std::vector<double> th(bp.nseg);
    for (int sg = 0; sg < bp.nseg; sg++) th[sg] = (prec == MBL_FP32_IR64 ? 1e-7 : 1e-14) * anorm[sg];
    if (prec == MBL_FP32_IR64) factor_t<float>(bp, fb32_, shifted, 0.0, th, st);
    else factor_t<double>(bp, fb64_, shifted, 0.0, th, st);
    st.t_factor = wall_seconds() - t0;
}

// Refinement of the problems of a batch, each deciding when to stop exactly as
// refine() does for a lone problem (same residuals, same tests, in the same
// order); a problem that has stopped keeps its X while the others go on.  Where
// a lone solve would leave the plain refinement (FP32 contracting slowly, or
// no convergence), the batch cannot follow it: the problem is dropped from the
// batch (bs.dropped) and solved alone afterwards.
template <class T>
void Context::refine_batch(Plan &p, Factor<T> &f, int nrhs, const double *B, double *X,
                           const double *shifted, const std::vector<double> &anorm,
                           const std::vector<char> &skip, BatchSolveStats &bs) {
    hipStream_t s = stream;
    const int nseg = p.nseg;
    const int64_t N = p.dim, n = N / nseg;
    d_r.ensure(sizeof(double) * N * MAXRHS, &budget);
    d_d.ensure(sizeof(double) * N * MAXRHS, &budget);
    d_part.ensure(sizeof(double) * RES_PARTS * MAXRHS * 3 * nseg, &budget);
    d_on.ensure(sizeof(int) * MBL_SEG_MAX, &budget);
    double *r = d_r.ptr<double>(), *dd = d_d.ptr<double>();
    std::vector<int> on(nseg);
    for (int sg = 0; sg < nseg; sg++) on[sg] = (skip[sg] || bs.dropped[sg]) ? 0 : 1;
    auto count_pass = [&]() {
        for (int sg = 0; sg < nseg; sg++)
            if (on[sg]) { bs.passes[sg]++; bs.pass_rhs[sg] += nrhs; }
    };
    lu_apply<T>(p, f, nrhs, B, N, X, N);
    count_pass();
    std::vector<double> part((size_t)RES_PARTS * nrhs * 3 * nseg), prev(nseg, 1e300), be(nseg, 0.0);
    const double target = sizeof(T) == 8 ? refine_target : SOLVE_TARGET;
    for (int it = 0;; it++) {
        launch_residual_seg(nseg, n, p.rowptr.ptr<int32_t>(), p.col.ptr<int32_t>(), shifted, offv,
                            0.0, nrhs, B, X, r, d_part.ptr<double>(), RES_PARTS, s);
        d2h(part.data(), d_part.ptr<double>(), part.size(), s);
        MBL_HIP(hipStreamSynchronize(s));
        int active = 0;
        for (int sg = 0; sg < nseg; sg++) {
            if (!on[sg]) continue;
            const double *ps = &part[(size_t)sg * RES_PARTS * nrhs * 3];
            double e_max = 0.0;
            for (int v = 0; v < nrhs; v++) {
                double sr = 0, sx = 0, sb = 0;
                for (int q = 0; q < RES_PARTS; q++) {
                    const double *pp = &ps[((size_t)q * nrhs + v) * 3];
                    sr += pp[0]; sx += pp[1]; sb += pp[2];
                }
                double den = anorm[sg] * std::sqrt(sx) + std::sqrt(sb);
                double e = den > 0 ? std::sqrt(sr) / den : 0.0;
                e_max = std::max(e_max, e);
            }
            be[sg] = e_max;
            if (bs.hooks[sg] & (sizeof(T) == 4 ? MBL_HOOK_IR_STALL32 : MBL_HOOK_IR_STALL64)) {
                on[sg] = 0;                        // the lone solve fails here (test hook)
                bs.dropped[sg] = 1;
                continue;
            }
            bool stop = (e_max <= target || it >= 12);
            if (!stop && sizeof(T) == 4 && it >= 1 && e_max > 0.25 * prev[sg]) {
                on[sg] = 0;                        // a lone solve goes on with GMRES
                bs.dropped[sg] = 1;
                continue;
            }
            if (!stop && e_max > 0.5 * prev[sg] && it >= 3) stop = true;    // stagnation
            if (stop) {
                on[sg] = 0;
                bs.ir_iters[sg] = std::max(bs.ir_iters[sg], it);
                if (e_max > 1e-10) bs.dropped[sg] = 1;    // a lone solve reports the failure
                continue;
            }
            prev[sg] = e_max;
            active++;
        }
        if (debug_level() > 0)
            std::fprintf(stderr, "[mbl] refine batch L=%d x%d prec=%s it=%d active=%d\n", p.L, nseg,
                         sizeof(T) == 4 ? "fp32" : "fp64", it, active);
        if (!active) break;
        h2d(d_on.ptr<int>(), on.data(), nseg, s);
        lu_apply<T>(p, f, nrhs, r, N, dd, N);
        count_pass();
        launch_axpy_masked(n, nseg, nrhs, d_on.ptr<int>(), dd, X, s);
    }
}

void Context::shift_solve_batch(Plan &bp, int prec, int nrhs, const double *B, double *X,
                                const double *shifted, const std::vector<double> &anorm,
                                const std::vector<char> &skip, BatchSolveStats &bs) {
    double t0 = wall_seconds();
    for (int c = 0; c < nrhs; c += MAXRHS) {
        int nb = std::min(MAXRHS, nrhs - c);
        const int64_t o = (int64_t)c * bp.dim;
        if (prec == MBL_FP32_IR64) refine_batch<float>(bp, fb32_, nb, B + o, X + o, shifted, anorm, skip, bs);
        else refine_batch<double>(bp, fb64_, nb, B + o, X + o, shifted, anorm, skip, bs);
    }
    bs.t_solve += wall_seconds() - t0;
}

// ---------------------------------------------------------------- Krylov-Schur

// All eigenpairs of count symmetric m x m matrices A[k] (host, column-major)
// by the device Jacobi kernel, one workgroup each: w[k] ascending, Z[k]
// (m x m) the unit eigenvectors in the same order.
void Context::small_eig_batch(int count, int m, const std::vector<std::vector<double>> &A,
                              std::vector<std::vector<double>> &w,
                              std::vector<std::vector<double>> &Z, bool general) {
    hipStream_t s = stream;
    const size_t mm = (size_t)m * m;
    // device and page-locked host layout: thresholds and matrices (copied in
    // one transfer), then vectors, values and sweep counts (copied back in one)
    const size_t in_n = (size_t)count * (1 + mm), out_n = (size_t)count * (mm + m);
    const size_t bytes = sizeof(double) * (in_n + out_n) + sizeof(int) * (size_t)count;
    d_ritz.ensure(bytes + 64, &budget);
    h_ritz.ensure(bytes);
    double *dtol = d_ritz.ptr<double>(), *dA = dtol + count, *dV = dA + mm * count;
    double *dw = dV + mm * count;
    int *dinfo = reinterpret_cast<int *>(dw + (size_t)m * count);
    double *htol = h_ritz.ptr<double>(), *hA = htol + count, *hV = hA + mm * count;
    double *hw = hV + mm * count;
    int *hinfo = reinterpret_cast<int *>(hw + (size_t)m * count);
    for (int k = 0; k < count; k++) {
        double fro = 0.0;
        for (double x : A[k]) fro += x * x;
        // off-diagonal entries at or below 1e-17 ||A||_F are left in place:
        // their effect on the eigenvalues is below the rounding of ||A||
        htol[k] = 1e-17 * std::sqrt(fro);
        std::copy(A[k].begin(), A[k].begin() + mm, hA + mm * k);
    }
    h2d(dtol, htol, in_n, s);
    launch_jacobi_eig_batch(count, m, dA, dV, dw, dinfo, dtol, s, general);
    MBL_HIP(hipMemcpyAsync(hV, dV, sizeof(double) * out_n + sizeof(int) * (size_t)count,
                           hipMemcpyDeviceToHost, s));
    MBL_HIP(hipStreamSynchronize(s));
    w.assign(count, {});
    Z.assign(count, {});
    for (int k = 0; k < count; k++) {
        if (hinfo[k] < 0) throw Error(MBL_ENUMERIC, "Jacobi eigensolver: sweep limit reached");
        if (debug_level() > 1) std::fprintf(stderr, "[mbl] jacobi m=%d sweeps=%d\n", m, hinfo[k]);
        const double *wk = hw + (size_t)m * k, *vk = hV + mm * k;
        std::vector<int> perm(m);
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return wk[a] < wk[c]; });
        w[k].resize(m);
        Z[k].resize(mm);
        for (int j = 0; j < m; j++) {
            w[k][j] = wk[perm[j]];
            std::copy(vk + (size_t)perm[j] * m, vk + (size_t)(perm[j] + 1) * m,
                      Z[k].begin() + (size_t)j * m);
        }
    }
}

// ---------------------------------------------------------------- Krylov-Schur

// Thick-restart block Krylov-Schur on nseg independent problems of order n at
// once (dropped, if given: problems the operator gave up, which stop at the
// next Rayleigh-Ritz step without a result).  Their vectors are packed (problem s is rows [s n, (s + 1) n) of every
// column, ld = nseg n), the operator acts on packed blocks, and every
// reduction, small factorisation and Rayleigh-Ritz step is done per problem
// with exactly the arithmetic of a lone problem, so each problem's results do
// not depend on the others.  A problem whose wanted pairs have converged (or
// that reached max_restarts) writes its Ritz vectors to its rows of out and
// stops changing; the iteration ends when every problem has.
void Context::krylov_schur(int64_t n, int nseg, int b, int ncv, int nkeep, int nwant, Want want,
                           const KSOp &op, const std::function<bool(int, double, double)> &conv,
                           int max_restarts, const uint64_t *seeds, double *out,
                           std::vector<KSOut> &result, const std::vector<char> *dropped) {
    hipStream_t s = stream;
    const int cols = ncv + b;
    const bool full = (ncv >= n);   // the basis can span the whole space
    const int64_t ldv = n * nseg;
    MBL_REQUIRE(nwant <= nkeep && nkeep <= ncv && ncv % b == 0 && (full || nkeep + b <= ncv) &&
                    (full || nkeep % b == 0) && (!full || b == 1),
                MBL_EINVAL, "krylov_schur: inconsistent basis sizes");
    MBL_REQUIRE(nseg >= 1 && nseg <= MBL_SEG_MAX && (nseg == 1 || b > 1), MBL_EINVAL,
                "krylov_schur: batched problems need a block size above one");
    d_V.ensure(sizeof(double) * ldv * cols, &budget);
    d_V2.ensure(sizeof(double) * ldv * cols, &budget);
    d_W.ensure(sizeof(double) * ldv * b, &budget);
    // per problem: coefficient / projection block, Gram matrix, R^-1
    const int64_t SMS = (int64_t)cols * std::max(cols, b) + 2 * (int64_t)b * b;
    d_small.ensure(sizeof(double) * SMS * nseg + 64, &budget);
    int nparts = gemm_tn_parts(n);
    d_tnpart.ensure(sizeof(double) * (size_t)nparts * cols * b * nseg, &budget);
    double *V = d_V.ptr<double>(), *V2 = d_V2.ptr<double>(), *W = d_W.ptr<double>();
    double *sm = d_small.ptr<double>();
    double *tnp = d_tnpart.ptr<double>();
    double *smG = sm + (int64_t)cols * std::max(cols, b), *smRi = smG + b * b;
    std::vector<std::vector<double>> T(nseg, std::vector<double>((size_t)cols * cols, 0.0));
    auto Tat = [&](int sg, int i, int j) -> double & { return T[sg][(size_t)j * cols + i]; };

    // classical Gram-Schmidt, twice, of blk against V[:, 0:c0]; coefficients
    // summed (single problem, vector at a time)
    std::vector<double> hh;
    auto project = [&](int c0, double *blk, std::vector<double> &hsum) {
        hsum.assign((size_t)c0 * b, 0.0);
        if (c0 == 0) return;
        for (int pass = 0; pass < 2; pass++) {
            launch_gemm_tn(n, c0, b, V, n, blk, n, sm, tnp, nparts, s);
            launch_gemm_nn(n, c0, b, -1.0, V, n, sm, c0, 1.0, blk, n, s);
            hh.resize((size_t)c0 * b);
            d2h(hh.data(), sm, hh.size(), s);
            MBL_HIP(hipStreamSynchronize(s));
            for (size_t q = 0; q < hh.size(); q++) hsum[q] += hh[q];
        }
    };
    // dst = src R^-1 (Cholesky QR, two passes, host factors; single problem);
    // src is used as scratch
    std::vector<double> G, Ri;
    auto cholqr = [&](double *src, double *dst, std::vector<double> &R) -> bool {
        G.resize((size_t)b * b);
        bool ok = true;
        std::vector<double> Rp[2];
        double *from = src, *to = dst;
        for (int pass = 0; pass < 2; pass++) {
            launch_gemm_tn(n, b, b, from, n, from, n, sm, tnp, nparts, s);
            d2h(G.data(), sm, G.size(), s);
            MBL_HIP(hipStreamSynchronize(s));
            if (!cholesky_upper(b, G.data(), Rp[pass], 1e-24)) ok = false;
            upper_inverse(b, Rp[pass], Ri);
            h2d(sm, Ri.data(), Ri.size(), s);
            launch_gemm_nn(n, b, b, 1.0, from, n, sm, b, 0.0, to, n, s);
            std::swap(from, to);
        }
        launch_copy(n * b, from, dst, s);   // from == src after two passes
        R.assign((size_t)b * b, 0.0);      // R = R2 R1
        for (int j = 0; j < b; j++)
            for (int i = 0; i < b; i++) {
                double acc = 0.0;
                for (int k = 0; k < b; k++) acc += Rp[1][(size_t)k * b + i] * Rp[0][(size_t)j * b + k];
                R[(size_t)j * b + i] = acc;
            }
        return ok;
    };

    // Blocks of more than one vector expand without host round trips: the
    // Cholesky factors are computed on the device, the projection coefficients
    // and R factors are copied to page-locked memory asynchronously, and the
    // projected matrices are assembled once per restart cycle.
    const bool async = (b > 1);
    std::vector<char> finished(nseg, 0);
    struct Stage { int cur; size_t h1, h2, r1, r2, fl; };
    std::vector<Stage> stages;
    const size_t stage_max =
        (size_t)(cols / b + 1) * (2 * (size_t)cols * b + 2 * (size_t)b * b) * nseg;
    const size_t flag_max = (size_t)2 * (cols / b + 1) * nseg;
    if (async) h_stage.ensure(sizeof(double) * stage_max + sizeof(int) * flag_max);
    double *hp = h_stage.ptr<double>();
    int *hflag = async ? reinterpret_cast<int *>(hp + stage_max) : nullptr;
    // The same layout on the device: the kernels write the coefficient blocks,
    // R factors and breakdown flags of every block expansion straight into it,
    // and one copy per restart cycle brings the used part to page-locked
    // memory (a copy per block would stall the stream on the copy engine).
    if (async) d_stage.ensure(sizeof(double) * stage_max + sizeof(int) * flag_max, &budget);
    double *ds = async ? d_stage.ptr<double>() : nullptr;
    int *dsflag = async ? reinterpret_cast<int *>(ds + stage_max) : nullptr;
    size_t hoff = 0, foff = 0;
    auto stage_block = [&](int c0, double *blk, double *dst) {
        Stage stg{c0, 0, 0, 0, 0, 0};
        const size_t hb = (size_t)c0 * b * nseg, rb = (size_t)b * b * nseg;
        stg.h1 = hoff;
        stg.h2 = hoff + hb;
        stg.r1 = hoff + 2 * hb;
        stg.r2 = hoff + 2 * hb + rb;
        stg.fl = foff;
        hoff += 2 * (hb + rb);
        foff += 2 * (size_t)nseg;
        const int64_t hs = (int64_t)c0 * b;            // per problem: c0 x b, ld c0
        for (int pass = 0; pass < 2; pass++) {             // CGS2 against V[:, 0:c0]
            double *h = ds + (pass ? stg.h2 : stg.h1);
            launch_gemm_tn_seg(nseg, n, c0, b, V, ldv, n, blk, ldv, n, h, hs, tnp, nparts, s);
            launch_gemm_nn_seg(nseg, n, c0, b, -1.0, V, ldv, n, h, c0, hs, 1.0, blk, ldv, n, s);
        }
        double *from = blk, *to = dst;                      // Cholesky QR, twice
        for (int pass = 0; pass < 2; pass++) {
            launch_gemm_tn_seg(nseg, n, b, b, from, ldv, n, from, ldv, n, smG, SMS, tnp, nparts, s);
            launch_small_chol_batch(nseg, b, smG, SMS, ds + (pass ? stg.r2 : stg.r1), (int64_t)b * b,
                                    smRi, SMS, dsflag + stg.fl + pass, 2, 1e-24, s);
            launch_gemm_nn_seg(nseg, n, b, b, 1.0, from, ldv, n, smRi, b, SMS, 0.0, to, ldv, n, s);
            std::swap(from, to);
        }
        launch_copy(ldv * b, from, dst, s);                 // from == blk after two passes
        stages.push_back(stg);
    };
    auto assemble_stages = [&]() {
        if (hoff > 0)
            MBL_HIP(hipMemcpyAsync(hp, ds, sizeof(double) * hoff, hipMemcpyDeviceToHost, s));
        if (foff > 0)
            MBL_HIP(hipMemcpyAsync(hflag, dsflag, sizeof(int) * foff, hipMemcpyDeviceToHost, s));
        MBL_HIP(hipStreamSynchronize(s));
        for (size_t k = 0; k < stages.size(); k++) {
            const Stage &stg = stages[k];
            const int c0 = stg.cur;
            for (int sg = 0; sg < nseg; sg++) {
                if (finished[sg] || (dropped && (*dropped)[sg])) continue;   // basis unused
                if (hflag[stg.fl + 2 * sg] || hflag[stg.fl + 2 * sg + 1])
                    throw Error(MBL_ENUMERIC, "block Krylov breakdown");
                if (c0 == 0) continue;            // the start block: no coupling to keep
                const double *h1 = hp + stg.h1 + (size_t)sg * c0 * b;
                const double *h2 = hp + stg.h2 + (size_t)sg * c0 * b;
                for (int j = 0; j < b; j++)
                    for (int i = 0; i < c0; i++) {
                        double v = h1[(size_t)j * c0 + i] + h2[(size_t)j * c0 + i];
                        Tat(sg, i, c0 - b + j) = v;
                        Tat(sg, c0 - b + j, i) = v;
                    }
                const double *R1 = hp + stg.r1 + (size_t)sg * b * b;   // R = R2 R1
                const double *R2 = hp + stg.r2 + (size_t)sg * b * b;
                for (int j = 0; j < b; j++)
                    for (int i = 0; i < b; i++) {
                        double acc = 0.0;
                        for (int q = 0; q < b; q++) acc += R2[(size_t)q * b + i] * R1[(size_t)j * b + q];
                        Tat(sg, c0 + i, c0 - b + j) = acc;
                        Tat(sg, c0 - b + j, c0 + i) = acc;
                    }
            }
        }
        stages.clear();
        hoff = 0;
        foff = 0;
    };

    result.assign(nseg, KSOut{});
    int nfinished = 0;
    std::vector<double> R, hsum;
    launch_fill_start_seg(nseg, n, b, seeds, W, ldv, s);
    if (async) {
        // the start block through the same device Cholesky QR as the expansion
        // (its coupling to an empty basis is not used)
        stage_block(0, W, V);
        assemble_stages();
    } else if (!cholqr(W, V, R)) {
        throw Error(MBL_ENUMERIC, "start block is rank deficient");
    }
    for (auto &t : T) std::fill(t.begin(), t.end(), 0.0);
    int cur = b;
    for (int restart = 0;; restart++) {
        while (async && cur < cols) {
            op(V + (int64_t)(cur - b) * ldv, W, b, finished);
            for (int sg = 0; sg < nseg; sg++)
                if (!finished[sg]) result[sg].napply += b;
            stage_block(cur, W, V + (int64_t)cur * ldv);
            cur += b;
        }
        if (async) assemble_stages();
        while (cur < cols) {
            // expand the block [cur - b, cur) into [cur, cur + b) (single problem)
            op(V + (int64_t)(cur - b) * n, W, b, finished);
            result[0].napply += b;
            project(cur, W, hsum);
            for (int j = 0; j < b; j++)
                for (int i = 0; i < cur; i++) {
                    double v = hsum[(size_t)j * cur + i];
                    Tat(0, i, cur - b + j) = v;
                    Tat(0, cur - b + j, i) = v;
                }
            bool ok = cholqr(W, V + (int64_t)cur * n, R);
            if (!ok) {
                if (b != 1) throw Error(MBL_ENUMERIC, "block Krylov breakdown");
                // invariant subspace found: continue with a fresh direction and
                // zero coupling (the Krylov relation then holds exactly)
                R.assign(1, 0.0);
                std::vector<double> R0;
                bool ok2 = false;
                if (cur < n) {
                    launch_fill_start(n, 1, seeds[0] + 977ULL * (uint64_t)(cur + 1), W, s);
                    project(cur, W, hh);
                    ok2 = cholqr(W, V + (int64_t)cur * n, R0);
                }
                if (!ok2) MBL_HIP(hipMemsetAsync(V + (int64_t)cur * n, 0, sizeof(double) * n, s));
            }
            for (int j = 0; j < b; j++)
                for (int i = 0; i < b; i++) {
                    Tat(0, cur + i, cur - b + j) = R[(size_t)j * b + i];
                    Tat(0, cur - b + j, cur + i) = R[(size_t)j * b + i];
                }
            cur += b;
        }
        // Rayleigh-Ritz on the first m columns of every running problem; the
        // last block is the residual
        const int m = cur - b;
        // problems dropped by the operator stop here, with no result
        for (int sg = 0; sg < nseg; sg++)
            if (!finished[sg] && dropped && (*dropped)[sg]) {
                finished[sg] = 1;
                nfinished++;
            }
        if (nfinished == nseg) {
            MBL_HIP(hipStreamSynchronize(s));
            return;
        }
        std::vector<int> live;
        for (int sg = 0; sg < nseg; sg++)
            if (!finished[sg]) live.push_back(sg);
        std::vector<std::vector<double>> Tm(live.size()), wall, Z;
        for (size_t q = 0; q < live.size(); q++) {
            Tm[q].resize((size_t)m * m);
            for (int j = 0; j < m; j++)
                for (int i = 0; i < m; i++) Tm[q][(size_t)j * m + i] = Tat(live[q], i, j);
        }
        small_eig_batch((int)live.size(), m, Tm, wall, Z);
        std::vector<std::vector<double>> CYs(nseg);
        std::vector<int> to_finish;
        // the restart coefficients of every problem (its kept Ritz vectors, or
        // the identity for one that finished earlier: its unused columns stay
        // orthonormal and bounded), gathered for one copy to the device
        const size_t ycount = (size_t)m * nkeep;
        h_coef.ensure(sizeof(double) * ycount * nseg);
        double *hc = h_coef.ptr<double>();
        if ((int)live.size() < nseg) {
            std::vector<char> is_live(nseg, 0);
            for (int sg : live) is_live[sg] = 1;
            for (int sg = 0; sg < nseg; sg++) {
                if (is_live[sg]) continue;
                double *I = hc + ycount * sg;
                std::fill(I, I + ycount, 0.0);
                for (int k = 0; k < nkeep; k++) I[(size_t)k * m + k] = 1.0;
            }
        }
        for (size_t q = 0; q < live.size(); q++) {
            const int sg = live[q];
            KSOut &res = result[sg];
            const std::vector<double> &w = wall[q];
            res.tmin = w.front();
            res.tmax = w.back();
            std::vector<int> order(m);
            std::iota(order.begin(), order.end(), 0);
            if (want == Want::LargestAbs) {
                std::stable_sort(order.begin(), order.end(),
                                 [&](int a, int c) { return std::fabs(w[a]) > std::fabs(w[c]); });
            } else {
                order.clear();
                for (int lo = 0, hi = m - 1; lo <= hi; lo++, hi--) {
                    order.push_back(lo);
                    if (hi != lo) order.push_back(hi);
                }
            }
            std::vector<int> sel(order.begin(), order.begin() + nkeep);
            std::vector<double> Y((size_t)m * nkeep);
            for (int k = 0; k < nkeep; k++)
                std::copy(Z[q].begin() + (size_t)sel[k] * m, Z[q].begin() + (size_t)(sel[k] + 1) * m,
                          Y.begin() + (size_t)k * m);
            res.theta.assign(nkeep, 0.0);
            res.rho.assign(nkeep, 0.0);
            std::vector<double> &CY = CYs[sg];
            CY.assign((size_t)b * nkeep, 0.0);
            for (int k = 0; k < nkeep; k++) {
                res.theta[k] = w[sel[k]];
                double acc = 0.0;
                for (int i = 0; i < b; i++) {
                    double v = 0.0;
                    for (int j = 0; j < m; j++) v += Tat(sg, m + i, j) * Y[(size_t)k * m + j];
                    CY[(size_t)k * b + i] = v;
                    acc += v * v;
                }
                res.rho[k] = std::sqrt(acc);
            }
            int nconv = 0;
            for (int k = 0; k < nwant; k++) nconv += conv(sg, res.theta[k], res.rho[k]) ? 1 : 0;
            res.nconv = nconv;
            res.restarts = restart;
            std::copy(Y.begin(), Y.end(), hc + ycount * sg);
            if (nconv == nwant || restart >= max_restarts) to_finish.push_back(sg);
        }
        MBL_HIP(hipMemcpy2DAsync(sm, sizeof(double) * SMS, hc, sizeof(double) * ycount,
                                 sizeof(double) * ycount, nseg, hipMemcpyHostToDevice, s));
        for (int sg : to_finish) {
            launch_gemm_nn_seg(1, n, m, nwant, 1.0, V + (int64_t)sg * n, ldv, 0, sm + SMS * sg, m, 0,
                               0.0, out + (int64_t)sg * n, ldv, 0, s);
            result[sg].theta.resize(nwant);
            result[sg].rho.resize(nwant);
            finished[sg] = 1;
            nfinished++;
        }
        if (nfinished == nseg) {
            MBL_HIP(hipStreamSynchronize(s));
            return;
        }
        // thick restart: kept Ritz vectors, then the residual block.  Every
        // problem moves; one that finished earlier keeps the first nkeep
        // columns of its basis (identity coefficients, copied above).
        launch_gemm_nn_seg(nseg, n, m, nkeep, 1.0, V, ldv, n, sm, m, SMS, 0.0, V2, ldv, n, s);
        launch_copy(ldv * b, V + (int64_t)m * ldv, V2 + (int64_t)nkeep * ldv, s);
        std::swap(V, V2);
        for (int sg : live) {
            if (finished[sg]) continue;
            std::fill(T[sg].begin(), T[sg].end(), 0.0);
            for (int k = 0; k < nkeep; k++) Tat(sg, k, k) = result[sg].theta[k];
            for (int k = 0; k < nkeep; k++)
                for (int i = 0; i < b; i++) {
                    Tat(sg, nkeep + i, k) = CYs[sg][(size_t)k * b + i];
                    Tat(sg, k, nkeep + i) = CYs[sg][(size_t)k * b + i];
                }
        }
        cur = nkeep + b;
        MBL_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace mbl

namespace mbl {

void Context::extremal(Plan &p, double &emin, double &emax, int &napply) {
    extremal_seg(p, d_diag.ptr<double>(), &emin, &emax, &napply);
}

void Context::extremal_seg(Plan &p, const double *diag, double *emin, double *emax,
                           int *napply) {
    const int nseg = p.nseg;
    const int64_t n = p.dim / nseg;
    int b = n >= 128 ? 4 : 1;
    int ncv = 64, nkeep = 16, nwant = 2;
    if (ncv >= n) { b = 1; ncv = (int)n; nkeep = std::max(1, (int)n - 1); nwant = std::min(2, nkeep); }
    d_psi.ensure(sizeof(double) * p.dim * nwant, &budget);
    std::vector<double> scale(nseg, 1.0);
    auto op = [&](const double *X, double *Y, int nb, const std::vector<char> &) {
        spmv(p, 0.0, nb, X, Y, diag);
    };
    std::vector<uint64_t> seeds(nseg, 0x6A09E667F3BCC909ULL);
    std::vector<KSOut> rs;
    // scale: the largest |theta| seen so far
    krylov_schur(n, nseg, b, ncv, nkeep, nwant, Want::BothEnds, op,
                 [&](int sg, double th, double rho) {
                     scale[sg] = std::max(scale[sg], std::fabs(th));
                     return rho <= 1e-12 * scale[sg];
                 },
                 300, seeds.data(), d_psi.ptr<double>(), rs);
    for (int sg = 0; sg < nseg; sg++) {
        const KSOut &r = rs[sg];
        double lo = r.tmin, hi = r.tmax;
        if (!r.theta.empty()) {
            lo = r.theta[0];
            hi = (nwant > 1) ? r.theta[1] : r.tmax;
            if (lo > hi) std::swap(lo, hi);
        }
        emin[sg] = lo;
        emax[sg] = hi;
        napply[sg] = r.napply;
        if (r.nconv < nwant && ncv < n)
            throw Error(MBL_ENOTCONV, "extremal eigenvalues did not converge");
    }
}

namespace {
int round_up(int a, int b) { return (a + b - 1) / b * b; }

void check_problem(const mbl_problem &pr) {
    MBL_REQUIRE(pr.L >= 2 && pr.L <= MBL_L_MAX, MBL_EINVAL, "L must satisfy 2 <= L <= 22");
    int64_t n = binom(pr.L, sector_nup(pr.L));
    MBL_REQUIRE(pr.nev >= 1 && pr.nev <= n, MBL_EINVAL, "nev must satisfy 1 <= nev <= dim");
    MBL_REQUIRE(std::isfinite(pr.sigma) || (pr.eps >= 0.0 && pr.eps <= 1.0), MBL_EINVAL,
                "eps must lie in [0, 1]");
    MBL_REQUIRE(pr.prec == MBL_FP64 || pr.prec == MBL_FP32_IR64, MBL_EINVAL, "unknown precision");
    MBL_REQUIRE(pr.nev <= 256, MBL_EINVAL, "nev above 256 is not supported");
}

// Basis sizes of the shift-invert iteration: nw pairs converged (a few more
// than nev, so that the selection can be certified), block b, nkeep kept at a
// restart, ncv basis columns.
struct KShape {
    int nw, b, nkeep, ncv;
};
KShape krylov_shape(int64_t n, const mbl_problem &pr) {
    KShape k;
    const int nev = pr.nev;
    k.nw = (int)std::min<int64_t>(n, nev + 2 + nev / 16);
    k.b = pr.block > 0 ? std::min(pr.block, 16) : default_block(n);
    k.nkeep = round_up(k.nw + std::max(8, k.nw / 2), k.b);
    k.ncv = pr.ncv > 0 ? round_up(pr.ncv, k.b)
                       : round_up(std::max(2 * k.nw + 2 * k.b, k.nkeep + 3 * k.b), k.b);
    if (k.ncv + k.b > n) {              // small sector: a full-space basis, vector at a time
        k.b = 1;
        k.ncv = (int)n;
        k.nkeep = std::min<int>(k.nkeep, (int)n);
    }
    k.nkeep = std::max(k.nkeep, k.nw);
    return k;
}

// The shift of the LU and the norm its refinement is measured against.  The LU
// is taken at sigma_f = sigma -+ delta: a shift that coincides with an
// eigenvalue (eps = 0 or 1 puts sigma on E_min / E_max) would make H - sigma
// singular.  delta is far below the level spacing; a few extra pairs are
// converged around sigma_f and the nev nearest sigma are selected, with a
// check that the window provably contains them.
struct Shift {
    double emin, emax, hnorm, sigma, delta, sigma_f, anorm;
};
Shift make_shift(const mbl_problem &pr, double emin, double emax) {
    Shift z;
    z.emin = emin;
    z.emax = emax;
    z.hnorm = std::max(std::fabs(emin), std::fabs(emax));
    if (z.hnorm == 0.0) z.hnorm = 1.0;
    z.sigma = std::isfinite(pr.sigma) ? pr.sigma : emin + pr.eps * (emax - emin);
    z.delta = 1e-6 * z.hnorm;
    const bool upper = std::isfinite(pr.sigma) ? true : (pr.eps >= 0.5);
    z.sigma_f = z.sigma + (upper ? z.delta : -z.delta);
    z.anorm = z.hnorm + std::fabs(z.sigma_f);
    return z;
}

// Rayleigh quotients E, squared norms nrm and squared FP64 residuals
// rr = ||H psi - E psi||^2 of the nw packed Ritz vectors of every problem of p
// (psi: p.dim x nw; diag: the diagonals of H, packed); E[s * nw + j].
void rayleigh_residuals(Context &ctx, Plan &p, const double *diag, int nw, double *psi,
                        std::vector<double> &E, std::vector<double> &nrm,
                        std::vector<double> &rr) {
    hipStream_t s = ctx.stream;
    const int nseg = p.nseg;
    const int64_t N = p.dim, n = N / nseg;
    const size_t cnt = (size_t)nseg * nw;
    ctx.d_hpsi.ensure(sizeof(double) * N * nw, &ctx.budget);
    ctx.d_e.ensure(sizeof(double) * 4 * std::max<size_t>(cnt, 256), &ctx.budget);
    const int nparts = 64;
    ctx.d_cpart.ensure(sizeof(double) * nparts * cnt, &ctx.budget);
    double *hpsi = ctx.d_hpsi.ptr<double>(), *de = ctx.d_e.ptr<double>();
    double *cp = ctx.d_cpart.ptr<double>();
    ctx.spmv(p, 0.0, nw, psi, hpsi, diag);
    launch_coldot_seg(nseg, n, nw, psi, N, psi, N, n, de + cnt, cp, nparts, s);
    launch_coldot_seg(nseg, n, nw, psi, N, hpsi, N, n, de, cp, nparts, s);
    E.resize(cnt);
    nrm.resize(cnt);
    rr.resize(cnt);
    d2h(E.data(), de, cnt, s);
    d2h(nrm.data(), de + cnt, cnt, s);
    MBL_HIP(hipStreamSynchronize(s));
    for (size_t j = 0; j < cnt; j++) E[j] /= nrm[j];
    h2d(de, E.data(), cnt, s);
    launch_sub_scaled_cols_seg(nseg, n, nw, de, psi, N, hpsi, N, s);
    launch_coldot_seg(nseg, n, nw, hpsi, N, hpsi, N, n, de + 2 * cnt, cp, nparts, s);
    d2h(rr.data(), de + 2 * cnt, cnt, s);
    MBL_HIP(hipStreamSynchronize(s));
}

// Selection of the nev pairs nearest sigma among the nw Ritz pairs of one
// problem (vectors psi, column stride ld; E, nrm, rr as above), the check that
// the window holds them, and the observables of the selected vectors into res.
// Returns the number of certified pairs.
int select_and_observe(Context &ctx, Plan &p, const mbl_problem &pr, mbl_result &res,
                       const double *psi, int64_t ld, const double *E, const double *nrm,
                       const double *rr, int nw, const Shift &z, double tol, int ks_nconv) {
    hipStream_t s = ctx.stream;
    const int64_t n = p.dim;
    const int nev = pr.nev;
    const double sigma = z.sigma, sigma_f = z.sigma_f, hnorm = z.hnorm;
    ctx.d_psi2.ensure(sizeof(double) * n * nev, &ctx.budget);
    ctx.d_e.ensure(sizeof(double) * 4 * std::max(nw, 256), &ctx.budget);
    double *de = ctx.d_e.ptr<double>();
    // the nev nearest sigma (ties: lower energy first), then ascending energy
    std::vector<int> ord(nw);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) {
        double da = std::fabs(E[a] - sigma), dc = std::fabs(E[c] - sigma);
        return da != dc ? da < dc : E[a] < E[c];
    });
    ord.resize(nev);
    // Window check: the Krylov method finds the levels nearest sigma_f first,
    // so its converged pairs cover a ball around sigma_f up to the nearest
    // pair that has not converged.  The selection (the nev nearest sigma) is
    // provably complete when it lies inside that ball.
    double unconv = HUGE_VAL, Rwin = 0.0, rsel = 0.0;
    for (int j = 0; j < nw; j++)
        if (std::sqrt(rr[j] / nrm[j]) > tol * hnorm)
            unconv = std::min(unconv, std::fabs(E[j] - sigma_f));
    for (int j = 0; j < nw; j++) {
        const double dj = std::fabs(E[j] - sigma_f);
        if (dj < unconv) Rwin = std::max(Rwin, dj);
    }
    for (int j : ord) rsel = std::max(rsel, std::fabs(E[j] - sigma));
    bool window_ok = (nw == n && ks_nconv == nw) ||
                     (rsel + z.delta <= Rwin * (1.0 + 1e-12) && rsel + z.delta < unconv);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return E[a] < E[c]; });
    std::vector<double> Es(nev), rs(nev);
    int nconv = 0;
    double maxr = 0.0;
    for (int j = 0; j < nev; j++) {
        Es[j] = E[ord[j]];
        rs[j] = std::sqrt(rr[ord[j]] / nrm[ord[j]]) / hnorm;
        launch_copy(n, psi + (int64_t)ord[j] * ld, ctx.d_psi2.ptr<double>() + (int64_t)j * n, s);
        if (rs[j] <= tol) nconv++;
        maxr = std::max(maxr, rs[j]);
    }
    if (!window_ok) nconv = std::min(nconv, nev - 1);
    // the Krylov method stopped at its restart limit: nothing is certified
    // beyond the pairs its own test accepted
    if (ks_nconv < nw) nconv = std::min(nconv, ks_nconv);
    h2d(de, Es.data(), nev, s);
    double *psis = ctx.d_psi2.ptr<double>();
    res.nconv = nconv;
    res.max_resid = maxr;
    if (res.evals) std::copy(Es.begin(), Es.end(), res.evals);
    if (res.resid) std::copy(rs.begin(), rs.end(), res.resid);

    // observables
    if (pr.flags & (MBL_WANT_OBS | MBL_WANT_OBS_EXTRA)) {
        ctx.obs.prepare(pr.L, p.basis.ptr<uint32_t>(), n, nev, &ctx.budget, s);
        ctx.d_obs.ensure(sizeof(double) * OBS_NQ * nev, &ctx.budget);
        ctx.d_r_out.ensure(sizeof(double) * std::max(1, nev), &ctx.budget);
        ctx.d_se.ensure(sizeof(double) * nev, &ctx.budget);
        ctx.obs.vector_sums(p.basis.ptr<uint32_t>(), psis, n, nev, ctx.d_obs.ptr<double>(), s);
        ctx.obs.gap_ratios(nev, de, ctx.d_r_out.ptr<double>(), s);
        std::vector<double> q((size_t)OBS_NQ * nev), rv(std::max(1, nev - 2)), se(nev);
        bool want_se = res.se != nullptr;
        if (want_se)
            ctx.obs.entanglement(psis, n, nev, ctx.obs.norms_dev(), ctx.d_se.ptr<double>(), s);
        d2h(q.data(), ctx.d_obs.ptr<double>(), q.size(), s);
        if (nev >= 3) d2h(rv.data(), ctx.d_r_out.ptr<double>(), nev - 2, s);
        if (want_se) d2h(se.data(), ctx.d_se.ptr<double>(), nev, s);
        MBL_HIP(hipStreamSynchronize(s));
        if (want_se)
            for (int j = 0; j < nev; j++)
                if (!std::isfinite(se[j]))
                    throw Error(MBL_ENUMERIC, "entanglement: non-finite result");
        double rsum = 0.0;
        int rcnt = 0;
        for (int j = 0; j + 2 < nev; j++)
            if (!std::isnan(rv[j])) { rsum += rv[j]; rcnt++; }
        res.r_mean = rcnt ? rsum / rcnt : NAN;
        if (res.r && nev >= 3) std::copy(rv.begin(), rv.begin() + (nev - 2), res.r);
        for (int j = 0; j < nev; j++) {
            const double *c = &q[(size_t)j * OBS_NQ];
            if (res.s1) res.s1[j] = c[1];
            if (res.se) res.se[j] = se[j];
            if (pr.flags & MBL_WANT_OBS_EXTRA) {
                if (res.s2) res.s2[j] = -std::log(c[2]);
                if (res.fluct) res.fluct[j] = c[4] - c[3] * c[3];
                if (res.dynfrac) res.dynfrac[j] = 1.0 - (c[5] * c[5] + c[6] * c[6]) / c[7];
                if (res.kl && j + 1 < nev) res.kl[j] = c[8];
            }
        }
    }
    if ((pr.flags & MBL_WANT_VECTORS) && res.evecs) {
        d2h(res.evecs, psis, (size_t)n * nev, s);
        MBL_HIP(hipStreamSynchronize(s));
    }
    return nconv;
}

void set_shift(mbl_result &res, const Shift &z) {
    res.emin = z.emin;
    res.emax = z.emax;
    res.sigma = z.sigma;
    res.hnorm = z.hnorm;
}

const uint32_t HOOKS = MBL_HOOK_IR_STALL32 | MBL_HOOK_IR_STALL64 | MBL_HOOK_NO_CONV;
const uint64_t KRYLOV_SEED = 0xA5A5A5A5A5A5A5A5ULL;   // xor-ed with the disorder seed
}  // namespace

void solve_problem(Context &ctx, const mbl_problem &pr, mbl_result &res, const double *extremal) {
    check_problem(pr);
    const int64_t n = binom(pr.L, sector_nup(pr.L));
    // test hooks of this request, cleared however the request ends
    struct HookScope {
        Context &c;
        HookScope(Context &cx, const mbl_problem &q) : c(cx) {
            c.hooks = q.flags & HOOKS;
            c.budget.armed = q.fail_alloc_bytes;
            c.budget.since_armed = 0;
            c.refine_target = Context::eig_refine_target(q.tol > 0 ? q.tol : 1e-10);
        }
        ~HookScope() {
            c.hooks = 0; c.budget.armed = 0; c.budget.since_armed = 0;
            c.refine_target = Context::SOLVE_TARGET;
        }
    } hook_scope(ctx, pr);
    double tol = pr.tol > 0 ? pr.tol : 1e-10;
    double t_start = wall_seconds(), t0 = t_start;
    std::memset(res.t_phase, 0, sizeof(res.t_phase));

    const int64_t passes0 = ctx.lu_passes, pass_rhs0 = ctx.lu_pass_rhs;
    Plan &p = ctx.plan(pr.L);
    ctx.set_realization(p, pr.J, pr.fields, pr.h, pr.seed, pr.fields == nullptr);
    res.t_phase[0] = wall_seconds() - t0;

    t0 = wall_seconds();
    double emin = 0, emax = 0;
    int nap = 0;
    if (extremal) { emin = extremal[0]; emax = extremal[1]; }
    else ctx.extremal(p, emin, emax, nap);
    const Shift z = make_shift(pr, emin, emax);
    ctx.hnorm_ = z.hnorm;
    set_shift(res, z);
    res.t_phase[1] = wall_seconds() - t0;

    t0 = wall_seconds();
    ctx.ensure_symbolic(p);
    res.t_phase[2] = wall_seconds() - t0;

    t0 = wall_seconds();
    SolveStats st;
    int prec = pr.prec;
    ctx.factor(p, prec, z.sigma_f, z.anorm, st);
    res.t_phase[3] = wall_seconds() - t0;

    // block Krylov-Schur on (H - sigma_f)^-1
    t0 = wall_seconds();
    const KShape k = krylov_shape(n, pr);
    int max_restarts = pr.max_restarts > 0 ? pr.max_restarts : 300;
    ctx.d_psi.ensure(sizeof(double) * n * k.nw, &ctx.budget);
    bool fell_back = false;
    auto op = [&](const double *X, double *Y, int nb, const std::vector<char> &) {
        try {
            ctx.shift_solve(p, prec, nb, X, Y, st);
            if (prec == MBL_FP32_IR64 && st.gmres_inner > 8) {
                // the FP32 factor needs many GMRES steps per solve here (kappa u_32
                // near one): this result stands, later solves use an FP64 factor
                prec = MBL_FP64;
                fell_back = true;
                SolveStats s2;
                ctx.factor(p, prec, z.sigma_f, z.anorm, s2);
            }
        } catch (const Error &e) {
            if (e.code != MBL_ENUMERIC || prec != MBL_FP32_IR64) throw;
            // FP32 refinement did not reach the target: refactor in FP64
            prec = MBL_FP64;
            fell_back = true;
            SolveStats s2;
            ctx.factor(p, prec, z.sigma_f, z.anorm, s2);
            ctx.shift_solve(p, prec, nb, X, Y, st);
        }
    };
    const bool never_conv = (ctx.hooks & MBL_HOOK_NO_CONV) != 0;
    auto conv = [&](int, double th, double rho) {
        return !never_conv && th != 0.0 && rho * z.anorm <= 0.1 * tol * z.hnorm * std::fabs(th);
    };
    uint64_t kseed = pr.seed ^ KRYLOV_SEED;
    std::vector<Context::KSOut> kss;
    ctx.krylov_schur(n, 1, k.b, k.ncv, k.nkeep, k.nw, Context::Want::LargestAbs, op, conv,
                     max_restarts, &kseed, ctx.d_psi.ptr<double>(), kss);
    const Context::KSOut &ks = kss[0];
    res.t_phase[4] = wall_seconds() - t0;
    res.t_phase[7] = st.t_solve;
    res.n_restarts = ks.restarts;
    res.n_opapply = ks.napply;
    res.n_passes = (int)(ctx.lu_passes - passes0);
    res.n_pass_rhs = (int)(ctx.lu_pass_rhs - pass_rhs0);
    res.ir_iters_max = st.ir_iters;
    res.n_perturbed = st.n_perturbed;
    res.fallback = fell_back ? 1 : 0;
    res.batch = 1;

    // energies (Rayleigh quotients) and FP64 residuals ||H psi - E psi||, the
    // selection and the observables
    t0 = wall_seconds();
    std::vector<double> E, nrm, rr;
    rayleigh_residuals(ctx, p, ctx.d_diag.ptr<double>(), k.nw, ctx.d_psi.ptr<double>(), E, nrm, rr);
    int nconv = select_and_observe(ctx, p, pr, res, ctx.d_psi.ptr<double>(), n, E.data(),
                                   nrm.data(), rr.data(), k.nw, z, tol, ks.nconv);
    res.t_phase[5] = wall_seconds() - t0;
    res.t_phase[6] = wall_seconds() - t_start;
    if (nconv < pr.nev)
        throw Error(MBL_ENOTCONV, "only " + std::to_string(nconv) + " of " +
                                      std::to_string(pr.nev) + " pairs reached tol");
}

bool batchable(const mbl_problem *prs, int count) {
    if (count < 2 || count > MBL_SEG_MAX) return false;
    const mbl_problem &a = prs[0];
    if (a.L < 2 || a.L > MBL_L_MAX) return false;
    const int64_t n = binom(a.L, sector_nup(a.L));
    // block iterations throughout (extremal energies and shift-invert)
    if (n < 128) return false;
    for (int q = 0; q < count; q++) {
        const mbl_problem &c = prs[q];
        if (c.L != a.L || c.J != a.J || c.nev != a.nev || c.prec != a.prec || c.tol != a.tol ||
            c.block != a.block || c.ncv != a.ncv || c.max_restarts != a.max_restarts)
            return false;
        // the refinement-stall hooks are followed inside a batch (the problem
        // leaves it); the others are not
        if ((c.flags & MBL_HOOK_NO_CONV) || c.fail_alloc_bytes) return false;
        if (c.nev < 1 || c.nev > std::min<int64_t>(n, 256)) return false;
    }
    return krylov_shape(n, a).b > 1;
}

bool solve_batch(Context &ctx, int count, const mbl_problem *prs, mbl_result *res, int *status) {
    if (!batchable(prs, count)) return false;
    for (int q = 0; q < count; q++) check_problem(prs[q]);
    const mbl_problem &a = prs[0];
    const int L = a.L, nseg = count;
    const int64_t n = binom(L, sector_nup(L)), N = n * nseg;
    const double tol = a.tol > 0 ? a.tol : 1e-10;
    const int prec = a.prec;
    hipStream_t s = ctx.stream;
    struct TargetScope {                   // refinement target of these requests
        Context &c;
        TargetScope(Context &cx, double tol) : c(cx) { c.refine_target = Context::eig_refine_target(tol); }
        ~TargetScope() { c.refine_target = Context::SOLVE_TARGET; }
    } target_scope(ctx, tol);
    try {
        double t_start = wall_seconds(), t0 = t_start;
        double tph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        Plan &p = ctx.plan(L);
        ctx.ensure_symbolic(p);
        Plan &bp = ctx.batch_plan(L, nseg);
        // diagonals of every problem, packed
        ctx.d_bdiag.ensure(sizeof(double) * N, &ctx.budget);
        ctx.d_bshift.ensure(sizeof(double) * N, &ctx.budget);
        for (int q = 0; q < nseg; q++) {
            const mbl_problem &c = prs[q];
            ctx.set_realization(p, c.J, c.fields, c.h, c.seed, c.fields == nullptr);
            launch_copy(n, ctx.d_diag.ptr<double>(), ctx.d_bdiag.ptr<double>() + q * n, s);
        }
        tph[0] = wall_seconds() - t0;

        t0 = wall_seconds();
        std::vector<double> emin(nseg), emax(nseg);
        std::vector<int> nap(nseg);
        ctx.extremal_seg(bp, ctx.d_bdiag.ptr<double>(), emin.data(), emax.data(), nap.data());
        std::vector<Shift> z(nseg);
        std::vector<double> anorm(nseg);
        SegVals sf{};
        for (int q = 0; q < nseg; q++) {
            z[q] = make_shift(prs[q], emin[q], emax[q]);
            anorm[q] = z[q].anorm;
            sf.v[q] = z[q].sigma_f;
        }
        tph[1] = wall_seconds() - t0;

        t0 = wall_seconds();
        launch_shift_seg(nseg, n, ctx.d_bdiag.ptr<double>(), sf, ctx.d_bshift.ptr<double>(), s);
        SolveStats st;
        ctx.factor_batch(bp, prec, ctx.d_bshift.ptr<double>(), anorm, st);
        tph[3] = wall_seconds() - t0;

        // block Krylov-Schur on every (H_s - sigma_f,s)^-1
        t0 = wall_seconds();
        const KShape k = krylov_shape(n, a);
        const int max_restarts = a.max_restarts > 0 ? a.max_restarts : 300;
        ctx.d_psi.ensure(sizeof(double) * N * k.nw, &ctx.budget);
        Context::BatchSolveStats bs(nseg);
        for (int q = 0; q < nseg; q++)
            bs.hooks[q] = prs[q].flags & (MBL_HOOK_IR_STALL32 | MBL_HOOK_IR_STALL64);
        auto op = [&](const double *X, double *Y, int nb, const std::vector<char> &finished) {
            ctx.shift_solve_batch(bp, prec, nb, X, Y, ctx.d_bshift.ptr<double>(), anorm, finished, bs);
        };
        // dropped problems whose extremal energies are known need not wait for
        // the Krylov run: they are solved alone at the end
        auto conv = [&](int sg, double th, double rho) {
            return th != 0.0 && rho * z[sg].anorm <= 0.1 * tol * z[sg].hnorm * std::fabs(th);
        };
        std::vector<uint64_t> seeds(nseg);
        for (int q = 0; q < nseg; q++) seeds[q] = prs[q].seed ^ KRYLOV_SEED;
        std::vector<Context::KSOut> kss;
        ctx.krylov_schur(n, nseg, k.b, k.ncv, k.nkeep, k.nw, Context::Want::LargestAbs, op, conv,
                         max_restarts, seeds.data(), ctx.d_psi.ptr<double>(), kss, &bs.dropped);
        tph[4] = wall_seconds() - t0;
        tph[7] = bs.t_solve;

        t0 = wall_seconds();
        std::vector<double> E, nrm, rr;
        rayleigh_residuals(ctx, bp, ctx.d_bdiag.ptr<double>(), k.nw, ctx.d_psi.ptr<double>(), E, nrm,
                           rr);
        std::vector<int> nconv(nseg);
        for (int q = 0; q < nseg; q++) {
            if (bs.dropped[q]) continue;
            mbl_result &r = res[q];
            set_shift(r, z[q]);
            r.n_restarts = kss[q].restarts;
            r.n_opapply = kss[q].napply;
            r.n_passes = bs.passes[q];
            r.n_pass_rhs = bs.pass_rhs[q];
            r.ir_iters_max = bs.ir_iters[q];
            r.n_perturbed = st.perturbed[q];
            r.fallback = 0;
            r.batch = nseg;
            const size_t o = (size_t)q * k.nw;
            nconv[q] = select_and_observe(ctx, p, prs[q], r, ctx.d_psi.ptr<double>() + q * n, N,
                                          E.data() + o, nrm.data() + o, rr.data() + o, k.nw, z[q],
                                          tol, kss[q].nconv);
        }
        tph[5] = wall_seconds() - t0;
        tph[6] = wall_seconds() - t_start;
        int ndropped = 0;
        for (int q = 0; q < nseg; q++) {
            if (bs.dropped[q]) { ndropped++; continue; }
            std::copy(tph, tph + 8, res[q].t_phase);
            status[q] = nconv[q] < prs[q].nev ? MBL_ENOTCONV : MBL_OK;
        }
        if (ndropped) {
            // the dropped problems alone, on fresh buffers (those of the batch
            // are given back first)
            ctx.trim();
            for (int q = 0; q < nseg; q++) {
                if (!bs.dropped[q]) continue;
                try {
                    solve_problem(ctx, prs[q], res[q]);
                    status[q] = MBL_OK;
                } catch (const Error &e) {
                    set_last_error(e.what());
                    status[q] = e.code;
                }
            }
        }
    } catch (const Error &e) {
        if (e.code != MBL_ENOMEM) throw;
        // the batch's buffers do not fit: the problems go alone, on fresh buffers
        ctx.trim();
        return false;
    }
    return true;
}

}  // namespace mbl
