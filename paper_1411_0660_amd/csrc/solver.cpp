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
                      &d_part, &d_V, &d_V2, &d_W, &d_small, &d_ritz, &d_tnpart, &d_gV, &d_gZ, &d_gpart,
                      &d_gcoef, &d_psi, &d_psi2, &d_hpsi, &d_e, &d_cpart, &d_obs, &d_r_out,
                      &d_se})
        b->reset();
    for (DevBuf *b : {&f32_.uinv, &f64_.uinv}) b->reset();
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
    FrontTree &t = p.tree;
    int nf = (int)t.fronts.size();
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
                rb.push_back(cdiv64(d.m - k1, TRSM_L_ROWS));
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

void Context::spmv(Plan &p, double shift, int nvec, const double *x, double *y) {
    bool pr = prof_on("spmv");
    if (pr) prof_begin();
    launch_spmv(p.dim, p.rowptr.ptr<int32_t>(), p.col.ptr<int32_t>(), d_diag.ptr<double>(), offv,
                shift, nvec, x, y, stream);
    // per vector: columns (4 B/nnz), rowptr, diagonal, x gathered, y written
    if (pr) prof_end(4.0 * p.nnz + 4.0 * p.dim + 8.0 * p.dim + nvec * 16.0 * p.dim,
                     2.0 * nvec * (double)p.nnz);
}

// ---------------------------------------------------------------- factor

template <class T>
void Context::factor_t(Plan &p, Factor<T> &f, double sigma, double thresh_rel, SolveStats &st) {
    hipStream_t s = stream;
    if (f.L != p.L) {
        // invalid until every buffer is in place: an allocation that throws
        // part way must not leave buffers of another size behind a valid L
        f.L = -1;
        f.valid = false;
        f.arena.reset();
        f.arena.alloc(sizeof(T) * p.arena_elems, &budget);
        f.ipiv.alloc(sizeof(int32_t) * std::max<int64_t>(1, p.dim), &budget);
        f.prow.alloc(sizeof(int32_t) * std::max<int64_t>(1, p.dim), &budget);
        f.npert.alloc(sizeof(int32_t), &budget);
        f.uinv.alloc(sizeof(double) * FNB * FNB * std::max<size_t>(1, p.h_fd.size()), &budget);
        f.L = p.L;
    }
    f.valid = false;
    MBL_HIP(hipMemsetAsync(f.npert.template ptr<int32_t>(), 0, sizeof(int32_t), s));
    T *A = f.arena.template ptr<T>();
    const FrontDesc *fd = p.d_fd.ptr<FrontDesc>();
    double thresh = thresh_rel * anorm_;
    for (size_t l = 0; l < p.levels.size(); l++) {
        LevelTasks &lv = p.levels[l];
        launch_front_pull<T>(A, fd, p.d_pullmap.ptr<int32_t>(), p.d_child_ids.ptr<int32_t>(),
                             lv.pull, s);
        launch_front_assemble<T>(A, fd, lv.ecount, p.d_efront.ptr<int32_t>() + lv.ebegin,
                                 p.d_epos.ptr<int32_t>() + lv.ebegin,
                                 p.d_esrc.ptr<int32_t>() + lv.ebegin, d_diag.ptr<double>(), sigma,
                                 offv, s);
        for (size_t t = 0; t < lv.steps.size(); t++) {
            StepTasks &S = lv.steps[t];
            launch_panel<T>(A, fd, f.ipiv.template ptr<int32_t>(), f.npert.template ptr<int32_t>(),
                            S.panel, (int)t, thresh, f.uinv.template ptr<double>(), s);
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
    int32_t np = 0;
    d2h(&np, f.npert.template ptr<int32_t>(), 1, s);
    MBL_HIP(hipStreamSynchronize(s));
    st.n_perturbed = np;
    f.valid = true;
    f.sigma = sigma;
}

void Context::factor(Plan &p, int prec, double sigma, double anorm, SolveStats &st) {
    ensure_symbolic(p);
    anorm_ = anorm;
    double t0 = wall_seconds();
    if (prec == MBL_FP32_IR64) factor_t<float>(p, f32_, sigma, 1e-7, st);
    else factor_t<double>(p, f64_, sigma, 1e-14, st);
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
    if (!use_graphs_ || timed || ldb != n || ldx != n) {
        lu_apply_seq<T>(p, f, nrhs, b, ldb, x, ldx);
        return;
    }
    // The launch sequence of one application is the same every time for a
    // given plan, factor, right-hand-side count and work buffers: it is
    // captured once as a graph between fixed staging vectors and replayed.
    d_vec.ensure(sizeof(double) * std::max<int64_t>(1, p.vec_elems), &budget);
    d_yv.ensure(sizeof(double) * std::max<int64_t>(1, p.y_elems), &budget);
    d_upart.ensure(sizeof(double) * std::max<int64_t>(1, p.part_elems), &budget);
    d_xnew.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_gin.ensure(sizeof(double) * n * MAXRHS, &budget);
    d_gout.ensure(sizeof(double) * n * MAXRHS, &budget);
    GraphKey key{p.L, (int)sizeof(T), nrhs,
                 {f.arena.template ptr<void>(), f.prow.template ptr<void>(), d_vec.ptr<void>(),
                  d_yv.ptr<void>(),
                  d_upart.ptr<void>(), d_xnew.ptr<void>(), d_gin.ptr<void>(), d_gout.ptr<void>()}};
    auto it = graphs_.find(key);
    if (it == graphs_.end()) {
        if (graphs_.size() >= 32) clear_graphs();
        hipGraph_t g = nullptr;
        MBL_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            lu_apply_seq<T>(p, f, nrhs, d_gin.ptr<double>(), n, d_gout.ptr<double>(), n);
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
void Context::lu_apply_seq(Plan &p, Factor<T> &f, int nrhs, const double *b, int64_t ldb,
                           double *x, int64_t ldx) {
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
        launch_fwd_l21<T>(A, fd, lv.l21, nrhs, vec, part, s);
        if (pr) prof_end(lv.l21.elems * sizeof(T) + 8.0 * nrhs * lv.l21.rows, 2.0 * nrhs * lv.l21.elems);
        launch_fwd_l21_reduce(fd, lv.l21red, nrhs, vec, part, s);
    }
    for (size_t l = p.levels.size(); l-- > 0;) {
        LevelTasks &lv = p.levels[l];
        bool pr = prof_on("u12") && lv.u12.total > 0;
        if (pr) prof_begin();
        launch_bwd_u12<T>(A, fd, lv.u12, nrhs, p.d_contrib.ptr<int32_t>(), xnew, p.dim, part, s);
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
    const double target = 1e-13;

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

// ---------------------------------------------------------------- Krylov-Schur

// All eigenpairs of the symmetric m x m matrix A (host, column-major) by the
// device Jacobi kernel: w ascending, Z (m x m) the unit eigenvectors in the
// same order.
void Context::small_eig(int m, const std::vector<double> &A, std::vector<double> &w,
                        std::vector<double> &Z) {
    hipStream_t s = stream;
    const size_t mm = (size_t)m * m;
    d_ritz.ensure(sizeof(double) * (2 * mm + m + 1), &budget);
    double *dA = d_ritz.ptr<double>(), *dV = dA + mm, *dw = dV + mm;
    int *dinfo = reinterpret_cast<int *>(dw + m);
    double fro = 0.0;
    for (double x : A) fro += x * x;
    fro = std::sqrt(fro);
    h2d(dA, A.data(), mm, s);
    // off-diagonal entries at or below 1e-17 ||A||_F are left in place: their
    // effect on the eigenvalues is below the rounding of ||A||
    launch_jacobi_eig(m, dA, dV, dw, dinfo, 1e-17 * fro, s);
    std::vector<double> wu(m), Vu(mm);
    int info = 0;
    d2h(wu.data(), dw, m, s);
    d2h(Vu.data(), dV, mm, s);
    d2h(&info, dinfo, 1, s);
    MBL_HIP(hipStreamSynchronize(s));
    if (info < 0) throw Error(MBL_ENUMERIC, "Jacobi eigensolver: sweep limit reached");
    if (debug_level() > 1) std::fprintf(stderr, "[mbl] jacobi m=%d sweeps=%d\n", m, info);
    std::vector<int> perm(m);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return wu[a] < wu[c]; });
    w.resize(m);
    Z.resize(mm);
    for (int j = 0; j < m; j++) {
        w[j] = wu[perm[j]];
        std::copy(Vu.begin() + (size_t)perm[j] * m, Vu.begin() + (size_t)(perm[j] + 1) * m,
                  Z.begin() + (size_t)j * m);
    }
}

Context::KSOut Context::krylov_schur(int64_t n, int b, int ncv, int nkeep, int nwant, Want want,
                                     const std::function<void(const double *, double *, int)> &op,
                                     const std::function<bool(double, double)> &conv,
                                     int max_restarts, uint64_t seed, double *out) {
    hipStream_t s = stream;
    const int cols = ncv + b;
    const bool full = (ncv >= n);   // the basis can span the whole space
    MBL_REQUIRE(nwant <= nkeep && nkeep <= ncv && ncv % b == 0 && (full || nkeep + b <= ncv) &&
                    (full || nkeep % b == 0) && (!full || b == 1),
                MBL_EINVAL, "krylov_schur: inconsistent basis sizes");
    d_V.ensure(sizeof(double) * n * cols, &budget);
    d_V2.ensure(sizeof(double) * n * cols, &budget);
    d_W.ensure(sizeof(double) * n * b, &budget);
    d_small.ensure(sizeof(double) * (size_t)cols * std::max(cols, b) * 2, &budget);
    int nparts = gemm_tn_parts(n);
    d_tnpart.ensure(sizeof(double) * (size_t)nparts * cols * b, &budget);
    double *V = d_V.ptr<double>(), *V2 = d_V2.ptr<double>(), *W = d_W.ptr<double>();
    double *sm = d_small.ptr<double>();
    double *tnp = d_tnpart.ptr<double>();
    std::vector<double> T((size_t)cols * cols, 0.0);
    auto Tat = [&](int i, int j) -> double & { return T[(size_t)j * cols + i]; };

    // classical Gram-Schmidt, twice, of blk against V[:, 0:c0]; coefficients summed
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
    // dst = src R^-1 (Cholesky QR, two passes); src is used as scratch
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
    // projected matrix is assembled once per restart cycle.
    const bool async = (b > 1);
    struct Stage { int cur; size_t h1, h2, r1, r2; };
    std::vector<Stage> stages;
    const size_t stage_max = (size_t)(cols / b + 1) * (2 * (size_t)cols * b + 2 * (size_t)b * b);
    double *smG = sm + (size_t)cols * std::max(cols, b), *smR = smG + b * b, *smRi = smR + b * b;
    int *dflag = reinterpret_cast<int *>(smRi + b * b);
    if (async) h_stage.ensure(sizeof(double) * stage_max + sizeof(int) * 2 * (cols / b + 1));
    double *hp = h_stage.ptr<double>();
    int *hflag = async ? reinterpret_cast<int *>(hp + stage_max) : nullptr;
    size_t hoff = 0;
    auto stage_block = [&](int c0, double *blk, double *dst) {
        Stage stg{c0, 0, 0, 0, 0};
        const int k = (int)stages.size();
        for (int pass = 0; pass < 2; pass++) {             // CGS2 against V[:, 0:c0]
            launch_gemm_tn(n, c0, b, V, n, blk, n, sm, tnp, nparts, s);
            launch_gemm_nn(n, c0, b, -1.0, V, n, sm, c0, 1.0, blk, n, s);
            (pass ? stg.h2 : stg.h1) = hoff;
            MBL_HIP(hipMemcpyAsync(hp + hoff, sm, sizeof(double) * c0 * b,
                                   hipMemcpyDeviceToHost, s));
            hoff += (size_t)c0 * b;
        }
        double *from = blk, *to = dst;                      // Cholesky QR, twice
        for (int pass = 0; pass < 2; pass++) {
            launch_gemm_tn(n, b, b, from, n, from, n, smG, tnp, nparts, s);
            launch_small_chol(b, smG, smR, smRi, dflag + pass, 1e-24, s);
            (pass ? stg.r2 : stg.r1) = hoff;
            MBL_HIP(hipMemcpyAsync(hp + hoff, smR, sizeof(double) * b * b, hipMemcpyDeviceToHost,
                                   s));
            hoff += (size_t)b * b;
            launch_gemm_nn(n, b, b, 1.0, from, n, smRi, b, 0.0, to, n, s);
            std::swap(from, to);
        }
        launch_copy(n * b, from, dst, s);                   // from == blk after two passes
        MBL_HIP(hipMemcpyAsync(hflag + 2 * k, dflag, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
        stages.push_back(stg);
    };
    auto assemble_stages = [&]() {
        MBL_HIP(hipStreamSynchronize(s));
        for (size_t k = 0; k < stages.size(); k++) {
            const Stage &stg = stages[k];
            if (hflag[2 * k] || hflag[2 * k + 1]) throw Error(MBL_ENUMERIC, "block Krylov breakdown");
            const int c0 = stg.cur;
            for (int j = 0; j < b; j++)
                for (int i = 0; i < c0; i++) {
                    double v = hp[stg.h1 + (size_t)j * c0 + i] + hp[stg.h2 + (size_t)j * c0 + i];
                    Tat(i, c0 - b + j) = v;
                    Tat(c0 - b + j, i) = v;
                }
            const double *R1 = hp + stg.r1, *R2 = hp + stg.r2;   // R = R2 R1
            for (int j = 0; j < b; j++)
                for (int i = 0; i < b; i++) {
                    double acc = 0.0;
                    for (int q = 0; q < b; q++) acc += R2[(size_t)q * b + i] * R1[(size_t)j * b + q];
                    Tat(c0 + i, c0 - b + j) = acc;
                    Tat(c0 - b + j, c0 + i) = acc;
                }
        }
        stages.clear();
        hoff = 0;
    };

    KSOut res;
    std::vector<double> R, hsum;
    launch_fill_start(n, b, seed, W, s);
    if (!cholqr(W, V, R)) throw Error(MBL_ENUMERIC, "start block is rank deficient");
    int cur = b;
    for (int restart = 0;; restart++) {
        while (async && cur < cols) {
            op(V + (int64_t)(cur - b) * n, W, b);
            res.napply += b;
            stage_block(cur, W, V + (int64_t)cur * n);
            cur += b;
        }
        if (async) assemble_stages();
        while (cur < cols) {
            // expand the block [cur - b, cur) into [cur, cur + b)
            op(V + (int64_t)(cur - b) * n, W, b);
            res.napply += b;
            project(cur, W, hsum);
            for (int j = 0; j < b; j++)
                for (int i = 0; i < cur; i++) {
                    double v = hsum[(size_t)j * cur + i];
                    Tat(i, cur - b + j) = v;
                    Tat(cur - b + j, i) = v;
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
                    launch_fill_start(n, 1, seed + 977ULL * (uint64_t)(cur + 1), W, s);
                    project(cur, W, hh);
                    ok2 = cholqr(W, V + (int64_t)cur * n, R0);
                }
                if (!ok2) MBL_HIP(hipMemsetAsync(V + (int64_t)cur * n, 0, sizeof(double) * n, s));
            }
            for (int j = 0; j < b; j++)
                for (int i = 0; i < b; i++) {
                    Tat(cur + i, cur - b + j) = R[(size_t)j * b + i];
                    Tat(cur - b + j, cur + i) = R[(size_t)j * b + i];
                }
            cur += b;
        }
        // Rayleigh-Ritz on the first m columns; the last block is the residual
        int m = cur - b;
        std::vector<double> Tm((size_t)m * m), C((size_t)b * m);
        for (int j = 0; j < m; j++) {
            for (int i = 0; i < m; i++) Tm[(size_t)j * m + i] = Tat(i, j);
            for (int i = 0; i < b; i++) C[(size_t)j * b + i] = Tat(m + i, j);
        }
        std::vector<double> wall, Z, Y;
        small_eig(m, Tm, wall, Z);
        res.tmin = wall.front();
        res.tmax = wall.back();
        std::vector<int> order(m);
        std::iota(order.begin(), order.end(), 0);
        if (want == Want::LargestAbs) {
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int c) { return std::fabs(wall[a]) > std::fabs(wall[c]); });
        } else {
            order.clear();
            for (int lo = 0, hi = m - 1; lo <= hi; lo++, hi--) {
                order.push_back(lo);
                if (hi != lo) order.push_back(hi);
            }
        }
        std::vector<int> sel(order.begin(), order.begin() + nkeep);
        Y.resize((size_t)m * nkeep);
        for (int q = 0; q < nkeep; q++)
            std::copy(Z.begin() + (size_t)sel[q] * m, Z.begin() + (size_t)(sel[q] + 1) * m,
                      Y.begin() + (size_t)q * m);
        const std::vector<double> &w = wall;
        res.theta.assign(nkeep, 0.0);
        res.rho.assign(nkeep, 0.0);
        std::vector<double> CY((size_t)b * nkeep, 0.0);
        for (int q = 0; q < nkeep; q++) {
            res.theta[q] = w[sel[q]];
            double acc = 0.0;
            for (int i = 0; i < b; i++) {
                double v = 0.0;
                for (int j = 0; j < m; j++) v += C[(size_t)j * b + i] * Y[(size_t)q * m + j];
                CY[(size_t)q * b + i] = v;
                acc += v * v;
            }
            res.rho[q] = std::sqrt(acc);
        }
        int nconv = 0;
        for (int q = 0; q < nwant; q++) nconv += conv(res.theta[q], res.rho[q]) ? 1 : 0;
        res.nconv = nconv;
        res.restarts = restart;
        bool done = (nconv == nwant) || restart >= max_restarts;
        h2d(sm, Y.data(), Y.size(), s);
        if (done) {
            launch_gemm_nn(n, m, nwant, 1.0, V, n, sm, m, 0.0, out, n, s);
            MBL_HIP(hipStreamSynchronize(s));
            res.theta.resize(nwant);
            res.rho.resize(nwant);
            return res;
        }
        // thick restart: kept Ritz vectors, then the residual block
        launch_gemm_nn(n, m, nkeep, 1.0, V, n, sm, m, 0.0, V2, n, s);
        launch_copy(n * b, V + (int64_t)m * n, V2 + (int64_t)nkeep * n, s);
        std::swap(V, V2);
        std::fill(T.begin(), T.end(), 0.0);
        for (int q = 0; q < nkeep; q++) Tat(q, q) = res.theta[q];
        for (int q = 0; q < nkeep; q++)
            for (int i = 0; i < b; i++) {
                Tat(nkeep + i, q) = CY[(size_t)q * b + i];
                Tat(q, nkeep + i) = CY[(size_t)q * b + i];
            }
        cur = nkeep + b;
        MBL_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace mbl

namespace mbl {

void Context::extremal(Plan &p, double &emin, double &emax, int &napply) {
    int64_t n = p.dim;
    int b = n >= 128 ? 4 : 1;
    int ncv = 64, nkeep = 16, nwant = 2;
    if (ncv >= n) { b = 1; ncv = (int)n; nkeep = std::max(1, (int)n - 1); nwant = std::min(2, nkeep); }
    d_psi.ensure(sizeof(double) * n * nwant, &budget);
    double scale = 1.0;
    auto op = [&](const double *X, double *Y, int nb) { spmv(p, 0.0, nb, X, Y); };
    auto conv = [&](double th, double rho) { return rho <= 1e-12 * scale; };
    // scale from a first pass: |theta| extremes
    scale = 1.0;
    KSOut r = krylov_schur(n, b, ncv, nkeep, nwant, Want::BothEnds, op,
                           [&](double th, double rho) {
                               scale = std::max(scale, std::fabs(th));
                               return conv(th, rho);
                           },
                           300, 0x6A09E667F3BCC909ULL, d_psi.ptr<double>());
    emin = std::min(r.tmin, r.theta.empty() ? r.tmin : r.theta[0]);
    emax = std::max(r.tmax, r.theta.empty() ? r.tmax : r.theta.back());
    if (!r.theta.empty()) {
        emin = r.theta[0];
        emax = (nwant > 1) ? r.theta[1] : r.tmax;
        if (emin > emax) std::swap(emin, emax);
    }
    napply = r.napply;
    if (r.nconv < nwant && ncv < n)
        throw Error(MBL_ENOTCONV, "extremal eigenvalues did not converge");
}

namespace {
int round_up(int a, int b) { return (a + b - 1) / b * b; }
}

void solve_problem(Context &ctx, const mbl_problem &pr, mbl_result &res, const double *extremal) {
    MBL_REQUIRE(pr.L >= 2 && pr.L <= MBL_L_MAX, MBL_EINVAL, "L must satisfy 2 <= L <= 22");
    int64_t n = binom(pr.L, sector_nup(pr.L));
    MBL_REQUIRE(pr.nev >= 1 && pr.nev <= n, MBL_EINVAL, "nev must satisfy 1 <= nev <= dim");
    MBL_REQUIRE(std::isfinite(pr.sigma) || (pr.eps >= 0.0 && pr.eps <= 1.0), MBL_EINVAL,
                "eps must lie in [0, 1]");
    MBL_REQUIRE(pr.prec == MBL_FP64 || pr.prec == MBL_FP32_IR64, MBL_EINVAL, "unknown precision");
    MBL_REQUIRE(pr.nev <= 256, MBL_EINVAL, "nev above 256 is not supported");
    hipStream_t s = ctx.stream;
    // test hooks of this request, cleared however the request ends
    struct HookScope {
        Context &c;
        HookScope(Context &cx, const mbl_problem &q) : c(cx) {
            c.hooks = q.flags & (MBL_HOOK_IR_STALL32 | MBL_HOOK_IR_STALL64 | MBL_HOOK_NO_CONV);
            c.budget.armed = q.fail_alloc_bytes;
            c.budget.since_armed = 0;
        }
        ~HookScope() { c.hooks = 0; c.budget.armed = 0; c.budget.since_armed = 0; }
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
    double hnorm = std::max(std::fabs(emin), std::fabs(emax));
    if (hnorm == 0.0) hnorm = 1.0;
    ctx.hnorm_ = hnorm;
    double sigma = std::isfinite(pr.sigma) ? pr.sigma : emin + pr.eps * (emax - emin);
    res.emin = emin; res.emax = emax; res.sigma = sigma; res.hnorm = hnorm;
    res.t_phase[1] = wall_seconds() - t0;

    t0 = wall_seconds();
    ctx.ensure_symbolic(p);
    res.t_phase[2] = wall_seconds() - t0;

    // The LU is taken at sigma_f = sigma -+ delta: a shift that coincides with an
    // eigenvalue (eps = 0 or 1 puts sigma on E_min / E_max) would make H - sigma
    // singular.  delta is far below the level spacing; a few extra pairs are
    // converged around sigma_f and the nev nearest sigma are selected, with a
    // check that the window provably contains them.
    t0 = wall_seconds();
    const double delta = 1e-6 * hnorm;
    const bool upper = std::isfinite(pr.sigma) ? true : (pr.eps >= 0.5);
    const double sigma_f = sigma + (upper ? delta : -delta);
    double anorm = hnorm + std::fabs(sigma_f);
    SolveStats st;
    int prec = pr.prec;
    ctx.factor(p, prec, sigma_f, anorm, st);
    res.t_phase[3] = wall_seconds() - t0;

    // block Krylov-Schur on (H - sigma_f)^-1
    t0 = wall_seconds();
    int nev = pr.nev;
    int nw = (int)std::min<int64_t>(n, nev + 2 + nev / 16);
    int b = pr.block > 0 ? std::min(pr.block, 16) : default_block((int64_t)n);
    int nkeep = round_up(nw + std::max(8, nw / 2), b);
    int ncv = pr.ncv > 0 ? round_up(pr.ncv, b) : round_up(std::max(2 * nw + 2 * b, nkeep + 3 * b), b);
    if (ncv + b > n) {               // small sector: a full-space basis, vector at a time
        b = 1;
        ncv = (int)n;
        nkeep = std::min<int>(nkeep, (int)n);
    }
    nkeep = std::max(nkeep, nw);
    int max_restarts = pr.max_restarts > 0 ? pr.max_restarts : 300;
    ctx.d_psi.ensure(sizeof(double) * n * nw, &ctx.budget);
    bool fell_back = false;
    auto op = [&](const double *X, double *Y, int nb) {
        try {
            ctx.shift_solve(p, prec, nb, X, Y, st);
            if (prec == MBL_FP32_IR64 && st.gmres_inner > 8) {
                // the FP32 factor needs many GMRES steps per solve here (kappa u_32
                // near one): this result stands, later solves use an FP64 factor
                prec = MBL_FP64;
                fell_back = true;
                SolveStats s2;
                ctx.factor(p, prec, sigma_f, anorm, s2);
            }
        } catch (const Error &e) {
            if (e.code != MBL_ENUMERIC || prec != MBL_FP32_IR64) throw;
            // FP32 refinement did not reach the target: refactor in FP64
            prec = MBL_FP64;
            fell_back = true;
            SolveStats s2;
            ctx.factor(p, prec, sigma_f, anorm, s2);
            ctx.shift_solve(p, prec, nb, X, Y, st);
        }
    };
    const bool never_conv = (ctx.hooks & MBL_HOOK_NO_CONV) != 0;
    auto conv = [&](double th, double rho) {
        return !never_conv && th != 0.0 && rho * anorm <= 0.1 * tol * hnorm * std::fabs(th);
    };
    uint64_t kseed = pr.seed ^ 0xA5A5A5A5A5A5A5A5ULL;
    Context::KSOut ks = ctx.krylov_schur(n, b, ncv, nkeep, nw, Context::Want::LargestAbs, op, conv,
                                         max_restarts, kseed, ctx.d_psi.ptr<double>());
    res.t_phase[4] = wall_seconds() - t0;
    res.t_phase[7] = st.t_solve;
    res.n_restarts = ks.restarts;
    res.n_opapply = ks.napply;
    res.n_passes = (int)(ctx.lu_passes - passes0);
    res.n_pass_rhs = (int)(ctx.lu_pass_rhs - pass_rhs0);
    res.ir_iters_max = st.ir_iters;
    res.n_perturbed = st.n_perturbed;
    res.fallback = fell_back ? 1 : 0;

    // energies (Rayleigh quotients) and FP64 residuals ||H psi - E psi||
    t0 = wall_seconds();
    ctx.d_hpsi.ensure(sizeof(double) * n * nw, &ctx.budget);
    ctx.d_psi2.ensure(sizeof(double) * n * nev, &ctx.budget);
    ctx.d_e.ensure(sizeof(double) * 4 * nw, &ctx.budget);
    int nparts = 64;
    ctx.d_cpart.ensure(sizeof(double) * nparts * nw, &ctx.budget);
    double *psi = ctx.d_psi.ptr<double>(), *hpsi = ctx.d_hpsi.ptr<double>();
    double *de = ctx.d_e.ptr<double>();
    ctx.spmv(p, 0.0, nw, psi, hpsi);
    launch_coldot(n, nw, psi, n, psi, n, de + nw, ctx.d_cpart.ptr<double>(), nparts, s);
    launch_coldot(n, nw, psi, n, hpsi, n, de, ctx.d_cpart.ptr<double>(), nparts, s);
    std::vector<double> E(nw), nrm(nw), rr(nw);
    d2h(E.data(), de, nw, s);
    d2h(nrm.data(), de + nw, nw, s);
    MBL_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < nw; j++) E[j] /= nrm[j];
    h2d(de, E.data(), nw, s);
    launch_sub_scaled_cols(n, nw, de, psi, n, hpsi, n, s);
    launch_coldot(n, nw, hpsi, n, hpsi, n, de + 2 * nw, ctx.d_cpart.ptr<double>(), nparts, s);
    d2h(rr.data(), de + 2 * nw, nw, s);
    MBL_HIP(hipStreamSynchronize(s));
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
    bool window_ok = (nw == n && ks.nconv == nw) ||
                     (rsel + delta <= Rwin * (1.0 + 1e-12) && rsel + delta < unconv);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return E[a] < E[c]; });
    std::vector<double> Es(nev), rs(nev);
    int nconv = 0;
    double maxr = 0.0;
    for (int j = 0; j < nev; j++) {
        Es[j] = E[ord[j]];
        rs[j] = std::sqrt(rr[ord[j]] / nrm[ord[j]]) / hnorm;
        launch_copy(n, psi + (int64_t)ord[j] * n, ctx.d_psi2.ptr<double>() + (int64_t)j * n, s);
        if (rs[j] <= tol) nconv++;
        maxr = std::max(maxr, rs[j]);
    }
    if (!window_ok) nconv = std::min(nconv, nev - 1);
    // the Krylov method stopped at its restart limit: nothing is certified
    // beyond the pairs its own test accepted
    if (ks.nconv < nw) nconv = std::min(nconv, ks.nconv);
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
    res.t_phase[5] = wall_seconds() - t0;
    res.t_phase[6] = wall_seconds() - t_start;
    if (nconv < nev) throw Error(MBL_ENOTCONV, "only " + std::to_string(nconv) + " of " +
                                                   std::to_string(nev) + " pairs reached tol");
}

}  // namespace mbl
