// serve.cpp -- continuous batching of solve requests.
//
// Requests wait in arrival order.  A dispatcher thread sizes each one (the
// per-L plan and symbolic analysis are built once, by the owning context, and
// shared read-only by the slots) and admits it to an idle slot when the bytes
// all slots may hold -- their grow-only work buffers, counted at the largest
// footprint each slot has run -- plus its own footprint fit the budget.  A
// request that does not fit lets later ones pass, at most 2 x slots times, and
// idle slots give back their buffers when that makes it fit.  Each slot solves
// on its own stream in its own thread, so requests overlap on the device; the
// arithmetic of a request does not depend on the slot or on what else runs, so
// its result is the same alone and in the mix.  Queued requests that can share
// launches (one chain length and the same solver settings) are admitted
// together, up to the batch limit, and solved as one batch (solve_batch), each
// with its lone arithmetic.
#include "serve.hpp"

#include <algorithm>

namespace mbl {

size_t footprint_bytes(const Plan &p, int prec, int nev, int block) {
    size_t n = (size_t)p.dim;
    int b = block > 0 ? std::min(block, 16) : default_block((int64_t)n);
    int nw = (int)std::min<size_t>(n, (size_t)nev + 2 + nev / 16);
    size_t cols = (size_t)std::max(2 * nw + 2 * b, nw + std::max(8, nw / 2) + 3 * b) + 2 * b;
    cols = std::min(cols, n + 16);
    size_t bytes = 0;
    const size_t panel_inv = 8 * (size_t)FNB * FNB * std::max<size_t>(1, p.h_fd.size());
    bytes += 8 * (size_t)p.arena_elems + 12 * n + panel_inv;     // FP64 fronts, pivots, row maps
    if (prec == MBL_FP32_IR64) bytes += 4 * (size_t)p.arena_elems + 12 * n + panel_inv;  // FP32
    bytes += 8 * (size_t)p.vec_elems * 2 + 8 * n * 16 * 6; // solve vectors, x_new, r, d, staging
    bytes += 8 * (size_t)p.part_elems;                      // L21 / U12 partial products
    bytes += 8 * n * cols * 2 + 8 * n * 16;                 // Krylov bases + work block
    if (prec == MBL_FP32_IR64) bytes += 8 * n * 16 * 62;    // GMRES bases (30 + 31 blocks)
    bytes += 8 * n * (size_t)(nw + 8) * 4;                  // Ritz vectors, H psi, copies
    // observables: the scattered magnetization blocks and the Golub-Kahan
    // bases of every returned vector (at most 2 dim per vector), block map,
    // per-vector reduction partials
    bytes += 8 * n * (size_t)nev * 3 + 4 * n + 8 * (size_t)nev * (64 * 9 + 64);
    // projected-matrix buffers: staging, Jacobi matrix and vectors, and the
    // partial sums of the tall-skinny products (at most 512 row ranges)
    const size_t c = cols + 16;
    bytes += 8 * (2 * c * c) + 8 * (2 * c * c + c + 1) + 8 * 512 * c * 16;
    bytes += 8 * (2 * c * c + 2 * c * 16) + 4 * 2 * c;     // device staging of the expansions
    bytes += (size_t)1 << 20;                               // small per-request buffers
    return bytes;
}

Server::Server(Context *owner, int slots, size_t budget, int max_batch)
    : owner_(owner), budget_(budget) {
    set_max_batch(max_batch);
    t0_ = wall_seconds();
    stats_.slots = slots;
    stats_.budget_bytes = budget;
    for (int i = 0; i < slots; i++) {
        std::unique_ptr<Slot> sl(new Slot);
        sl->ctx.reset(new Context(*owner, budget));
        slots_.push_back(std::move(sl));
    }
    for (int i = 0; i < slots; i++) slots_[i]->th = std::thread([this, i] { worker(i); });
    dispatcher_ = std::thread([this] { dispatcher(); });
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    for (auto &sl : slots_) sl->cv.notify_all();
    if (dispatcher_.joinable()) dispatcher_.join();
    for (auto &sl : slots_)
        if (sl->th.joinable()) sl->th.join();
    std::lock_guard<std::mutex> lk(mu_);
    for (uint64_t t : queue_) finish_locked(t, MBL_EBUSY);   // never started
    queue_.clear();
}

void Server::set_max_batch(int m) {
    std::lock_guard<std::mutex> lk(mu_);
    max_batch_ = std::max(1, std::min(m, MBL_SEG_MAX));
}

uint64_t Server::submit(const mbl_problem &prob, mbl_result *res) {
    std::lock_guard<std::mutex> lk(mu_);
    uint64_t t = next_++;
    Req &r = reqs_[t];
    r.prob = prob;
    r.res = res;
    r.t_submit = wall_seconds() - t0_;
    queue_.push_back(t);
    stats_.submitted++;
    cv_.notify_all();
    return t;
}

int Server::poll(uint64_t ticket, int *done) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return MBL_ENOTFOUND;
    *done = it->second.done ? 1 : 0;
    return MBL_OK;
}

int Server::wait(uint64_t ticket, int *status) {
    std::unique_lock<std::mutex> lk(mu_);
    if (reqs_.find(ticket) == reqs_.end()) return MBL_ENOTFOUND;
    done_cv_.wait(lk, [&] { return reqs_[ticket].done; });
    if (status) *status = reqs_[ticket].status;
    reqs_.erase(ticket);
    return MBL_OK;
}

void Server::info(mbl_serve_info *out) {
    std::lock_guard<std::mutex> lk(mu_);
    *out = stats_;
    out->running = running_;
    out->queued = (int64_t)queue_.size();
    size_t held = 0;
    for (auto &sl : slots_) held += sl->held;
    out->held_bytes = held;
}

void Server::finish_locked(uint64_t t, int status) {
    Req &r = reqs_[t];
    r.status = status;
    r.done = true;
    r.t_done = wall_seconds() - t0_;
    if (r.res) {
        r.res->t_submit = r.t_submit;
        r.res->t_start = r.t_start;
        r.res->t_done = r.t_done;
    }
    stats_.completed++;
    done_cv_.notify_all();
}

bool Server::admit_locked() {
    bool any = false;
    const int nslots = (int)slots_.size();
    std::vector<uint64_t> skipped;
    // the idle slot a request of `need` bytes fits in with the least growth
    auto find_slot = [&](size_t need) {
        size_t total = 0;
        for (auto &sl : slots_) total += sl->held;
        int best = -1;
        size_t best_growth = 0;
        for (int s = 0; s < nslots; s++) {
            Slot &sl = *slots_[s];
            if (sl.busy) continue;
            size_t grown = std::max(sl.held, need);
            if (total - sl.held + grown > budget_) continue;
            size_t growth = grown - sl.held;
            if (best < 0 || growth < best_growth) { best = s; best_growth = growth; }
        }
        return best;
    };
    auto idle = [&] {
        for (auto &sl : slots_)
            if (!sl->busy) return true;
        return false;
    };
    for (auto it = queue_.begin(); it != queue_.end();) {
        // nothing can be admitted while every slot is busy (the queue may be
        // long: do not walk it then)
        if (!idle()) break;
        uint64_t t = *it;
        Req &r = reqs_[t];
        if (!r.sized) break;                      // arrival order: size first
        if (r.fp > budget_) {                     // can never fit
            it = queue_.erase(it);
            finish_locked(t, MBL_ENOMEM);
            continue;
        }
        // queued requests that can share this one's launches, in arrival order
        std::vector<uint64_t> batch{t};
        if (max_batch_ > 1) {
            int looked = 0;                       // companions come from the next 256 requests
            for (auto jt = std::next(it);
                 jt != queue_.end() && (int)batch.size() < max_batch_ && looked < 256; ++jt, ++looked) {
                Req &u = reqs_[*jt];
                if (!u.sized) break;
                mbl_problem pair[2] = {r.prob, u.prob};
                if (batchable(pair, 2)) batch.push_back(*jt);
            }
        }
        // the largest part of the batch that fits an idle slot (each problem
        // of a batch holds what it would alone)
        size_t count = batch.size();
        int best = find_slot(count * r.fp);
        while (best < 0 && count > 1) {
            count /= 2;
            best = find_slot(count * r.fp);
        }
        if (best < 0) {
            count = 1;
            size_t busy_held = 0, total = 0;
            for (auto &sl : slots_) {
                total += sl->held;
                if (sl->busy) busy_held += sl->held;
            }
            if (busy_held + r.fp <= budget_) {
                // idle slots give their buffers back until the request fits
                for (int s = 0; s < nslots && best < 0; s++) {
                    Slot &sl = *slots_[s];
                    if (sl.busy || sl.held == 0) continue;
                    {
                        std::lock_guard<std::recursive_mutex> g(sl.ctx->mu);
                        sl.ctx->trim();
                    }
                    total -= sl.held;
                    sl.held = 0;
                    stats_.trims++;
                    if (total + r.fp <= budget_) best = s;
                }
            }
        }
        if (best < 0) {
            skipped.push_back(t);
            if (r.bypassed >= 2 * nslots) break;  // stop letting later requests pass
            ++it;
            continue;
        }
        batch.resize(count);
        Slot &sl = *slots_[best];
        sl.held = std::max(sl.held, count * r.fp);
        sl.busy = true;
        sl.tickets = batch;
        const double now = wall_seconds() - t0_;
        for (uint64_t u : batch) reqs_[u].t_start = now;
        running_ += (int)count;
        stats_.admitted += (int64_t)count;
        if (count > 1) {
            stats_.batches++;
            stats_.batched += (int64_t)count;
        }
        stats_.max_running = std::max<int64_t>(stats_.max_running, running_);
        for (uint64_t u : skipped) {
            reqs_[u].bypassed++;
            stats_.bypasses++;
        }
        // the batch leaves the queue (its companions all queued after the head);
        // the scan goes on from the head's place
        const auto pos = it - queue_.begin();
        queue_.erase(std::remove_if(queue_.begin() + pos, queue_.end(),
                                    [&](uint64_t u) {
                                        return std::find(batch.begin(), batch.end(), u) !=
                                               batch.end();
                                    }),
                     queue_.end());
        it = queue_.begin() + pos;
        sl.cv.notify_one();
        any = true;
    }
    return any;
}

void Server::dispatcher() {
    (void)hipSetDevice(owner_->device);
    std::unique_lock<std::mutex> lk(mu_);
    while (!stop_) {
        // size the first request that has no footprint yet (plans are built
        // by the owning context, outside the queue lock)
        uint64_t t = 0;
        for (uint64_t u : queue_)
            if (!reqs_[u].sized) { t = u; break; }
        if (t) {
            mbl_problem prob = reqs_[t].prob;
            lk.unlock();
            int code = MBL_OK;
            size_t fp = 0;
            try {
                MBL_REQUIRE(prob.L >= 2 && prob.L <= MBL_L_MAX, MBL_EINVAL,
                            "L must satisfy 2 <= L <= 22");
                std::lock_guard<std::recursive_mutex> g(owner_->mu);
                Plan &p = owner_->plan(prob.L);
                owner_->ensure_symbolic(p);
                fp = footprint_bytes(p, prob.prec, prob.nev > 0 ? prob.nev : 1, prob.block);
            } catch (const Error &e) {
                code = e.code;
            } catch (const std::exception &) {
                code = MBL_EDEVICE;
            }
            lk.lock();
            if (code != MBL_OK) {
                queue_.erase(std::find(queue_.begin(), queue_.end(), t));
                finish_locked(t, code);
            } else {
                reqs_[t].fp = fp;
                reqs_[t].sized = true;
            }
            admit_locked();
            continue;
        }
        if (!admit_locked()) cv_.wait(lk);
    }
}

// One request on a slot, capped at the bytes the slot was admitted with.
int Server::solve_alone(Slot &sl, size_t admitted, const mbl_problem &prob, mbl_result *res,
                        bool &retried) {
    int st = MBL_OK;
    for (int attempt = 0; attempt < 2; attempt++) {
        st = MBL_OK;
        try {
            std::lock_guard<std::recursive_mutex> g(sl.ctx->mu);
            // the slot may hold no more device memory than it was admitted with
            sl.ctx->budget.limit = admitted;
            solve_problem(*sl.ctx, prob, *res);
        } catch (const Error &e) {
            st = e.code;
        } catch (const std::bad_alloc &) {
            st = MBL_ENOMEM;
        } catch (const std::exception &) {
            st = MBL_EDEVICE;
        }
        // buffers kept from earlier, differently sized requests can push a
        // slot past its admission: it gives them back and runs once more
        if (st != MBL_ENOMEM || attempt > 0) break;
        std::lock_guard<std::recursive_mutex> g(sl.ctx->mu);
        if (sl.ctx->budget.used == 0) break;
        sl.ctx->trim();
        retried = true;
    }
    return st;
}

void Server::worker(int s) {
    (void)hipSetDevice(owner_->device);
    Slot &sl = *slots_[s];
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        sl.cv.wait(lk, [&] { return stop_ || sl.busy; });
        if (!sl.busy) return;                     // stopping, nothing assigned
        const std::vector<uint64_t> tickets = sl.tickets;
        const int count = (int)tickets.size();
        std::vector<mbl_problem> probs(count);
        std::vector<mbl_result *> outs(count);
        for (int q = 0; q < count; q++) {
            probs[q] = reqs_[tickets[q]].prob;
            outs[q] = reqs_[tickets[q]].res;
        }
        const size_t admitted = sl.held;
        lk.unlock();
        std::vector<int> st(count, MBL_OK);
        bool retried = false, done = false;
        if (count > 1) {
            // one batch: its plan is built by the owning context, then every
            // problem is solved with its lone arithmetic in shared launches
            std::vector<mbl_result> res(count);
            for (int q = 0; q < count; q++) res[q] = *outs[q];
            try {
                {
                    std::lock_guard<std::recursive_mutex> g(owner_->mu);
                    owner_->batch_plan(probs[0].L, count);
                }
                std::lock_guard<std::recursive_mutex> g(sl.ctx->mu);
                sl.ctx->budget.limit = admitted;
                done = solve_batch(*sl.ctx, count, probs.data(), res.data(), st.data());
            } catch (const std::exception &) {
                done = false;
            }
            if (done)
                for (int q = 0; q < count; q++) *outs[q] = res[q];
        }
        if (!done)
            for (int q = 0; q < count; q++) st[q] = solve_alone(sl, admitted, probs[q], outs[q], retried);
        lk.lock();
        if (retried) stats_.retries++;
        stats_.max_slot_peak = std::max<size_t>(stats_.max_slot_peak, sl.ctx->budget.peak);
        sl.busy = false;
        running_ -= count;
        for (int q = 0; q < count; q++) finish_locked(tickets[q], st[q]);
        cv_.notify_all();
    }
}

}  // namespace mbl
