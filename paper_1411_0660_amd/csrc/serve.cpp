// serve.cpp -- request queue: requests are taken in arrival order by a worker
// thread and run through the same path as mbl_solve.
#include "serve.hpp"

#include <algorithm>

namespace mbl {

size_t footprint_bytes(const Plan &p, int prec, int nev, int block) {
    size_t n = (size_t)p.dim;
    size_t es = (prec == MBL_FP32_IR64) ? 4 : 8;
    int b = block > 0 ? block : 8;
    size_t cols = (size_t)std::max(2 * nev + 2 * b, nev + nev / 2 + 3 * b) + 2 * b;
    size_t bytes = 0;
    bytes += es * (size_t)p.arena_elems + 4 * n;           // fronts + pivots
    if (prec == MBL_FP32_IR64) bytes += 0;                  // FP64 fallback is allocated on demand
    bytes += 8 * (size_t)p.vec_elems + 8 * n * 16 * 3;      // solve vectors, x_new, r, d
    bytes += 8 * n * cols * 2 + 8 * n * b;                  // Krylov bases + work block
    bytes += 8 * n * (size_t)nev * 4;                       // Ritz vectors, H psi, sorted copy, blocks
    return bytes;
}

Server::Server(Context *ctx) : ctx_(ctx) { worker_ = std::thread([this] { loop(); }); }

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
}

uint64_t Server::submit(const mbl_problem &prob, mbl_result *res) {
    std::lock_guard<std::mutex> lk(mu_);
    uint64_t t = next_++;
    Req r;
    r.prob = prob;
    r.res = res;
    reqs_[t] = r;
    queue_.push_back(t);
    cv_.notify_one();
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
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return MBL_ENOTFOUND;
    done_cv_.wait(lk, [&] { return reqs_[ticket].done; });
    if (status) *status = reqs_[ticket].status;
    reqs_.erase(ticket);
    return MBL_OK;
}

void Server::loop() {
    for (;;) {
        uint64_t t;
        mbl_problem prob;
        mbl_result *res;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [&] { return stop_ || !queue_.empty(); });
            if (stop_ && queue_.empty()) return;
            t = queue_.front();
            queue_.pop_front();
            prob = reqs_[t].prob;
            res = reqs_[t].res;
        }
        int st = MBL_OK;
        try {
            std::lock_guard<std::recursive_mutex> g(ctx_->mu);
            MBL_HIP(hipSetDevice(ctx_->device));
            solve_problem(*ctx_, prob, *res);
        } catch (const Error &e) {
            set_last_error(e.what());
            st = e.code;
        } catch (const std::exception &e) {
            set_last_error(e.what());
            st = MBL_EDEVICE;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            reqs_[t].status = st;
            reqs_[t].done = true;
        }
        done_cv_.notify_all();
    }
}

}  // namespace mbl
