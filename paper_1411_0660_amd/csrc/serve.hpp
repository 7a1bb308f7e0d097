// serve.hpp -- continuous batching of solve requests (mbl_submit / mbl_poll /
// mbl_wait): a fixed set of slots, each a solver context with its own HIP
// stream and host thread, so the work of several requests overlaps on the
// device; requests are admitted in arrival order as slots and device memory
// free up, by the predicted footprint of their factor and Krylov storage, and
// queued requests that can share launches are solved as one batch.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mbl.h"
#include "kernels.hpp"
#include "solver.hpp"

namespace mbl {

// Predicted device bytes of one request of chain length L (factor fronts,
// solve vectors, Krylov basis, eigenvectors, observables workspace); an FP32
// request also counts the FP64 factor its refinement may fall back to.
size_t footprint_bytes(const Plan &p, int prec, int nev, int block);

class Server {
  public:
    // `owner` builds the per-L plans that the slots share; `budget` bounds the
    // device bytes the slots hold together (grow-only work buffers included);
    // at most max_batch queued requests that can be batched are solved together.
    Server(Context *owner, int slots, size_t budget, int max_batch);
    void set_max_batch(int m);
    ~Server();
    uint64_t submit(const mbl_problem &prob, mbl_result *res);
    int poll(uint64_t ticket, int *done);
    int wait(uint64_t ticket, int *status);
    void info(mbl_serve_info *out);

  private:
    struct Req {
        mbl_problem prob;
        mbl_result *res = nullptr;
        int status = 1;            // 1 pending, else the mbl status
        bool done = false;
        bool sized = false;
        size_t fp = 0;             // predicted footprint
        int bypassed = 0;          // later requests admitted ahead of this one
        double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
    };
    struct Slot {
        std::unique_ptr<Context> ctx;
        std::thread th;
        std::condition_variable cv;
        bool busy = false;
        std::vector<uint64_t> tickets;   // the request, or the batch, it solves
        size_t held = 0;           // bytes its work buffers may hold (largest admitted)
    };
    void dispatcher();
    void worker(int s);
    int solve_alone(Slot &sl, size_t admitted, const mbl_problem &prob, mbl_result *res,
                    bool &retried);
    bool admit_locked();
    void finish_locked(uint64_t t, int status);

    Context *owner_;
    size_t budget_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<uint64_t> queue_;
    std::map<uint64_t, Req> reqs_;
    std::vector<std::unique_ptr<Slot>> slots_;
    std::thread dispatcher_;
    uint64_t next_ = 1;
    bool stop_ = false;
    int running_ = 0;
    int max_batch_ = MBL_SEG_MAX;
    mbl_serve_info stats_{};
    double t0_ = 0.0;
};

}  // namespace mbl
