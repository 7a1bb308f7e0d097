// serve.hpp -- request queue of the C ABI (mbl_submit / mbl_poll / mbl_wait).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "../../include/mbl.h"
#include "solver.hpp"

namespace mbl {

// Predicted device bytes of one request of chain length L (factor fronts,
// solve vectors, Krylov basis, eigenvectors, observables workspace).
size_t footprint_bytes(const Plan &p, int prec, int nev, int block);

class Server {
  public:
    explicit Server(Context *ctx);
    ~Server();
    uint64_t submit(const mbl_problem &prob, mbl_result *res);
    int poll(uint64_t ticket, int *done);
    int wait(uint64_t ticket, int *status);

  private:
    struct Req {
        mbl_problem prob;
        mbl_result *res;
        int status = 1;      // 1 pending, else the mbl status
        bool done = false;
    };
    void loop();
    Context *ctx_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<uint64_t> queue_;
    std::map<uint64_t, Req> reqs_;
    uint64_t next_ = 1;
    bool stop_ = false;
    std::thread worker_;
};

}  // namespace mbl
