// Host-side parallel loop of libdgx (mesh set-up and octree tables).
#pragma once

#include <algorithm>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace dgx {

// Runs fn(begin, end, thread) over [0, n) in contiguous ranges on up to 16
// host threads (one when n is small).  A range whose thread cannot be
// started runs on the calling thread; an exception thrown by fn (a failed
// allocation) is rethrown here once every thread has ended.
template <typename F>
void host_parallel(int n, F fn) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::min<long>({16L, (long)hw, (long)(n / 512) + 1});
    if (nt <= 1) {
        fn(0, n, 0);
        return;
    }
    std::exception_ptr err;
    std::mutex mu;
    auto run = [&](int b, int e, int t) {
        try {
            fn(b, e, t);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            if (!err) err = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const int b = (int)((long)n * t / nt), e = (int)((long)n * (t + 1) / nt);
        bool started = false;
        try {
            th.emplace_back(run, b, e, t);
            started = true;
        } catch (...) {
        }
        if (!started) run(b, e, t);
    }
    for (auto &x : th) x.join();
    if (err) std::rethrow_exception(err);
}

}  // namespace dgx
