// Host-side parallel loop of libdgx (mesh set-up and octree tables).
#pragma once

#include <algorithm>
#include <thread>
#include <vector>

namespace dgx {

// Runs fn(begin, end, thread) over [0, n) in contiguous ranges on up to 16
// host threads (one when n is small).
template <typename F>
void host_parallel(int n, F fn) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::min<long>({16L, (long)hw, (long)(n / 512) + 1});
    if (nt <= 1) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        const int b = (int)((long)n * t / nt), e = (int)((long)n * (t + 1) / nt);
        th.emplace_back([=] { fn(b, e, t); });
    }
    for (auto &x : th) x.join();
}

}  // namespace dgx
