// CPU driver of the library's host-side octree code (csrc/host_octree.h) for
// the tests: reads a command and a leaf set on stdin, prints the result.
//
//   adapt  base n, then n lines "L i j k target": one adaptation pass; prints
//          "error <text>" or the new leaves in element order, then their
//          transfer rows (kOctTab ints each)
//   throw  n: a parallel loop over n items whose range with the last item
//          throws; prints "caught" when the exception reaches the caller
#include <cstdio>
#include <iostream>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../paper_2511_17551_amd/csrc/host_octree.h"

int main() {
    std::string cmd;
    std::cin >> cmd;
    if (cmd == "adapt") {
        int base, n;
        std::cin >> base >> n;
        std::vector<dgx::OctLeaf> old(n);
        std::vector<int> target(n);
        for (int e = 0; e < n; ++e) std::cin >> old[e].L >> old[e].i >> old[e].j >> old[e].k >> target[e];
        std::vector<dgx::OctLeaf> out;
        std::vector<int32_t> tab;
        const std::string err = dgx::oct_adapt(base, old, target.data(), out, tab);
        if (!err.empty()) {
            std::printf("error %s\n", err.c_str());
            return 0;
        }
        std::printf("%zu\n", out.size());
        for (size_t e = 0; e < out.size(); ++e) {
            std::printf("%d %d %d %d", out[e].L, out[e].i, out[e].j, out[e].k);
            for (int q = 0; q < dgx::kOctTab; ++q) std::printf(" %d", tab[e * dgx::kOctTab + q]);
            std::printf("\n");
        }
        return 0;
    }
    if (cmd == "throw") {
        int n;
        std::cin >> n;
        std::vector<int> hit(n, 0);
        try {
            dgx::host_parallel(n, [&](int b, int e, int) {
                for (int i = b; i < e; ++i) hit[i] = 1;
                if (e == n) throw std::runtime_error("planted");
            });
        } catch (const std::runtime_error &) {
            int all = 1;
            for (int v : hit) all &= v;
            std::printf("caught %d\n", all);
            return 0;
        }
        std::printf("not caught\n");
        return 0;
    }
    return 1;
}
