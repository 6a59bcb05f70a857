// Host check of the LBVH node construction used by the build kernel:
// for sorted unique keys, every internal node except the root and every leaf
// has exactly one parent, and every node's leaves form a contiguous range.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../../paper_2402_13034_amd/csrc/rt_lbvh_core.hpp"

static int check(std::vector<uint64_t> keys)
{
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    int64_t n = (int64_t)keys.size();
    if (n < 2) return 0;
    std::vector<int32_t> cl(n - 1), cr(n - 1), pin(n - 1, 0), pleaf(n, 0);
    for (int64_t i = 0; i < n - 1; ++i) {
        rt::lbvh_node(keys.data(), n, i, &cl[i], &cr[i]);
        for (int32_t c : {cl[i], cr[i]}) {
            if (c < 0) {
                if (~c >= n) return 1;
                pleaf[~c]++;
            } else {
                if (c >= n - 1 || c == 0) return 2;
                pin[c]++;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i)
        if (pleaf[i] != 1) return 3;
    for (int64_t i = 1; i < n - 1; ++i)
        if (pin[i] != 1) return 4;
    // ranges: leaves under each node contiguous, depth bounded
    std::vector<int64_t> lo(n - 1), hi(n - 1);
    std::vector<int64_t> stack = {0};
    std::vector<int> depth(n - 1, 0);
    int64_t visited_leaves = 0;
    int maxd = 0;
    while (!stack.empty()) {
        int64_t v = stack.back();
        stack.pop_back();
        for (int32_t c : {cl[v], cr[v]}) {
            if (c < 0) {
                visited_leaves++;
                maxd = std::max(maxd, depth[v] + 1);
            } else {
                depth[c] = depth[v] + 1;
                stack.push_back(c);
            }
        }
    }
    if (visited_leaves != n) return 5;
    printf("n=%lld maxdepth=%d\n", (long long)n, maxd);
    return 0;
}

int main()
{
    std::mt19937_64 rng(1234);
    int fails = 0;
    for (int trial = 0; trial < 40; ++trial) {
        int64_t n = 2 + (int64_t)(rng() % (trial < 20 ? 50 : 100000));
        std::vector<uint64_t> keys(n);
        int dup_bits = (int)(rng() % 30);
        for (int64_t i = 0; i < n; ++i) {
            uint64_t m = (rng() & 0x3fffffffull) >> dup_bits << dup_bits;   // many equal Morton codes
            keys[i] = (m << 32) | (uint64_t)i;
        }
        int r = check(keys);
        if (r) {
            printf("FAIL trial %d n=%lld code %d\n", trial, (long long)n, r);
            fails++;
        }
    }
    return fails ? 1 : 0;
}
