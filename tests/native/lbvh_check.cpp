// Host check of the LBVH node construction used by the build kernel:
// for sorted unique keys (one word, or two words as the build uses them:
// triangle index in word 0, Morton code in word 1), every internal node
// except the root and every leaf has exactly one parent, and every node's
// leaves form a contiguous range.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../../paper_2402_13034_amd/csrc/rt_lbvh_core.hpp"

// keys: W words per key; sorted and made unique here (lexicographic from the top word)
template <int W>
static int check(std::vector<uint64_t> flat)
{
    std::vector<std::vector<uint64_t>> rows(flat.size() / W);
    for (size_t i = 0; i < rows.size(); ++i)
        for (int w = W - 1; w >= 0; --w) rows[i].push_back(flat[W * i + w]);   // most significant first
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    std::vector<uint64_t> keys;
    for (auto& r : rows)
        for (int w = W - 1; w >= 0; --w) keys.push_back(r[w]);   // back to word 0 first
    int64_t n = (int64_t)rows.size();
    if (n < 2) return 0;
    std::vector<int32_t> cl(n - 1), cr(n - 1), pin(n - 1, 0), pleaf(n, 0);
    for (int64_t i = 0; i < n - 1; ++i) {
        rt::lbvh_node<W>(keys.data(), n, i, &cl[i], &cr[i]);
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
        std::vector<uint64_t> keys(n), keys2(2 * n);
        int dup_bits = (int)(rng() % 30);
        int dup_bits2 = (int)(rng() % 63);
        for (int64_t i = 0; i < n; ++i) {
            uint64_t m = (rng() & 0x3fffffffull) >> dup_bits << dup_bits;   // many equal Morton codes
            keys[i] = (m << 32) | (uint64_t)i;
            keys2[2 * i] = (uint64_t)i;                                        // index, then a 63-bit code
            keys2[2 * i + 1] = (rng() & 0x7fffffffffffffffull) >> dup_bits2 << dup_bits2;
        }
        int r = check<1>(keys);
        int r2 = check<2>(keys2);
        if (r || r2) {
            printf("FAIL trial %d n=%lld code %d / %d\n", trial, (long long)n, r, r2);
            fails++;
        }
    }
    return fails ? 1 : 0;
}
