// Karras (HPG 2012) node construction: for internal node i of a binary radix
// tree over n sorted, unique keys of W 64-bit words (word W-1 the most
// significant), find its key range and split and return its children (>= 0
// internal node, < 0 leaf ~index).  Shared by the build kernel and its
// host-side test.
#pragma once
#include <stdint.h>

#ifndef RT_HD
#if defined(__HIPCC__)
#define RT_HD __host__ __device__
#else
#define RT_HD
#endif
#endif

namespace rt {

RT_HD inline int lbvh_clz64(uint64_t x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __clzll((long long)x);
#else
    return x ? __builtin_clzll(x) : 64;
#endif
}

// length of the common prefix of keys i and j (-1 outside 0..n-1)
template <int W>
RT_HD inline int lbvh_delta(const uint64_t* k, int64_t n, int64_t i, int64_t j)
{
    if (j < 0 || j >= n) return -1;
    if (W == 1) return lbvh_clz64(k[i] ^ k[j]);
    const uint64_t hi = k[2 * i + 1] ^ k[2 * j + 1];
    return hi ? lbvh_clz64(hi) : 64 + lbvh_clz64(k[2 * i] ^ k[2 * j]);
}

template <int W>
RT_HD inline void lbvh_node(const uint64_t* keys, int64_t n, int64_t i, int32_t* cl, int32_t* cr)
{
    int d = (lbvh_delta<W>(keys, n, i, i + 1) - lbvh_delta<W>(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = lbvh_delta<W>(keys, n, i, i - d);
    int64_t lmax = 2;
    while (lbvh_delta<W>(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (lbvh_delta<W>(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = lbvh_delta<W>(keys, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) >> 1;
        if (lbvh_delta<W>(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t g = i + s * d + (d < 0 ? -1 : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    *cl = (lo == g) ? ~(int32_t)g : (int32_t)g;
    *cr = (hi == g + 1) ? ~(int32_t)(g + 1) : (int32_t)(g + 1);
}

}  // namespace rt
