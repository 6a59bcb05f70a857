// Tracing: discovery rays, candidate surface sequences, image-method paths,
// visibility legs, the per-element RIS expansion and the field.
//
// Stages (all on one stream; sizes are read back where buffers depend on them):
//  1. discovery  spherical-Fibonacci rays from the Tx (full sphere) and from
//                the RIS centre u (half-space in front of the RIS); closest
//                hit + specular bounce up to K times (stand-in for the
//                analytic first stage of the hybrid tracer, Section II).
//  2. dedupe     every prefix of every hit list, mapped to surfaces, packed
//                21 bits per surface into a key of one 64-bit word (orders
//                up to 3) or two (orders 4 and 5: surfaces 0-2 in word 0,
//                3-4 in word 1); hash set, then sort (+ unique for two words).
//  3. images     per candidate: images of the source in the surfaces' planes.
//  4. paths      per (receiver, candidate): image-method back-trace, surface
//                containment and side tests (FP64); the valid cells are
//                appended per wave and sorted into (receiver, candidate) order.
//  5. legs       each record's legs tested for occlusion (second stage of the
//                hybrid tracer; relaunch of Section IV-A).
//  6. field      Tx -> Rx: eq. (3) in the form of eq. (8) per path, summed per
//                receiver in record order (deterministic).
//  7. RIS        per (receiver, element): the direct element path and every
//                sequence valid from u re-run through the image method from
//                the element (Section II-B), legs re-checked, field of
//                eqs. (4)-(8) without Gamma summed into H[r, m].
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <utility>
#include <vector>

#include "rt_host.hpp"

namespace rt {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ void wave_count_add(unsigned long long* ctr, unsigned v)
{
    // one atomic per wave
    unsigned long long s = v;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(ctr, s);
}

// Block-staged append: a block gathers its values in LDS (LDS atomics) and
// reserves room for all of them with one global atomic; values past `cap`
// are dropped while the counter keeps counting (the host checks it).  The
// order of the appended values is not fixed: callers sort them.
template <int NMAX>
struct BlockAppend {
    uint64_t* vals;   // LDS, NMAX entries
    int* n;           // LDS counter
    unsigned long long* base;   // LDS
    __device__ void init()
    {
        if (threadIdx.x == 0) *n = 0;
        __syncthreads();
    }
    __device__ void push(uint64_t v)
    {
        int slot = atomicAdd(n, 1);
        if (slot < NMAX) vals[slot] = v;
    }
    // every thread of the block must call flush
    __device__ void flush(uint64_t* out, int64_t cap, unsigned long long* counter)
    {
        __syncthreads();
        const int cnt = *n < NMAX ? *n : NMAX;
        if (threadIdx.x == 0) *base = cnt > 0 ? atomicAdd(counter, (unsigned long long)cnt) : 0ull;
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            const unsigned long long idx = *base + (unsigned long long)t;
            if (idx < (unsigned long long)cap) out[idx] = vals[t];
        }
    }
};

// --------------------------------------------------------------------------
// 1. discovery
// --------------------------------------------------------------------------
__device__ __forceinline__ void fib_dir(int64_t i, int64_t n, double* out)
{
    const double g = (sqrt(5.0) - 1.0) / 2.0;
    double z = 1.0 - (double)(2 * i + 1) / (double)n;
    double x = (double)i * g;
    double ph = 6.283185307179586 * (x - floor(x));
    double r = sqrt(1.0 - z * z);
    out[0] = r * cos(ph);
    out[1] = r * sin(ph);
    out[2] = z;
}

constexpr int DISC_B = 128;


// Launch order of the discovery rows.  Consecutive Fibonacci rows form a
// thin band of directions (z falls linearly with the row); within a chunk of
// RT_FIB_CHUNK rows a wave should trace neighbouring azimuths.  The azimuth
// of row i0 + j is 2 pi frac(frac(i0 g) + frac(j g)), so the azimuth order of
// a chunk is one fixed order of j (by frac(j g)), rotated by an offset that
// depends on the chunk: position j of chunk c launches row
// c RT_FIB_CHUNK + perm[(off[c] + j) mod RT_FIB_CHUNK].  The tables are built
// once per context on the host; they only order the work (any order gives
// the same results).
#define RT_FIB_CHUNK 8192
#define RT_FIB_MAX_CHUNKS (((int64_t)1 << 31) / RT_FIB_CHUNK)

static void fib_tables(Ctx& c, const int32_t** perm, const int32_t** off)
{
    std::lock_guard<std::mutex> lk(c.fib_mu);
    if (!c.fib_perm) {
        const double g = (std::sqrt(5.0) - 1.0) / 2.0;
        std::vector<std::pair<double, int32_t>> fr(RT_FIB_CHUNK);
        for (int j = 0; j < RT_FIB_CHUNK; ++j) {
            const double x = (double)j * g;
            fr[j] = {x - std::floor(x), j};
        }
        std::sort(fr.begin(), fr.end());
        std::vector<int32_t> pm(RT_FIB_CHUNK), of((size_t)RT_FIB_MAX_CHUNKS);
        std::vector<double> fv(RT_FIB_CHUNK);
        for (int k = 0; k < RT_FIB_CHUNK; ++k) {
            pm[k] = fr[k].second;
            fv[k] = fr[k].first;
        }
        for (int64_t ch = 0; ch < RT_FIB_MAX_CHUNKS; ++ch) {
            const double x = (double)(ch * RT_FIB_CHUNK) * g;
            const double f0 = x - std::floor(x);
            of[(size_t)ch] = (int32_t)(std::lower_bound(fv.begin(), fv.end(), 1.0 - f0) - fv.begin()) % RT_FIB_CHUNK;
        }
        int32_t *dp = nullptr, *dofs = nullptr;
        HIP_CHECK(hipMalloc(&dp, sizeof(int32_t) * RT_FIB_CHUNK));
        HIP_CHECK(hipMalloc(&dofs, sizeof(int32_t) * (size_t)RT_FIB_MAX_CHUNKS));
        HIP_CHECK(hipMemcpy(dp, pm.data(), sizeof(int32_t) * RT_FIB_CHUNK, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(dofs, of.data(), sizeof(int32_t) * (size_t)RT_FIB_MAX_CHUNKS, hipMemcpyHostToDevice));
        c.fib_perm = dp;
        c.fib_off = dofs;
    }
    *perm = c.fib_perm;
    *off = c.fib_off;
}

// Rows not launched keep -1 hit lists.
__global__ void k_fill_neg(int32_t* p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = -1;
}

// De-duplication of prefix keys in an open-addressing hash set (keys != 0,
// capacity a power of two, linear probing; a probe run longer than max_probe
// raises the overflow flag, and the caller repeats with a larger set).  A slot is read before the
// compare-and-swap, so the many repeats of a key cost no atomics.
// mix64 is the 64-bit finalizer (fmix64) of Austin Appleby's public-domain
// MurmurHash3, constants as published.
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ void hash_insert(unsigned long long* table, uint64_t mask, uint64_t max_probe,
                                            uint64_t key, int* overflow)
{
    uint64_t h = mix64(key) & mask;
    for (uint64_t probe = 0; probe <= max_probe; ++probe) {
        // a plain read may be stale only as 0 (a slot changes once, 0 -> key); the CAS decides then
        unsigned long long cur = table[h];
        if (cur == key) return;
        if (cur == 0ull) {
            unsigned long long prev = atomicCAS(&table[h], 0ull, (unsigned long long)key);
            if (prev == 0ull || prev == key) return;
        }
        h = (h + 1) & mask;
    }
    atomicOr(overflow, 1);
}

// Two-word keys (orders 4 and 5): a slot is two words, word 0 (never 0 for a
// key: it holds the first surface) claimed by compare-and-swap, then word 1
// published with bit 63 set (0 = not yet written).  A lane that finds word 0
// equal to its key's but word 1 not (yet) equal probes on and may insert the
// key a second time; the sort that follows removes such duplicates, so a key
// is never lost and never kept twice.
#define RT_W1_SET (1ull << 63)
__device__ __forceinline__ void hash_insert2(unsigned long long* table, uint64_t mask, uint64_t max_probe,
                                             uint64_t k0, uint64_t k1, int* overflow)
{
    const unsigned long long w1 = (unsigned long long)(k1 | RT_W1_SET);
    uint64_t h = mix64(k0 ^ mix64(k1)) & mask;
    for (uint64_t probe = 0; probe <= max_probe; ++probe) {
        unsigned long long cur = table[2 * h];
        if (cur == 0ull) {
            const unsigned long long prev = atomicCAS(&table[2 * h], 0ull, (unsigned long long)k0);
            if (prev == 0ull) {
                atomicExch(&table[2 * h + 1], w1);
                return;
            }
            cur = prev;
        }
        if (cur == k0 && table[2 * h + 1] == w1) return;
        h = (h + 1) & mask;
    }
    atomicOr(overflow, 1);
}

// Discovery over the direction-sorted ray list; every prefix of every hit
// list (as surface ids) goes into the hash set.  Neighbouring lanes trace
// neighbouring directions, so a lane skips a key equal to its left
// neighbour's (one of them inserts it).  KM: the largest order of the
// instance (K <= KM); keys of orders above 3 have two words.
// CNT: the counting build: each lane walks the binary tree on its own (the
// method's per-ray LBVH walk, same hits) and the node visits, triangle tests
// and segments are added to work[0..2].
template <bool BRUTE, int STK, int KM, bool CNT>
__global__ __launch_bounds__(DISC_B) void k_discover(SceneView s, double sx, double sy, double sz,
                                                     const int32_t* perm, const int32_t* off, int64_t rows,
                                                     int hemi, double hx, double hy, double hz, int K,
                                                     int32_t* hits, unsigned long long* segs,
                                                     unsigned long long* table, uint64_t mask, uint64_t max_probe,
                                                     int* overflow, unsigned long long* work)
{
    constexpr int W = KM > RT_KM_SMALL ? 2 : 1;
    // per-lane stacks for the brute-force build and the counting build, one stack per wave for the wave walk
    __shared__ int stack[BRUTE ? 1 : (CNT ? STK * DISC_B : RT_STACK4 * (DISC_B / 64))];
    WorkCount wc;
    int64_t t = (int64_t)blockIdx.x * DISC_B + threadIdx.x;
    unsigned nseg = 0;
    uint64_t keys[KM], keys1[KM];   // key of each prefix: word 0, word 1
#pragma unroll
    for (int q = 0; q < KM; ++q) keys[q] = keys1[q] = 0ull;
    const int64_t ch = t / RT_FIB_CHUNK;
    const int64_t i = ch * RT_FIB_CHUNK + perm[(off[ch] + (int)(t % RT_FIB_CHUNK)) % RT_FIB_CHUNK];
    // the bounce loop runs for the whole wave; a lane drops out when its ray escapes
    double d64[3] = {0.0, 0.0, 1.0};
    bool alive = i < rows;
    if (alive) {
        fib_dir(i, rows, d64);
        alive = hemi ? (d64[0] * hx + d64[1] * hy + d64[2] * hz) > 0.0 : true;
    }
    const bool alive0 = alive;   // launched row (its hit list is written)
    float ox = (float)sx, oy = (float)sy, oz = (float)sz;
    float dx = (float)d64[0], dy = (float)d64[1], dz = (float)d64[2];
    int skip = -1;
    uint64_t acc = 0, acc1 = 0;
    int hid[KM];   // hit ids, stored after the walk (no store between the walk's loads)
#pragma unroll
    for (int q = 0; q < KM; ++q) hid[q] = -1;
    int* wst = stack + (BRUTE ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * RT_STACK4);
    for (int b = 0; b < K; ++b) {
        if (__ballot(alive) == 0ull) break;
        float tt;
        int id;
        if (alive) ++nseg;
        int slot;
        if (BRUTE)
            slot = alive ? closest_hit<true>(s, ox, oy, oz, dx, dy, dz, (float)RT_EPS, skip, nullptr, 0, tt, id) : -1;
        else if (CNT)
            slot = alive ? closest_hit<false, true>(s, ox, oy, oz, dx, dy, dz, (float)RT_EPS, skip,
                                                    stack + threadIdx.x, DISC_B, tt, id, &wc)
                         : -1;
        else
            slot = closest_hit_wave4(s, alive, ox, oy, oz, dx, dy, dz, (float)RT_EPS, skip, wst, tt, id);
        alive = alive && slot >= 0;
        if (alive) {
            const uint64_t field = (uint64_t)(__float_as_int(s.tri4[3 * slot + 1].w) + 1);
            if (W == 1 || b < 3)
                acc |= field << (RT_KEY_BITS * b);
            else
                acc1 |= field << (RT_KEY_BITS * (b - 3));
            // constant indices only, so the ids and keys stay in registers
#pragma unroll
            for (int q = 0; q < KM; ++q) {
                hid[q] = b == q ? id : hid[q];
                keys[q] = b == q ? acc : keys[q];
                if (W == 2) keys1[q] = b == q ? acc1 : keys1[q];
            }
            float px = ox + tt * dx, py = oy + tt * dy, pz = oz + tt * dz;
            reflect32(s.tri4[3 * slot + 1], s.tri4[3 * slot + 2], dx, dy, dz);
            ox = px;
            oy = py;
            oz = pz;
            skip = id;
        }
    }
    if (hits && alive0)
#pragma unroll
        for (int b = 0; b < KM; ++b)
            if (b < K) hits[i * K + b] = hid[b];
#pragma unroll
    for (int b = 0; b < KM; ++b) {
        const uint64_t left = __shfl_up(keys[b], 1, 64);
        const uint64_t left1 = W == 2 ? __shfl_up(keys1[b], 1, 64) : 0ull;
        const bool first = (threadIdx.x & 63) == 0 || left != keys[b] || (W == 2 && left1 != keys1[b]);
        if (b < K && keys[b] != 0ull && first) {
            if (W == 1)
                hash_insert(table, mask, max_probe, keys[b], overflow);
            else
                hash_insert2(table, mask, max_probe, keys[b], keys1[b], overflow);
        }
    }
    wave_count_add(segs, nseg);
    if (CNT) {
        wave_count_add(work + 0, wc.nodes);
        wave_count_add(work + 1, wc.tris);
        wave_count_add(work + 2, nseg);
    }
}

// --------------------------------------------------------------------------
// 2. candidate keys: surface ids + 1, 21 bits per bounce; 0 = none
// --------------------------------------------------------------------------
// every sequence of <= K surfaces without immediate repeat, as keys of W
// words (0 for skipped)
template <int W>
__global__ void k_exhaustive_keys(int64_t n_surf, int K, int64_t total, uint64_t* keys)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    // idx enumerates order k = 1..K blocks of n_surf^k entries
    int64_t base = 0, cnt = n_surf;
    int k = 1;
    while (k <= K && idx >= base + cnt) {
        base += cnt;
        cnt *= n_surf;
        ++k;
    }
    int64_t r = idx - base;
    uint64_t key = 0, key1 = 0;
    int prev = -1;
    bool ok = true;
    for (int j = 0; j < k; ++j) {
        int sidx = (int)(r % n_surf);
        r /= n_surf;
        if (sidx == prev) ok = false;
        prev = sidx;
        if (j < 3)
            key |= (uint64_t)(sidx + 1) << (RT_KEY_BITS * j);
        else
            key1 |= (uint64_t)(sidx + 1) << (RT_KEY_BITS * (j - 3));
    }
    keys[W * idx] = ok ? key : 0ull;
    if (W == 2) keys[W * idx + 1] = ok ? key1 : 0ull;
}

// surface id (or -1) of position j of a key of W words
template <int W>
__device__ __forceinline__ int key_surface(const uint64_t* key, int j)
{
    const uint64_t w = (W == 2 && j >= 3) ? key[1] : key[0];
    const int sh = RT_KEY_BITS * (j >= 3 ? j - 3 : j);
    const uint64_t v = (w >> sh) & ((1ull << RT_KEY_BITS) - 1);
    return v ? (int)v - 1 : -1;
}

// --------------------------------------------------------------------------
// 3. candidates: decode keys, images of the source
// --------------------------------------------------------------------------
// per candidate: order, KM surface ids (-1 padded), KM images (3 doubles each)
template <int KM>
__global__ void k_cand_prep(const uint64_t* keys, int64_t n, SceneView s, double sx, double sy, double sz,
                            int32_t* ck, int32_t* cseq, double* cimg)
{
    constexpr int W = KM > RT_KM_SMALL ? 2 : 1;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint64_t* key = keys + W * c;
    int k = 0;
    int seq[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        seq[j] = key_surface<W>(key, j);
        if (seq[j] >= 0 && k == j) k = j + 1;
    }
    ck[c] = k;
    double I[3] = {sx, sy, sz};
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        cseq[KM * c + j] = seq[j];
        if (j < k) {
            double o[3];
            mirror(s.s_plane + 4 * seq[j], I, o);
            I[0] = o[0];
            I[1] = o[1];
            I[2] = o[2];
        }
        cimg[3 * KM * c + 3 * j + 0] = I[0];
        cimg[3 * KM * c + 3 * j + 1] = I[1];
        cimg[3 * KM * c + 3 * j + 2] = I[2];
    }
}

// --------------------------------------------------------------------------
// 4. path geometry per (rx, candidate); valid cells compacted per wave
// --------------------------------------------------------------------------
struct CandView {
    const int32_t* k;
    const int32_t* seq;
    const double* img;
    int64_t n;
};

template <int KM>
__device__ __forceinline__ bool geo_path(const SceneView& s, const CandView& cv, int64_t c, const double* S,
                                         const double* X, double (*P)[3], int* tri, int& k)
{
    k = cv.k[c];
    int seq[KM];
    double I[KM + 1][3];
    I[0][0] = S[0];
    I[0][1] = S[1];
    I[0][2] = S[2];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        seq[j] = cv.seq[KM * c + j];
        for (int q = 0; q < 3; ++q) I[j + 1][q] = cv.img[3 * KM * c + 3 * j + q];
    }
    return image_backtrace<KM>(s, seq, k, I, X, P, tri);
}



// occupied slots of the hash set, appended per wave (order is fixed by the sort that follows)
constexpr int TC_B = 256, TC_PT = 8;
// The occupied slots appended to out[1..] (out[0] = 0: the order-0 key).
__global__ __launch_bounds__(TC_B) void k_table_compact(const unsigned long long* table, int64_t cap, uint64_t* out,
                                                        int64_t out_cap, unsigned long long* counter)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0ull;
    out += 1;
    __shared__ uint64_t vals[TC_B * TC_PT];
    __shared__ int n;
    __shared__ unsigned long long base;
    BlockAppend<TC_B * TC_PT> app{vals, &n, &base};
    app.init();
    unsigned long long v[TC_PT];   // all loads in flight before the first append
    for (int j = 0; j < TC_PT; ++j) {
        const int64_t i = ((int64_t)blockIdx.x * TC_PT + j) * TC_B + threadIdx.x;
        v[j] = i < cap ? table[i] : 0ull;
    }
    for (int j = 0; j < TC_PT; ++j)
        if (v[j] != 0ull) app.push((uint64_t)v[j]);
    app.flush(out, out_cap, counter);
}

// The same for two-word slots (word 1 loses its written bit): the block
// gathers slot indices, then copies both words.
__global__ __launch_bounds__(TC_B) void k_table_compact2(const unsigned long long* table, int64_t cap, uint64_t* out,
                                                         int64_t out_cap, unsigned long long* counter)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[0] = 0ull;
        out[1] = 0ull;
    }
    out += 2;
    __shared__ uint64_t idx[TC_B * TC_PT];
    __shared__ int n;
    __shared__ unsigned long long base;
    if (threadIdx.x == 0) n = 0;
    __syncthreads();
    for (int j = 0; j < TC_PT; ++j) {
        const int64_t i = ((int64_t)blockIdx.x * TC_PT + j) * TC_B + threadIdx.x;
        if (i < cap && table[2 * i] != 0ull) idx[atomicAdd(&n, 1)] = (uint64_t)i;
    }
    __syncthreads();
    const int cnt = n;
    if (threadIdx.x == 0) base = cnt > 0 ? atomicAdd(counter, (unsigned long long)cnt) : 0ull;
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += TC_B) {
        const unsigned long long o = base + (unsigned long long)t;
        if (o < (unsigned long long)out_cap) {
            const uint64_t i = idx[t];
            out[2 * o] = table[2 * i];
            out[2 * o + 1] = table[2 * i + 1] & ~RT_W1_SET;
        }
    }
}

// Sort keys of the receivers: the 42-bit Morton code of the position (14 bits
// per axis over the scene's box, clamped to it) above the 22-bit index.  A
// scene without triangles has no box (null): every code is 0.
constexpr int RX_IDX_BITS = 22;
__global__ void k_rx_keys(const double* rx, int64_t R, const float* box, uint64_t* keys)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    uint64_t code = 0;
    for (int k = 0; k < 3 && box; ++k) {
        const float lo = box[k], ext = box[3 + k] - box[k];
        float u = ext > 0.0f ? ((float)rx[3 * r + k] - lo) / ext : 0.5f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const unsigned q = (unsigned)fminf(u * 16384.0f, 16383.0f);
        for (int b = 0; b < 14; ++b) code |= (uint64_t)((q >> b) & 1u) << (3 * b + 2 - k);
    }
    keys[r] = code << RX_IDX_BITS | (uint64_t)r;
}

// One wave takes GEO_CPW candidates for 64 receivers, so the candidate's
// surfaces, planes and triangles are wave-uniform (scalar loads, no divergence
// in the loops over a surface's triangles).  The receivers of a wave are 64
// consecutive ones of `order` (the receivers sorted by Morton code of their
// positions): neighbours, so that a candidate tends to fail for all lanes of a
// wave at the same bounce.  A block covers 32 candidates = one 32-bit word of
// the receiver's row of the validity mask (mask[r * n_words + w], bit b =
// candidate 32 w + b).
// grid: x = word (group of 32 candidates), y = block of 64 slots of `order`
constexpr int GEO_B = 256, GEO_CPW = 8;
template <int KM>
__global__ __launch_bounds__(GEO_B) void k_geo_mask(SceneView s, CandView cv, double sx, double sy, double sz,
                                                    const double* rx, const uint64_t* order, int64_t R,
                                                    int64_t n_words, uint32_t* mask)
{
    static_assert(GEO_B / 64 * GEO_CPW == 32, "one mask word per block");
    __shared__ uint32_t part[GEO_B / 64][64];
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.y * 64 + lane;
    const int64_t r = slot < R ? (int64_t)(order[slot] & ((1ull << RX_IDX_BITS) - 1ull)) : R;
    uint32_t bits = 0;
    if (r < R) {
        const double S[3] = {sx, sy, sz};
        const double X[3] = {rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]};
        const int64_t c0 = (int64_t)blockIdx.x * 32 + wib * GEO_CPW;
        for (int j = 0; j < GEO_CPW; ++j) {
            const int64_t c = c0 + j;
            if (c >= cv.n) break;
            double P[KM][3];
            int tri[KM];
            int k;
            if (geo_path<KM>(s, cv, c, S, X, P, tri, k)) bits |= 1u << j;
        }
    }
    part[wib][lane] = bits << (GEO_CPW * wib);
    __syncthreads();
    if (wib == 0 && r < R)
        mask[r * n_words + blockIdx.x] = part[0][lane] | part[1][lane] | part[2][lane] | part[3][lane];
}

// valid cells per receiver (one wave per receiver; entry R is 0)
__global__ void k_cell_count(const uint32_t* mask, int64_t R, int64_t n_words, int64_t* cnt)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r > R) return;
    int64_t n = 0;
    if (r < R)
        for (int64_t w = lane; w < n_words; w += 64) n += __popc(mask[r * n_words + w]);
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if (lane == 0) cnt[r] = n;
}

// cells r * n_cand + c of the set bits, in (receiver, candidate) order, from
// the receivers' exclusive offsets (one wave per receiver)
__global__ void k_cell_emit(const uint32_t* mask, int64_t R, int64_t n_words, int64_t n_cand, const int64_t* rstart,
                            uint64_t* cells)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= R) return;
    int64_t base = rstart[r];
    for (int64_t w0 = 0; w0 < n_words; w0 += 64) {
        const int64_t w = w0 + lane;
        uint32_t m = w < n_words ? mask[r * n_words + w] : 0u;
        const int cnt = __popc(m);
        int incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        int64_t pos = base + (incl - cnt);
        while (m) {
            const int b = __ffs((int)m) - 1;
            m &= m - 1u;
            cells[pos++] = (uint64_t)(r * n_cand + w * 32 + b);
        }
        base += __shfl(incl, 63, 64);
    }
}

// --------------------------------------------------------------------------
// 5/6. legs and field of each geometric path, in (receiver, candidate) order
// --------------------------------------------------------------------------
constexpr int LEG_B = 128;

template <int KM>
struct PathRec {
    int32_t rx, cand, k;
    int32_t tri[KM];
};

// Path points by value, constant indices only: V[0] = S, V[j] = P[j - 1] for
// j <= k, X from k + 1 on (so leg j runs from V[j] to V[j + 1]).
template <int KM>
__device__ __forceinline__ void path_points(const double* S, const double (*P)[3], const double* X, int k,
                                            double (*V)[3])
{
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        V[0][q] = S[q];
#pragma unroll
        for (int j = 1; j <= KM; ++j) V[j][q] = k >= j ? P[j - 1][q] : X[q];
        V[KM + 1][q] = X[q];
    }
}

// the point before X on the path (S for a direct path), by value
template <int KM>
__device__ __forceinline__ void last_point(const double* S, const double (*P)[3], int k, double* L)
{
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double v = S[q];
#pragma unroll
        for (int j = 1; j <= KM; ++j) v = k == j ? P[j - 1][q] : v;
        L[q] = v;
    }
}

__device__ __forceinline__ double seg_len(const double* a, const double* b)
{
    double w0 = b[0] - a[0], w1 = b[1] - a[1], w2 = b[2] - a[2];
    return sqrt(w0 * w0 + w1 * w1 + w2 * w2);
}

template <bool BRUTE, bool FIELD, int STK, int KM>
__global__ __launch_bounds__(LEG_B) void k_paths(SceneView s, CandView cv, TraceConst tc, double sx, double sy,
                                                 double sz, const double* rx, const uint64_t* cells, int64_t n,
                                                 uint8_t* valid, float2* amp, double* len, PathRec<KM>* recs,
                                                 unsigned long long* segs)
{
    __shared__ int stack[STK * LEG_B];
    int64_t i = (int64_t)blockIdx.x * LEG_B + threadIdx.x;
    unsigned nseg = 0;
    if (i < n) {
        const uint64_t cell = cells[i];
        const int64_t r = (int64_t)(cell / (uint64_t)cv.n), c = (int64_t)(cell - (uint64_t)r * cv.n);
        double S[3] = {sx, sy, sz};
        double X[3] = {rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]};
        double P[KM][3];
        int tri[KM];
#pragma unroll
        for (int j = 0; j < KM; ++j) tri[j] = -1;
        int k;
        bool ok = geo_path<KM>(s, cv, c, S, X, P, tri, k);
        float Ft = 1.0f, Fr = 1.0f;
        double V[KM + 2][3];
        path_points<KM>(S, P, X, k, V);
        if (FIELD && ok) {
            double v1[3], vl[3], L[3];
            last_point<KM>(S, P, k, L);
            for (int q = 0; q < 3; ++q) {
                v1[q] = V[1][q] - S[q];
                vl[q] = L[q] - X[q];
            }
            const bool on_t = pattern_gate_amp(tc.txa.pattern, tc.txa.param, v1, tc.txa.axis, tc.txa.axis_norm, Ft);
            const bool on_r = pattern_gate_amp(tc.rxa.pattern, tc.rxa.param, vl, tc.rxa.axis, tc.rxa.axis_norm, Fr);
            ok = on_t && on_r;
        }
        int sq[KM];
#pragma unroll
        for (int j = 0; j < KM; ++j) sq[j] = cv.seq[KM * c + j];
#pragma unroll
        for (int j = 0; j <= KM; ++j) {
            if (j > k || !ok) break;
            // leg j runs from V[j] to V[j + 1] (V[j + 1] = X when j = k)
            const int sa = j == 0 ? -1 : sq[j > 0 ? j - 1 : 0];
            const int sb = j == k ? -1 : sq[j < KM ? j : 0];
            ++nseg;
            if (leg_blocked<BRUTE>(s, V[j], V[j + 1], sa, sb, stack + threadIdx.x, LEG_B)) ok = false;
        }
        valid[i] = ok ? 1 : 0;
        PathRec<KM> pr;
        pr.rx = (int32_t)r;
        pr.cand = (int32_t)c;
        pr.k = k;
#pragma unroll
        for (int j = 0; j < KM; ++j) pr.tri[j] = j < k ? tri[j] : -1;
        recs[i] = pr;
        if (FIELD) {
            double D = 0.0, Lj[KM + 1];
#pragma unroll
            for (int j = 0; j <= KM; ++j) {
                Lj[j] = 0.0;
                if (j <= k) {
                    Lj[j] = seg_len(V[j], V[j + 1]);
                    D += Lj[j];
                }
            }
            float2 a = make_float2(0.0f, 0.0f);
            if (ok) {
                float ar = 1.0f, ai = 0.0f;
#pragma unroll
                for (int j = 0; j < KM; ++j) {
                    if (j >= k) break;
                    float2 Rc;
                    if (tc.fresnel) {
                        const double d[3] = {V[j + 1][0] - V[j][0], V[j + 1][1] - V[j][1], V[j + 1][2] - V[j][2]};
                        Rc = fresnel_coef(s, tri[j], d, Lj[j], tc.fresnel, tc.sig_scale);
                    } else {
                        Rc = s.refl[tri[j]];
                    }
                    float nr = ar * Rc.x - ai * Rc.y;
                    float ni = ar * Rc.y + ai * Rc.x;
                    ar = nr;
                    ai = ni;
                }
                float mag = sqrtf((float)tc.two_eta0_pt_gt) * Ft * sqrtf((float)tc.rxa.gain) * Fr *
                            (tc.lam_4pi * __builtin_amdgcn_rcpf((float)D));
                float cs, sn;
                phase_cs(D, tc.inv_lambda, cs, sn);
                a = make_float2(mag * (ar * cs - ai * sn), mag * (ar * sn + ai * cs));
            }
            amp[i] = a;
            len[i] = D;
        }
    }
    wave_count_add(segs, nseg);
}

// E_env[r] = sum of emitted paths of receiver r (FP64): one wave per
// receiver, lane l sums records l, l + 64, ... of its range, then a fixed
// butterfly over the lanes (the same order on every run).
constexpr int ENV_B = 256;
__global__ __launch_bounds__(ENV_B) void k_env_reduce(const int64_t* rstart, int64_t R, const uint8_t* valid,
                                                      const float2* amp, float2* E)
{
    const int64_t r = (int64_t)blockIdx.x * (ENV_B / 64) + (threadIdx.x >> 6);
    if (r >= R) return;   // whole waves leave together
    const int lane = threadIdx.x & 63;
    double er = 0.0, ei = 0.0;
    const int64_t j1 = rstart[r + 1];
    for (int64_t j = rstart[r] + lane; j < j1; j += 64)
        if (valid[j]) {
            const float2 a = amp[j];
            er += (double)a.x;
            ei += (double)a.y;
        }
    for (int o = 32; o > 0; o >>= 1) {
        er += __shfl_xor(er, o, 64);
        ei += __shfl_xor(ei, o, 64);
    }
    if (lane == 0) E[r] = make_float2((float)er, (float)ei);
}

// keep valid records: env path records for read-back
template <int KM>
__global__ void k_env_compact(const PathRec<KM>* recs, CandView cv, const uint8_t* valid, const int64_t* off2,
                              const float2* amp, const double* len, int64_t n, EnvRec* out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !valid[i]) return;
    const PathRec<KM>& pr = recs[i];
    EnvRec e;
    e.rx = pr.rx;
    e.order = pr.k;
#pragma unroll
    for (int j = 0; j < RT_MAX_K; ++j) {
        e.seq[j] = -1;
        e.tri[j] = -1;
    }
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        e.seq[j] = cv.seq[KM * pr.cand + j];
        e.tri[j] = pr.tri[j];
    }
    e.length = len[i];
    e.amp[0] = amp[i].x;
    e.amp[1] = amp[i].y;
    out[off2[i]] = e;
}

// valid centre sequences of order >= 1
template <int KM>
__global__ void k_u_flags(const PathRec<KM>* recs, const uint8_t* valid, int64_t n, uint8_t* f2)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    f2[i] = (valid[i] && recs[i].k >= 1) ? 1 : 0;
}

// Rows of useq_stride(KM) = 2 KM + 2 ints: rx, surfaces s_0..s_{KM-1},
// triangles t_0..t_{KM-1} reached from the centre, 0.
constexpr int useq_stride(int KM) { return 2 * KM + 2; }

template <int KM>
__global__ void k_u_compact(const PathRec<KM>* recs, CandView cv, const uint8_t* f2, const int64_t* off2, int64_t n,
                            int32_t* useq)
{
    constexpr int US = useq_stride(KM);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !f2[i]) return;
    int64_t o = off2[i];
    useq[US * o + 0] = recs[i].rx;
    for (int j = 0; j < KM; ++j) {
        useq[US * o + 1 + j] = cv.seq[KM * recs[i].cand + j];
        useq[US * o + 1 + KM + j] = recs[i].tri[j];
    }
    useq[US * o + US - 1] = 0;
}

__global__ void k_uptr_dev(const int64_t* rstart, int64_t n_rec, const int64_t* off2, const int64_t* total2,
                           int64_t R, int64_t* uptr)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > R) return;
    int64_t a = rstart[r];
    uptr[r] = (r < R && a < n_rec) ? off2[a] : *total2;
}

// Launch order of the per-element kernel, heaviest receiver first (the
// longest waves start first and short ones fill the tail): key = inverted
// cost (slots weighted by legs, 20 bits) above the receiver index.
template <int KM>
__global__ void k_ris_order(const int64_t* uptr, const int32_t* useq, int64_t R, uint64_t* keys)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    int64_t cost = 1;   // the direct slot: one leg
    for (int64_t u = uptr[r]; u < uptr[r + 1]; ++u) {
        const int32_t* row = useq + useq_stride(KM) * u;
        cost += 2;   // k + 1 legs, k >= 1
        for (int j = 1; j < KM; ++j) cost += row[1 + j] >= 0;
    }
    const uint64_t c = (uint64_t)(cost < 0xFFFFF ? cost : 0xFFFFF);
    keys[r] = ((0xFFFFFull - c) << 32) | (uint64_t)r;
}

// --------------------------------------------------------------------------
// 7. RIS
// --------------------------------------------------------------------------
// Field reaching element m (eqs. (4)-(6) without Gamma_m and F_out):
// T = sum over incoming paths p of A_t(v1_p) sqrt(G F_in(p) d_y d_z / 4pi)
// prod(R_p) e^{-jk d_p} / d_p; the direct leg, plus the reflections Tx ->
// surfaces -> m when they are modelled.
struct TxmRec {
    float2 T;
    int ok;        // some incoming path emitted (clear legs, F_t, F_in > 0)
    int pad;
};

template <bool BRUTE, int STK>
__global__ __launch_bounds__(64) void k_txm(SceneView s, TraceConst tc, RisView rv, TxmRec* out,
                                            unsigned long long* segs)
{
    __shared__ int stack[STK * 64];
    int m = blockIdx.x * 64 + threadIdx.x;
    unsigned nseg = 0;
    if (m < rv.M) {
        const double* e = rv.elem + 3 * m;
        double vt[3] = {e[0] - tc.tx[0], e[1] - tc.tx[1], e[2] - tc.tx[2]};
        double back[3] = {-vt[0], -vt[1], -vt[2]};
        double dt = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
        const double ct = cos_between(vt, tc.txa.axis, tc.txa.axis_norm);
        const double ci = cos_between(back, rv.normal, rv.normal_norm);
        const float Ft = pattern_amp(tc.txa.pattern, tc.txa.param, ct);   // sqrt(F_t)
        const float Fin = pattern_amp(1, rv.q, ci);                        // sqrt(F_in)
        bool ok = pattern_on(tc.txa.pattern, ct) && pattern_on(1, ci);
        if (ok) {
            ++nseg;
            ok = !leg_blocked<BRUTE>(s, tc.tx, e, -1, -1, stack + threadIdx.x, 64);
        }
        TxmRec r;
        r.ok = ok ? 1 : 0;
        r.pad = 0;
        r.T = make_float2(0.0f, 0.0f);
        if (ok) {
            const float fac = (float)(sqrt(tc.two_eta0_pt_gt) * (double)Ft *
                                      sqrt(rv.gain * rv.dy * rv.dz / (4.0 * 3.141592653589793)) * (double)Fin / dt);
            float cs, sn;
            phase_cs(dt, tc.inv_lambda, cs, sn);
            r.T = make_float2(fac * cs, fac * sn);
        }
        out[m] = r;
    }
    wave_count_add(segs, nseg);
}

// Incoming reflections (Section II-B, supporting reflections): the image
// method from the Tx to the RIS, restricted like the out side to the
// sequences valid from the Tx to the RIS centre u.
// 1) per Tx candidate of order >= 1: valid and unblocked from the Tx to u?
template <bool BRUTE, int STK, int KM>
__global__ __launch_bounds__(LEG_B) void k_in_centre(SceneView s, CandView cv, double sx, double sy, double sz,
                                                     double ux, double uy, double uz, uint8_t* ok_out,
                                                     unsigned long long* segs)
{
    __shared__ int stack[STK * LEG_B];
    const int64_t c = (int64_t)blockIdx.x * LEG_B + threadIdx.x;
    unsigned nseg = 0;
    if (c < cv.n) {
        const double S[3] = {sx, sy, sz};
        const double X[3] = {ux, uy, uz};
        double P[KM][3];
        int tri[KM];
        int k = 0;
        bool ok = cv.k[c] >= 1 && geo_path<KM>(s, cv, c, S, X, P, tri, k);
        double V[KM + 2][3];
        path_points<KM>(S, P, X, k, V);
        int sq[KM];
#pragma unroll
        for (int j = 0; j < KM; ++j) sq[j] = cv.seq[KM * c + j];
#pragma unroll
        for (int j = 0; j <= KM; ++j) {
            if (j > k || !ok) break;
            const int sa = j == 0 ? -1 : sq[j > 0 ? j - 1 : 0];
            const int sb = j == k ? -1 : sq[j < KM ? j : 0];
            ++nseg;
            if (leg_blocked<BRUTE>(s, V[j], V[j + 1], sa, sb, stack + threadIdx.x, LEG_B)) ok = false;
        }
        ok_out[c] = ok ? 1 : 0;
    }
    wave_count_add(segs, nseg);
}

__global__ void k_in_list(const uint8_t* ok, const int64_t* off, int64_t n, int32_t* list)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n && ok[c]) list[off[c]] = (int32_t)c;
}

// 2) per (sequence j of the list, element m): the path Tx -> seq -> m, its legs
// and its contribution to T_m (zero if not emitted); *n_in = list length
template <bool BRUTE, int STK, int KM>
__global__ __launch_bounds__(LEG_B) void k_in_elem(SceneView s, CandView cv, TraceConst tc, RisView rv,
                                                   const int32_t* list, const int64_t* n_in, float2* contrib,
                                                   uint8_t* emitted_out, unsigned long long* segs,
                                                   unsigned long long* n_paths)
{
    __shared__ int stack[STK * LEG_B];
    const int64_t i = (int64_t)blockIdx.x * LEG_B + threadIdx.x;
    const int64_t M = rv.M;
    const int64_t nl = *n_in;
    unsigned nseg = 0, emitted = 0;
    if (i < nl * M) {
        const int64_t j = i / M, m = i - j * M;
        const int64_t c = list[j];
        const double S[3] = {tc.tx[0], tc.tx[1], tc.tx[2]};
        const double X[3] = {rv.elem[3 * m], rv.elem[3 * m + 1], rv.elem[3 * m + 2]};
        double P[KM][3];
        int tri[KM];
        int k = 0;
        bool ok = geo_path<KM>(s, cv, c, S, X, P, tri, k);
        double V[KM + 2][3];
        path_points<KM>(S, P, X, k, V);
        float Ft = 0.0f, Fin = 0.0f;
        if (ok) {
            double v1[3], back[3], L[3];
            last_point<KM>(S, P, k, L);
            for (int q = 0; q < 3; ++q) {
                v1[q] = V[1][q] - S[q];
                back[q] = L[q] - X[q];
            }
            const double ct = cos_between(v1, tc.txa.axis, tc.txa.axis_norm);
            const double ci = cos_between(back, rv.normal, rv.normal_norm);
            Ft = pattern_amp(tc.txa.pattern, tc.txa.param, ct);
            Fin = pattern_amp(1, rv.q, ci);
            ok = pattern_on(tc.txa.pattern, ct) && pattern_on(1, ci);
        }
        int sq[KM];
#pragma unroll
        for (int q = 0; q < KM; ++q) sq[q] = cv.seq[KM * c + q];
#pragma unroll
        for (int q = 0; q <= KM; ++q) {
            if (q > k || !ok) break;
            const int sa = q == 0 ? -1 : sq[q > 0 ? q - 1 : 0];
            const int sb = q == k ? -1 : sq[q < KM ? q : 0];
            ++nseg;
            if (leg_blocked<BRUTE>(s, V[q], V[q + 1], sa, sb, stack + threadIdx.x, LEG_B)) ok = false;
        }
        float2 a = make_float2(0.0f, 0.0f);
        if (ok) {
            double D = 0.0, Lq[KM + 1];
#pragma unroll
            for (int q = 0; q <= KM; ++q) {
                Lq[q] = 0.0;
                if (q <= k) {
                    Lq[q] = seg_len(V[q], V[q + 1]);
                    D += Lq[q];
                }
            }
            float ar = 1.0f, ai = 0.0f;
#pragma unroll
            for (int q = 0; q < KM; ++q) {
                if (q >= k) break;
                float2 Rc;
                if (tc.fresnel) {
                    const double d[3] = {V[q + 1][0] - V[q][0], V[q + 1][1] - V[q][1], V[q + 1][2] - V[q][2]};
                    Rc = fresnel_coef(s, tri[q], d, Lq[q], tc.fresnel, tc.sig_scale);
                } else {
                    Rc = s.refl[tri[q]];
                }
                const float nr = ar * Rc.x - ai * Rc.y;
                const float ni = ar * Rc.y + ai * Rc.x;
                ar = nr;
                ai = ni;
            }
            const float mag = (float)(sqrt(tc.two_eta0_pt_gt) * (double)Ft *
                                      sqrt(rv.gain * rv.dy * rv.dz / (4.0 * 3.141592653589793)) * (double)Fin / D);
            float cs, sn;
            phase_cs(D, tc.inv_lambda, cs, sn);
            a = make_float2(mag * (ar * cs - ai * sn), mag * (ar * sn + ai * cs));
            emitted = 1;
        }
        contrib[i] = a;
        emitted_out[i] = (uint8_t)emitted;
    }
    wave_count_add(segs, nseg);
    wave_count_add(n_paths, emitted);
}

// 3) per element: T_m += the contributions of the list in list order (FP64)
__global__ void k_in_sum(const float2* contrib, const uint8_t* emitted, const int64_t* n_in, int64_t M,
                         TxmRec* txm)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int64_t nl = *n_in;
    TxmRec r = txm[m];
    double tr = r.T.x, ti = r.T.y;
    bool lit = r.ok != 0;
    for (int64_t j = 0; j < nl; ++j) {
        const float2 a = contrib[j * M + m];
        if (emitted[j * M + m]) lit = true;
        tr += (double)a.x;
        ti += (double)a.y;
    }
    r.T = make_float2((float)tr, (float)ti);
    r.ok = lit ? 1 : 0;
    txm[m] = r;
}

constexpr int RIS_B = 128;

// Back-trace like image_backtrace, but each reflection first tries the
// triangle the RIS-centre path used (hint); a point on a surface lies in
// exactly one of its triangles, so the result is the same as a full search.
template <bool CNT, int KM>
__device__ inline bool image_backtrace_hint(const SceneView& s, const int* seq, const int* hint, int k,
                                            const double (*I)[3], const double* X, double (*P)[3], int* tri,
                                            WorkCount* wc)
{
#pragma clang fp contract(off)
    double Q[3] = {X[0], X[1], X[2]};
#pragma unroll
    for (int i = KM; i >= 1; --i) {
        if (i > k) continue;
        const double* pl = s.s_plane + 4 * seq[i - 1];
        double w0 = Q[0] - I[i][0], w1 = Q[1] - I[i][1], w2 = Q[2] - I[i][2];
        double den = pl[0] * w0 + pl[1] * w1 + pl[2] * w2;
        if (den == 0.0) return false;
        double sp = (pl[3] - (pl[0] * I[i][0] + pl[1] * I[i][1] + pl[2] * I[i][2])) / den;
        if (!(sp > 0.0 && sp < 1.0)) return false;
        double p[3] = {I[i][0] + sp * w0, I[i][1] + sp * w1, I[i][2] + sp * w2};
        int h = hint[i - 1];
        if (CNT && h >= 0) wc->contain++;
        int t = (h >= 0 && contains_proj(s, h, p)) ? h : surface_contains<CNT>(s, seq[i - 1], p, wc);
        if (t < 0) return false;
        tri[i - 1] = t;
        P[i - 1][0] = p[0]; P[i - 1][1] = p[1]; P[i - 1][2] = p[2];
        Q[0] = p[0]; Q[1] = p[1]; Q[2] = p[2];
    }
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        if (i >= k) break;
        const double* pl = s.s_plane + 4 * seq[i];
        double prev[3], next[3];
        for (int q = 0; q < 3; ++q) {
            prev[q] = i == 0 ? I[0][q] : P[i > 0 ? i - 1 : 0][q];
            next[q] = (i == k - 1 || i + 1 >= KM) ? X[q] : P[i + 1 < KM ? i + 1 : 0][q];
        }
        double a = plane_side(pl, prev);
        double b = plane_side(pl, next);
        if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return false;
    }
    return true;
}

// CNT: counting build; work[0..4] += node visits, triangle tests,
// containment tests, (slot, element) pairs, legs.
#ifndef RT_RIS_WAVES_PER_SIMD
#define RT_RIS_WAVES_PER_SIMD 4   // register cap that measured fastest on the lab room
#endif

// FRES: Fresnel coefficients of the materials (tc.fresnel) instead of the fixed ones
template <bool BRUTE, bool KEEP, int STK, bool CNT, bool FRES, int KM>
__global__ __launch_bounds__(RIS_B, RT_RIS_WAVES_PER_SIMD) void k_ris(SceneView s, TraceConst tc, RisView rv, const TxmRec* txm,
                                               const double* rx, int64_t R, const int64_t* uptr,
                                               const int32_t* useq, const uint64_t* order, int n_mchunk, float2* H,
                                               uint8_t* rvalid, float2* camp, double* clen, unsigned long long* segs,
                                               unsigned long long* work, unsigned long long* fallbacks)
{
    // one traversal stack per wave (the 4-wide walk needs RT_STACK4 >= STK entries)
    __shared__ int wstack[RT_STACK4 * (RIS_B / 64)];
    // the rays of a slot's legs wait in LDS while earlier legs are walked (fewer live registers)
    __shared__ float legbuf[RIS_B / 64][KM + 1][7][64];
    // per-wave frontier and candidate lists of the tube walk
    __shared__ int tfront[RIS_B / 64][2 * RT_TUBE_FRONT];
    __shared__ int tcand[RIS_B / 64][RT_TUBE_CAND];
    __shared__ float ttube[RIS_B / 64][8 * (KM + 1)];
    constexpr int US = useq_stride(KM);
    static_assert(RT_STACK4 >= STK, "wave stack");
    WorkCount wc;
    unsigned pairs = 0;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave in block (uniform)
    const int64_t w = (int64_t)blockIdx.x * (RIS_B / 64) + wib;
    const int lane = threadIdx.x & 63;
    int* my_stack = wstack + wib * RT_STACK4;
    unsigned nseg = 0;
    unsigned n_fallback = 0;   // slots whose grouped leg walk fell back (wave-uniform)
    if (w < R * n_mchunk) {
        const int64_t wr = w / n_mchunk;
        const int64_t r = (int64_t)(order[wr] & 0xFFFFFFFFull);
        // the wave's 64 elements are neighbours on the RIS (Morton order of their
        // in-plane coordinates), so the legs of a slot stay in a thin tube
        const int mi = (int)(w - wr * n_mchunk) * 64 + lane;
        const bool active = mi < rv.M;
        const int mm = active ? rv.order[mi] : 0;
        const int m = mm;
        const double* e = rv.elem + 3 * mm;
        const double E[3] = {e[0], e[1], e[2]};
        double dt_keep = 0.0;   // |E - Tx| as the direct leg's length (kept paths only; 0 with the
                                // incoming reflections, whose element field sums several paths)
        if (KEEP && !(tc.flags & 32)) {
#pragma clang fp contract(off)
            const double v0 = E[0] - tc.tx[0], v1 = E[1] - tc.tx[1], v2 = E[2] - tc.tx[2];
            dt_keep = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        }
        const TxmRec t = txm[mm];
        const double X[3] = {rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]};
        const int64_t u0 = uptr[r], u1 = uptr[r + 1];
        const int64_t nsl = 1 + (u1 - u0);
        double acc_r = 0.0, acc_i = 0.0;
#pragma unroll 1
        for (int64_t sl = 0; sl < nsl; ++sl) {
            // the slot's sequence is the same for every lane of the wave
            int seq[KM], hint[KM];
#pragma unroll
            for (int j = 0; j < KM; ++j) seq[j] = hint[j] = -1;
            int k = 0;
            if (sl > 0) {
                const int32_t* row = useq + US * (u0 + sl - 1);
#pragma unroll
                for (int j = 0; j < KM; ++j) {
                    seq[j] = row[1 + j];
                    hint[j] = row[1 + KM + j];
                    if (seq[j] >= 0) k = j + 1;
                }
            }
            bool ok = active && t.ok;
            if (CNT && active) ++pairs;
            // phase 1 (FP64): image method, leg rays, length, amplitude
            float amp_r = 0.0f, amp_i = 0.0f;
            double Dr_keep = 0.0;
            {
                double P[KM][3];
                int tri[KM];
#pragma unroll
                for (int j = 0; j < KM; ++j) tri[j] = -1;
                {
                    double I[KM + 1][3];
                    I[0][0] = E[0];
                    I[0][1] = E[1];
                    I[0][2] = E[2];
#pragma unroll
                    for (int j = 0; j < KM; ++j)
                        if (j < k) mirror(s.s_plane + 4 * seq[j], I[j], I[j + 1]);
                    if (ok) ok = image_backtrace_hint<CNT, KM>(s, seq, hint, k, I, X, P, tri, &wc);
                }
                float Fout = 0.0f, Fr = 0.0f;
                if (ok) {
                    // first and last path points, selected by value (constant indices)
                    double f[3], l[3];
                    last_point<KM>(E, P, k, l);
                    for (int q = 0; q < 3; ++q) f[q] = k ? P[0][q] : X[q];
                    double v1[3] = {f[0] - E[0], f[1] - E[1], f[2] - E[2]};
                    double vl[3] = {l[0] - X[0], l[1] - X[1], l[2] - X[2]};
                    const bool on_o = pattern_gate_amp(1, rv.q, v1, rv.normal, rv.normal_norm, Fout);   // sqrt(F_out)
                    const bool on_r =
                        pattern_gate_amp(tc.rxa.pattern, tc.rxa.param, vl, tc.rxa.axis, tc.rxa.axis_norm, Fr);   // sqrt(F_r)
                    ok = on_o && on_r;
                }
                double Dr = 0.0;
                double Lk[KM + 1];   // leg lengths (the Fresnel angles use them)
#pragma unroll
                for (int j = 0; j <= KM; ++j) {
                    Lk[j] = 0.0;
                    if (j <= k) {
#pragma clang fp contract(off)
                        const double* A = j == 0 ? E : P[j - 1];
                        const double* B = j == k ? X : P[j];
                        double w0 = B[0] - A[0], w1 = B[1] - A[1], w2 = B[2] - A[2];
                        double L = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
                        if (FRES) Lk[j] = L;
                        Dr += L;
                        float* lb = &legbuf[wib][j][0][lane];
                        lb[0 * 64] = (float)A[0];
                        lb[1 * 64] = (float)A[1];
                        lb[2 * 64] = (float)A[2];
                        const double il = 1.0 / L;   // the leg ray's direction as leg_blocked forms it
                        lb[3 * 64] = (float)(w0 * il);
                        lb[4 * 64] = (float)(w1 * il);
                        lb[5 * 64] = (float)(w2 * il);
                        lb[6 * 64] = (float)(L - RT_EPS);
                    }
                }
                if (KEEP) Dr_keep = Dr;
                if (ok) {
                    float ar = 1.0f, ai = 0.0f;
#pragma unroll
                    for (int j = 0; j < KM; ++j) {
                        if (j >= k) break;
                        float2 Rc;
                        if (FRES) {
                            double d[3];
                            for (int q = 0; q < 3; ++q) d[q] = P[j][q] - (j == 0 ? E[q] : P[j > 0 ? j - 1 : 0][q]);
                            Rc = fresnel_coef(s, tri[j], d, Lk[j], tc.fresnel, tc.sig_scale);
                        } else {
                            Rc = s.refl[tri[j]];
                        }
                        float nr = ar * Rc.x - ai * Rc.y;
                        float ni = ar * Rc.y + ai * Rc.x;
                        ar = nr;
                        ai = ni;
                    }
                    const float mag = Fout * sqrtf((float)tc.rxa.gain) * Fr * (tc.lam_4pi * __builtin_amdgcn_rcpf((float)Dr));
                    float cs, sn;
                    phase_cs(Dr, tc.inv_lambda, cs, sn);
                    // incoming field x reflections x out-going phase
                    const float zr = t.T.x * ar - t.T.y * ai, zi = t.T.x * ai + t.T.y * ar;
                    amp_r = mag * (zr * cs - zi * sn);
                    amp_i = mag * (zr * sn + zi * cs);
                }
            }
            // phase 2 (FP32): visibility of every leg, the wave walking the BVH together
            const float tmin = (float)RT_EPS;
            if (BRUTE || CNT) {
#pragma unroll 1
                for (int j = 0; j <= k; ++j) {
                    const int sa = leg_surface_a<KM>(seq, j);
                    const int sb = leg_surface_b<KM>(seq, j, k);
                    const float* lb = &legbuf[wib][j][0][lane];
                    const float ox = lb[0 * 64], oy = lb[1 * 64], oz = lb[2 * 64];
                    const float dx = lb[3 * 64], dy = lb[4 * 64], dz = lb[5 * 64];
                    const float tmax = lb[6 * 64];
                    if (ok) ++nseg;
                    const bool searching = ok && tmax > tmin;
                    bool blocked;
                    if (BRUTE)
                        blocked = searching &&
                                  any_hit<true>(s, ox, oy, oz, dx, dy, dz, tmin, tmax, sa, sb, nullptr, 0);
                    else   // the counting build walks the binary tree: its work is what is counted
                        blocked = any_hit_wave<true>(s, searching, ox, oy, oz, dx, dy, dz, tmin, tmax, sa, sb,
                                                     my_stack, &wc);
                    ok = ok && !blocked;
                }
            } else {
                // every leg at once; legs are counted as the sequential test would (up to the first blocked one)
                const unsigned res = legs_blocked_tube<KM>(s, ok, k, seq, &legbuf[wib][0][0][0], ttube[wib],
                                                       tfront[wib], tcand[wib], my_stack);
                n_fallback += (res & RT_TUBE_FELL_BACK) ? 1u : 0u;   // same on every lane
                const unsigned bl = res & ~RT_TUBE_FELL_BACK;
                if (ok) nseg += bl ? (unsigned)(__ffs((int)bl)) : (unsigned)(k + 1);
                ok = ok && bl == 0u;
            }
            if (ok) {
                acc_r += (double)amp_r;
                acc_i += (double)amp_i;
            }
            if (KEEP && active) {
                const int64_t cell = (u0 + r + sl) * rv.M + m;
                if (rvalid) rvalid[cell] = ok ? 1 : 0;
                if (camp) {   // per-path amplitude and unfolded length (d_t + D_r; D_r alone with the incoming
                              // reflections): impulse response and per-path read-back
                    camp[cell] = ok ? make_float2(amp_r, amp_i) : make_float2(0.0f, 0.0f);
                    clen[cell] = dt_keep + Dr_keep;
                }
            }
        }
        if (active) H[r * rv.M + m] = make_float2((float)acc_r, (float)acc_i);
    }
    if (CNT) {
        wave_count_add(work + 0, wc.nodes);
        wave_count_add(work + 1, wc.tris);
        wave_count_add(work + 2, wc.contain);
        wave_count_add(work + 3, pairs);
        wave_count_add(work + 4, nseg);
    }
    wave_count_add(segs, nseg);
    if (!BRUTE && !CNT) wave_count_add(fallbacks, lane == 0 ? n_fallback : 0u);
}

// --------------------------------------------------------------------------
// host orchestration
// --------------------------------------------------------------------------
#define SEL_BOOL(b, NAME, ...)            \
    if (b) {                              \
        constexpr bool NAME = true;       \
        __VA_ARGS__;                      \
    } else {                              \
        constexpr bool NAME = false;      \
        __VA_ARGS__;                      \
    }
#define SEL_STK(stk, ...)                 \
    if ((stk) == 32) {                    \
        constexpr int STK = 32;           \
        __VA_ARGS__;                      \
    } else {                              \
        constexpr int STK = 64;           \
        __VA_ARGS__;                      \
    }

struct Cands {
    int64_t n = 0;
    Scratch keys, k, seq, img;
    CandView view() const {
        CandView v;
        v.k = k.as<int32_t>();
        v.seq = seq.as<int32_t>();
        v.img = img.as<double>();
        v.n = n;
        return v;
    }
};

static int stack_depth_for(const Scene& s, bool brute) { return (brute || s.max_depth < 31) ? 32 : 64; }

struct PathSet {
    int64_t n = 0;
    Scratch cells, valid, amp, len, recs, rstart;
};

// One source's candidate pipeline, split where the host needs a size.
struct Branch {
    const double* src = nullptr;
    const double* hemi = nullptr;
    int which = 0;
    hipStream_t st = nullptr;
    int64_t* d_cnt = nullptr;
    unsigned long long* d_app = nullptr;
    Scratch keys;
    int64_t nkeys = 0;
    Cands cd;
    PathSet ps;
    // hash set: 0 sized from the last call's count, 1 the standard set,
    // 2 sized for every prefix being distinct (after overflows)
    int table_level = 0;
    Scratch table;            // the hash set of the next phase A (cleared), cap slots
    int64_t cap = 0;
    uint64_t max_probe = 0;
    Scratch mask;             // geometric validity, R rows of n_words 32-bit words
    int64_t n_words = 0;
    unsigned long long* d_work = nullptr;   // counting build: node visits, triangle tests of discovery
    hipEvent_t ev_disc[2] = {nullptr, nullptr};   // around the discovery kernel (stage times only)
};

// RIS description for the kernels
static RisView make_ris_view(const TraceArgs& a)
{
    RisView rv;
    rv.M = (int32_t)a.ris->M;
    rv.pad = 0;
    rv.elem = a.ris->elem.as<double>();
    rv.order = a.ris->order.as<int32_t>();
    for (int q = 0; q < 3; ++q) {
        rv.centre[q] = a.ris->centre[q];
        rv.normal[q] = a.ris->normal[q];
    }
    rv.normal_norm = sqrt(rv.normal[0] * rv.normal[0] + rv.normal[1] * rv.normal[1] + rv.normal[2] * rv.normal[2]);
    rv.dy = a.ris->dy;
    rv.dz = a.ris->dz;
    rv.gain = a.ris->gain > 0 ? a.ris->gain
                              : 4.0 * 3.141592653589793 * a.ris->dy * a.ris->dz / (a.tc.lambda * a.tc.lambda);
    rv.q = a.ris->q;
    return rv;
}

// The field reaching every element (TxmRec per element, in txm): the direct
// leg, and with `incoming` the reflections Tx -> surfaces -> element for the
// Tx candidates valid at the RIS centre.  Launched on stream si (beside the
// path kernels); its scratch lives on si.
template <int KM>
static void ris_incident(Ctx& c, const SceneView& sv, int stk, const TraceArgs& a, bool brute, bool incoming,
                         const Branch& bt, const RisView& rv, unsigned long long* d_ctr, TxmRec* txm, hipStream_t si)
{
    const int64_t M = rv.M;
    unsigned long long* d_legs = d_ctr + 1;
    SEL_BOOL(brute, BR,
             SEL_STK(stk, hipLaunchKernelGGL((k_txm<BR, STK>), dim3(nblk(M, 64)), dim3(64), 0, si, sv, a.tc, rv, txm,
                                             d_legs)));
    HIP_CHECK(hipGetLastError());
    if (!incoming || M == 0 || bt.cd.n == 0) return;
    // sequences valid from the Tx to the RIS centre, then every (sequence, element)
    const int64_t nc = bt.cd.n;
    Scratch in_ok(c, (size_t)nc, si), in_off(c, sizeof(int64_t) * (size_t)nc, si),
        in_list(c, sizeof(int32_t) * (size_t)nc, si);
    int64_t* d_nin = (int64_t*)(d_ctr + 16);
    SEL_BOOL(brute, BR,
             SEL_STK(stk, hipLaunchKernelGGL((k_in_centre<BR, STK, KM>), dim3(nblk(nc, LEG_B)), dim3(LEG_B), 0, si, sv,
                                             bt.cd.view(), a.tc.tx[0], a.tc.tx[1], a.tc.tx[2], rv.centre[0],
                                             rv.centre[1], rv.centre[2], in_ok.as<uint8_t>(), d_legs)));
    HIP_CHECK(hipGetLastError());
    scan_flags(c, in_ok.as<uint8_t>(), in_off.as<int64_t>(), nc, d_nin, si);
    hipLaunchKernelGGL(k_in_list, dim3(nblk(nc, 256)), dim3(256), 0, si, in_ok.as<uint8_t>(), in_off.as<int64_t>(),
                       nc, in_list.as<int32_t>());
    HIP_CHECK(hipGetLastError());
    // launched for every candidate (no size read-back); rows past the list's length exit
    if (nc > ((int64_t)1 << 40) / M) throw inval_error("candidates x elements too large");
    Scratch contrib(c, sizeof(float2) * (size_t)(nc * M), si), emitted(c, (size_t)(nc * M), si);
    SEL_BOOL(brute, BR,
             SEL_STK(stk, hipLaunchKernelGGL((k_in_elem<BR, STK, KM>), dim3(nblk(nc * M, LEG_B)), dim3(LEG_B), 0, si, sv,
                                             bt.cd.view(), a.tc, rv, in_list.as<int32_t>(), d_nin,
                                             contrib.as<float2>(), emitted.as<uint8_t>(), d_legs, d_ctr + 17)));
    HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_in_sum, dim3(nblk(M, 128)), dim3(128), 0, si, contrib.as<float2>(), emitted.as<uint8_t>(),
                       d_nin, M, txm);
    HIP_CHECK(hipGetLastError());
}

// 64-bit words per candidate key: one up to order 3, two for orders 4 and 5
static inline int key_words(int K) { return K > RT_KM_SMALL ? 2 : 1; }
// end of the key bits: 21 per surface, orders above 3 continue in word 1
static inline int key_end_bit(int K) { return K > RT_KM_SMALL ? 64 + RT_KEY_BITS * (K - 3) : RT_KEY_BITS * K; }

// Phase A of the candidates: discovery rays, prefix keys into a hash set,
// occupied slots compacted behind a leading 0 (the empty sequence); the
// count is left in d_app[0] (overflow flag in d_app[1]).  Exhaustive mode:
// every surface sequence, sorted and de-duplicated (count in d_cnt).
// The hash set of a branch's phase A, allocated and cleared on `st`: probe
// runs of at most 256 (an overflow makes the caller repeat with the next
// level): first a set of at least 4x the last call's unique count, then 2^20
// slots, then at least 2 x (keys + 1) slots, at most 2^27, with unbounded
// probing.
static void prepare_table(Ctx& c, const TraceArgs& a, Branch& br, hipStream_t st)
{
    const int64_t rows = br.hemi ? 2 * a.n_rays : a.n_rays;
    const int64_t want = 2 * rows * a.tc.K + 2;
    auto set_size = [want](int64_t limit) {
        int64_t cap = 1024;
        while (cap < want && cap < limit) cap <<= 1;
        return cap;
    };
    int64_t cap = set_size(br.table_level == 2 ? ((int64_t)1 << 27) : ((int64_t)1 << 20));
    if (br.table_level == 0) {
        const int64_t h = c.cand_hint[br.which].load();
        int64_t l = 1024;
        while (h > 0 && l < 4 * h && l < cap) l <<= 1;
        if (h > 0 && l < cap)
            cap = set_size(l);
        else
            br.table_level = 1;   // no smaller set: an overflow goes straight to the last level
    }
    br.cap = cap;
    br.max_probe = br.table_level == 2 ? (uint64_t)(cap - 1) : (uint64_t)255;
    br.table = Scratch(c, sizeof(unsigned long long) * (size_t)key_words(a.tc.K) * (size_t)cap, st);
    HIP_CHECK(hipMemsetAsync(br.table.p, 0, br.table.bytes, st));
}

template <int KM>
static void cand_phase_a(Ctx& c, const SceneView& sv, int stk, const TraceArgs& a, bool brute, bool exhaustive,
                         bool keep_hits, Channel& ch, Branch& br, unsigned long long* d_segs)
{
    const int K = a.tc.K;
    constexpr int W = KM > RT_KM_SMALL ? 2 : 1;
    hipStream_t st = br.st;
    if (exhaustive) {
        int64_t ns = sv.n_surf;
        int64_t total = 0, p = 1;
        for (int k = 1; k <= K; ++k) {
            p *= ns;
            total += p;
            if (total > (int64_t)1 << 26) throw inval_error("exhaustive candidate set too large");
        }
        int64_t nkeys = total + 1;
        Scratch keys(c, sizeof(uint64_t) * W * (size_t)nkeys, st), sorted(c, sizeof(uint64_t) * W * (size_t)nkeys, st);
        HIP_CHECK(hipMemsetAsync(keys.p, 0, keys.bytes, st));
        if (total > 0)
            hipLaunchKernelGGL(k_exhaustive_keys<W>, dim3(nblk(total, 256)), dim3(256), 0, st, ns, K, total,
                               keys.as<uint64_t>());
        HIP_CHECK(hipGetLastError());
        sort_keys(c, keys.as<uint64_t>(), sorted.as<uint64_t>(), nkeys, W, 0, key_end_bit(K), st);
        br.keys = Scratch(c, sizeof(uint64_t) * W * (size_t)nkeys, st);
        unique_keys(c, sorted.as<uint64_t>(), br.keys.as<uint64_t>(), nkeys, W, br.d_cnt, st);
        return;
    }
    const double* src = br.src;
    const double* hemi_n = br.hemi;
    int64_t rows = hemi_n ? 2 * a.n_rays : a.n_rays;
    if (rows > ((int64_t)1 << 31)) throw inval_error("too many discovery rays");
    // hit lists are written only when the caller keeps them
    Scratch hits(c, keep_hits ? sizeof(int32_t) * (size_t)(rows * K) : 0, st);
    if (keep_hits && rows > 0 && K > 0) {
        hipLaunchKernelGGL(k_fill_neg, dim3(nblk(rows * K, 256)), dim3(256), 0, st, hits.as<int32_t>(), rows * K);
        HIP_CHECK(hipGetLastError());
    }
    if (!br.table.p) prepare_table(c, a, br, st);
    Scratch table = std::move(br.table);
    table.st = st;   // released on the branch's stream after its last reader
    const int64_t cap = br.cap;
    const uint64_t max_probe = br.max_probe;
    if (rows > 0 && K > 0 && sv.n_tri > 0) {
        const int32_t *perm, *off;
        fib_tables(c, &perm, &off);
        const int64_t n_launch = (rows + RT_FIB_CHUNK - 1) / RT_FIB_CHUNK * RT_FIB_CHUNK;
        const bool count = (a.tc.flags & 16) != 0 && !brute;
        if (br.ev_disc[0]) HIP_CHECK(hipEventRecord(br.ev_disc[0], st));
        SEL_BOOL(brute, BR, SEL_BOOL(count, CN,
                 SEL_STK(stk, hipLaunchKernelGGL((k_discover<BR, STK, KM, CN>), dim3(nblk(n_launch, DISC_B)),
                                                 dim3(DISC_B), 0, st, sv, src[0], src[1], src[2], perm, off, rows,
                                                 hemi_n ? 1 : 0, hemi_n ? hemi_n[0] : 0.0, hemi_n ? hemi_n[1] : 0.0,
                                                 hemi_n ? hemi_n[2] : 0.0, K, keep_hits ? hits.as<int32_t>() : nullptr,
                                                 d_segs, table.as<unsigned long long>(), (uint64_t)(cap - 1), max_probe,
                                                 (int*)(br.d_app + 1), br.d_work))));
        HIP_CHECK(hipGetLastError());
        if (br.ev_disc[1]) HIP_CHECK(hipEventRecord(br.ev_disc[1], st));
    }
    if (keep_hits) {
        ch.n_hits_rows[br.which] = rows;
        ch.hits[br.which] = std::move(hits);
    }
    br.keys = Scratch(c, sizeof(uint64_t) * W * (size_t)(cap + 1), st);
    if (W == 1)
        hipLaunchKernelGGL(k_table_compact, dim3(nblk(cap, TC_B * TC_PT)), dim3(TC_B), 0, st,
                           table.as<unsigned long long>(), cap, br.keys.as<uint64_t>(), cap, br.d_app);
    else
        hipLaunchKernelGGL(k_table_compact2, dim3(nblk(cap, TC_B * TC_PT)), dim3(TC_B), 0, st,
                           table.as<unsigned long long>(), cap, br.keys.as<uint64_t>(), cap, br.d_app);
    HIP_CHECK(hipGetLastError());
}

// Size read-back after phase A: number of unique candidates (incl. order 0),
// or -1 if the hash set overflowed below the last level.
static int64_t cand_count(Ctx& c, const Branch& br, bool exhaustive)
{
    if (exhaustive) return read_i64(br.d_cnt, br.st);
    int64_t hq[2];
    read_i64s((const int64_t*)br.d_app, hq, 2, br.st);
    if (hq[1] & 1) {
        if (br.table_level < 2) return -1;   // repeat phase A with the next set
        throw inval_error("candidate hash set overflow");
    }
    c.cand_hint[br.which].store(hq[0] + 1);
    return hq[0] + 1;
}

// Phase B: the unique keys in key order (the canonical candidate order).
// Returns their number: n for one-word keys (the hash set holds each once);
// two-word keys may have been inserted twice (see hash_insert2), so they are
// de-duplicated after the sort and counted again (one more size read-back).
static int64_t cand_phase_b(Ctx& c, const TraceArgs& a, bool exhaustive, Branch& br, int64_t n)
{
    if (exhaustive) return n;
    const int W = key_words(a.tc.K);
    Scratch sorted(c, sizeof(uint64_t) * W * (size_t)(n > 0 ? n : 1), br.st);
    sort_keys(c, br.keys.as<uint64_t>(), sorted.as<uint64_t>(), n, W, 0, key_end_bit(a.tc.K), br.st);
    if (W == 1) {
        br.keys = std::move(sorted);
        return n;
    }
    br.keys = Scratch(c, sizeof(uint64_t) * W * (size_t)(n > 0 ? n : 1), br.st);
    unique_keys(c, sorted.as<uint64_t>(), br.keys.as<uint64_t>(), n, W, br.d_cnt, br.st);
    const int64_t nu = read_i64(br.d_cnt, br.st);
    c.cand_hint[br.which].store(nu);
    return nu;
}

// candidate images and the geometric test of every (receiver, candidate) cell
template <int KM>
static void geo_launch(Ctx& c, const SceneView& sv, const TraceArgs& a, Branch& br, int64_t n_cand,
                       const uint64_t* rx_order)
{
    hipStream_t st = br.st;
    Cands& cd = br.cd;
    cd.n = n_cand;
    cd.keys = std::move(br.keys);
    cd.k = Scratch(c, sizeof(int32_t) * (size_t)n_cand, st);
    cd.seq = Scratch(c, sizeof(int32_t) * KM * (size_t)n_cand, st);
    cd.img = Scratch(c, sizeof(double) * 3 * KM * (size_t)n_cand, st);
    hipLaunchKernelGGL(k_cand_prep<KM>, dim3(nblk(n_cand, 128)), dim3(128), 0, st, cd.keys.as<uint64_t>(), n_cand, sv,
                       br.src[0], br.src[1], br.src[2], cd.k.as<int32_t>(), cd.seq.as<int32_t>(),
                       cd.img.as<double>());
    HIP_CHECK(hipGetLastError());
    const int64_t R = a.R;
    if (R > 0 && n_cand > ((int64_t)1 << 40) / R) throw inval_error("receivers x candidates too large for one call");
    if (nblk(R, 64) > 65535 || n_cand > 0x7fffffff) throw inval_error("receiver or candidate count too large");
    const int64_t n_words = (n_cand + 31) / 32;
    br.n_words = n_words;
    br.mask = Scratch(c, sizeof(uint32_t) * (size_t)(R * n_words), st);
    if (R * n_words > 0) {
        hipLaunchKernelGGL(k_geo_mask<KM>, dim3((unsigned)n_words, nblk(R, 64)), dim3(GEO_B), 0, st, sv, cd.view(),
                           br.src[0], br.src[1], br.src[2], a.rx_dev, rx_order, R, n_words,
                           br.mask.as<uint32_t>());
        HIP_CHECK(hipGetLastError());
    }
    // receivers' offsets into the valid cells; entry R = total
    Scratch cnt(c, sizeof(int64_t) * (size_t)(R + 1), st);
    br.ps.rstart = Scratch(c, sizeof(int64_t) * (size_t)(R + 1), st);
    hipLaunchKernelGGL(k_cell_count, dim3(nblk(R + 1, 4)), dim3(256), 0, st, br.mask.as<uint32_t>(), R, n_words,
                       cnt.as<int64_t>());
    HIP_CHECK(hipGetLastError());
    scan_i64(c, cnt.as<int64_t>(), br.ps.rstart.as<int64_t>(), R + 1, st);
}

// the valid cells in (receiver, candidate) order, legs and field of each path
template <int KM>
static void paths_launch(Ctx& c, const SceneView& sv, int stk, const TraceArgs& a, bool brute, bool field,
                         Branch& br, int64_t n, unsigned long long* d_segs)
{
    hipStream_t st = br.st;
    PathSet& ps = br.ps;
    const int64_t R = a.R;
    ps.n = n;
    ps.cells = Scratch(c, sizeof(uint64_t) * (size_t)(n > 0 ? n : 1), st);
    if (n > 0) {
        hipLaunchKernelGGL(k_cell_emit, dim3(nblk(R, 4)), dim3(256), 0, st, br.mask.as<uint32_t>(), R, br.n_words,
                           br.cd.n, ps.rstart.as<int64_t>(), ps.cells.as<uint64_t>());
        HIP_CHECK(hipGetLastError());
    }
    br.mask.release();
    ps.valid = Scratch(c, (size_t)(n > 0 ? n : 1), st);
    ps.recs = Scratch(c, sizeof(PathRec<KM>) * (size_t)(n > 0 ? n : 1), st);
    if (field) {
        ps.amp = Scratch(c, sizeof(float2) * (size_t)(n > 0 ? n : 1), st);
        ps.len = Scratch(c, sizeof(double) * (size_t)(n > 0 ? n : 1), st);
    }
    if (n == 0) return;
    CandView cv = br.cd.view();
    const double* src = br.src;
    SEL_BOOL(brute, BR,
             SEL_BOOL(field, FI,
                      SEL_STK(stk, hipLaunchKernelGGL((k_paths<BR, FI, STK, KM>), dim3(nblk(n, LEG_B)), dim3(LEG_B), 0,
                                                      st, sv, cv, a.tc, src[0], src[1], src[2], a.rx_dev,
                                                      ps.cells.as<uint64_t>(), n, ps.valid.as<uint8_t>(),
                                                      ps.amp.as<float2>(), ps.len.as<double>(),
                                                      ps.recs.as<PathRec<KM>>(), d_segs))));
    HIP_CHECK(hipGetLastError());
}

struct StageTimer {
    bool on;
    hipStream_t st;
    bool all;   // every stage, or only the marks that bracket the per-element kernel
    std::vector<hipEvent_t> ev;   // per mark, null where not recorded
    StageTimer(bool o, bool every, hipStream_t s) : on(o), st(s), all(every) {}
    // every event is a marker the device processes between kernels: record only what is asked for
    void mark(bool per_element = false, hipStream_t on_stream = nullptr) {
        hipEvent_t e = nullptr;
        if (on && (all || per_element)) {
            HIP_CHECK(hipEventCreate(&e));
            HIP_CHECK(hipEventRecord(e, on_stream ? on_stream : st));
        }
        ev.push_back(e);
    }
    ~StageTimer() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct Event {
    hipEvent_t e = nullptr;
    Event() { HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
    ~Event() { (void)hipEventDestroy(e); }
    Event(const Event&) = delete;
    Event& operator=(const Event&) = delete;
};

// events that can time the kernels between them
struct TimedEvent {
    hipEvent_t e = nullptr;
    TimedEvent() { HIP_CHECK(hipEventCreate(&e)); }
    ~TimedEvent() { (void)hipEventDestroy(e); }
    TimedEvent(const TimedEvent&) = delete;
    TimedEvent& operator=(const TimedEvent&) = delete;
};

template <int KM>
static void trace_km(Ctx& c, const TraceArgs& a, Channel& ch, TraceOut& out, bool timing, hipStream_t st)
{
    const SceneView sv = a.scene->view();
    const bool brute = (a.tc.flags & 4) != 0;
    const bool keep_hits = (a.tc.flags & 1) != 0;
    const bool keep_paths = (a.tc.flags & 2) != 0;
    const bool exhaustive = (a.tc.flags & 8) != 0;
    const bool count_work = (a.tc.flags & 16) != 0;
    const bool incoming = (a.tc.flags & 32) != 0;   // reflections Tx -> surfaces -> element
    const bool fresnel = a.tc.fresnel != 0;
    const bool keep_cir = (a.tc.flags & 256) != 0;   // per-path delays and amplitudes for rt_cir
    const int stk = stack_depth_for(*a.scene, brute);
    const int64_t R = a.R;
    const int64_t M = a.ris ? a.ris->M : 0;
    ch.R = R;
    ch.M = M;
    ch.K = a.tc.K;
    StageTimer tm(timing, (a.tc.flags & 512) != 0, st);
    tm.mark();   // 0

    // counters: [0] discovery segments, [1] leg segments, [2..4] Tx count / append / hash overflow,
    // [5..7] centre count / append / hash overflow, [8..12] work of the counting build,
    // [13] valid environment paths, [14] per-element slots whose grouped leg walk fell back,
    // [15] discovery segments of a repeated phase A (not reported)
    // 0 discovery segments, 1 legs, 2-4 Tx branch counts, 5-7 centre branch counts,
    // 8-12 work, 13 env paths, 14 leg-walk fallbacks, 15 dummy segments,
    // 16 incoming sequences, 17 incoming element paths
    // 18-20, 21-23: node visits, triangle tests, segments of the counting discovery build (Tx, centre)
    Scratch ctr(c, 8 * 24, st);
    HIP_CHECK(hipMemsetAsync(ctr.p, 0, 8 * 24, st));
    unsigned long long* d_ctr = ctr.as<unsigned long long>();
    unsigned long long* d_disc = d_ctr;
    unsigned long long* d_legs = d_ctr + 1;
    unsigned long long* d_work = d_ctr + 8;
    ch.E_env = Scratch(c, sizeof(float2) * (size_t)R, st);
    Scratch uptr, useq;
    if (a.ris) uptr = Scratch(c, sizeof(int64_t) * (size_t)(R + 1), st);
    tm.mark();   // 1

    // the Tx branch runs on `st`, the RIS-centre branch on a side stream
    Branch bt, bu;
    bt.src = a.tc.tx;
    bt.which = 0;
    bt.st = st;
    bt.d_cnt = (int64_t*)(d_ctr + 2);
    bt.d_app = d_ctr + 3;
    bt.d_work = d_ctr + 18;
    const bool time_disc = timing && (a.tc.flags & 512) != 0;
    std::unique_ptr<TimedEvent[]> ev_d(time_disc ? new TimedEvent[4] : nullptr);   // created only when asked for
    if (time_disc) {
        bt.ev_disc[0] = ev_d[0].e;
        bt.ev_disc[1] = ev_d[1].e;
    }
    const bool two = a.ris != nullptr;
    Event fork, join;
    SideStream side(c);   // returned to the pool after the join below
    if (two) {
        bu.src = a.ris->centre;
        bu.hemi = a.ris->normal;
        bu.which = 1;
        bu.st = side.s;
        bu.d_cnt = (int64_t*)(d_ctr + 5);
        bu.d_app = d_ctr + 6;
        bu.d_work = d_ctr + 21;
        if (time_disc) {
            bu.ev_disc[0] = ev_d[2].e;
            bu.ev_disc[1] = ev_d[3].e;
        }
    }
    // both hash sets are cleared here, ahead of either discovery (a clear queued
    // behind the other branch's discovery waits for free compute units)
    if (!exhaustive) {
        prepare_table(c, a, bt, st);
        if (two) prepare_table(c, a, bu, st);
    }
    if (two) {
        HIP_CHECK(hipEventRecord(fork.e, st));
        HIP_CHECK(hipStreamWaitEvent(bu.st, fork.e, 0));
    }
    // 1-3: candidates
    cand_phase_a<KM>(c, sv, stk, a, brute, exhaustive, keep_hits, ch, bt, d_disc);
    if (two) cand_phase_a<KM>(c, sv, stk, a, brute, exhaustive, keep_hits, ch, bu, d_disc);
    // the receivers in Morton order of their positions, for the geometry kernel
    // (queued behind the Tx discovery; the centre branch waits for it below)
    if (R >= ((int64_t)1 << RX_IDX_BITS)) throw inval_error("too many receivers");
    Scratch rx_order(c, sizeof(uint64_t) * (size_t)(R > 0 ? R : 1), st);
    Event rx_ready;
    if (R > 0) {
        Scratch rx_keys(c, sizeof(uint64_t) * (size_t)R, st);
        hipLaunchKernelGGL(k_rx_keys, dim3(nblk(R, 256)), dim3(256), 0, st, a.rx_dev, R, a.scene->box.as<float>(),
                           rx_keys.as<uint64_t>());
        HIP_CHECK(hipGetLastError());
        sort_keys(c, rx_keys.as<uint64_t>(), rx_order.as<uint64_t>(), R, 1, RX_IDX_BITS, 64, st);
    }
    HIP_CHECK(hipEventRecord(rx_ready.e, st));
    // Each branch goes on as soon as its own count is back, so the Tx branch
    // (launched first) does not wait for the centre branch's discovery.  An
    // overflow of a hash set repeats phase A with the next level (the
    // discovery segments were counted by the first pass).
    unsigned long long* d_dummy = d_ctr + 15;
    auto count_of = [&](Branch& br) {
        int64_t n = cand_count(c, br, exhaustive);
        while (n < 0) {
            br.table_level += 1;
            HIP_CHECK(hipMemsetAsync(br.d_app, 0, 2 * sizeof(unsigned long long), br.st));
            cand_phase_a<KM>(c, sv, stk, a, brute, exhaustive, keep_hits, ch, br, d_dummy);
            n = cand_count(c, br, exhaustive);
        }
        return n;
    };
    const int64_t n_tx = cand_phase_b(c, a, exhaustive, bt, count_of(bt));
    tm.mark();   // 2
    // 4: geometry of every (receiver, candidate)
    geo_launch<KM>(c, sv, a, bt, n_tx, rx_order.as<uint64_t>());
    const int64_t n_u0 = two ? cand_phase_b(c, a, exhaustive, bu, count_of(bu)) : 0;
    if (two) {
        HIP_CHECK(hipStreamWaitEvent(bu.st, rx_ready.e, 0));
        geo_launch<KM>(c, sv, a, bu, n_u0, rx_order.as<uint64_t>());
    }
    out.n_cand_tx = n_tx;
    out.n_cand_u = n_u0;
    // the field reaching every element, on its own stream (forked here, launched
    // after the path kernels so that they go first)
    RisView rv{};
    Scratch txm;
    Event in_fork, in_ready;
    SideStream side_in(c);
    if (a.ris) {
        rv = make_ris_view(a);
        txm = Scratch(c, sizeof(TxmRec) * (size_t)rv.M, st);
        HIP_CHECK(hipEventRecord(in_fork.e, st));
        HIP_CHECK(hipStreamWaitEvent(side_in.s, in_fork.e, 0));
    }
    // 5-6: legs and fields
    const int64_t g_tx = read_i64(bt.ps.rstart.as<int64_t>() + R, st);
    paths_launch<KM>(c, sv, stk, a, brute, true, bt, g_tx, d_legs);
    const int64_t g_u = two ? read_i64(bu.ps.rstart.as<int64_t>() + R, bu.st) : 0;
    if (two) paths_launch<KM>(c, sv, stk, a, brute, false, bu, g_u, d_legs);
    if (a.ris) {
        ris_incident<KM>(c, sv, stk, a, brute, incoming, bt, rv, d_ctr, txm.as<TxmRec>(), side_in.s);
        HIP_CHECK(hipEventRecord(in_ready.e, side_in.s));
    }

    // environment field per receiver (Tx branch)
    {
        PathSet& ps = bt.ps;
        if (R > 0) {
            hipLaunchKernelGGL(k_env_reduce, dim3(nblk(R, ENV_B / 64)), dim3(ENV_B), 0, st, ps.rstart.as<int64_t>(), R,
                               ps.valid.as<uint8_t>(), ps.amp.as<float2>(), ch.E_env.as<float2>());
            HIP_CHECK(hipGetLastError());
        }
        Scratch off2(c, sizeof(int64_t) * (size_t)(ps.n > 0 ? ps.n : 1), st);
        scan_flags(c, ps.valid.as<uint8_t>(), off2.as<int64_t>(), ps.n, (int64_t*)(d_ctr + 13), st);
        if (keep_paths) {
            const int64_t n_env = read_i64((const int64_t*)(d_ctr + 13), st);
            ch.env = Scratch(c, sizeof(EnvRec) * (size_t)n_env, st);
            if (ps.n > 0) {
                hipLaunchKernelGGL(k_env_compact<KM>, dim3(nblk(ps.n, 128)), dim3(128), 0, st, ps.recs.as<PathRec<KM>>(),
                                   bt.cd.view(), ps.valid.as<uint8_t>(), off2.as<int64_t>(), ps.amp.as<float2>(),
                                   ps.len.as<double>(), ps.n, ch.env.as<EnvRec>());
                HIP_CHECK(hipGetLastError());
            }
        }
        if (keep_cir) {   // the environment paths of every receiver, in record order
            ch.env_cells = ps.n;
            ch.env_rstart = std::move(ps.rstart);
            ch.env_valid = std::move(ps.valid);
            ch.env_amp = std::move(ps.amp);
            ch.env_len = std::move(ps.len);
        }
    }
    // sequences valid from the RIS centre, grouped by receiver (centre branch)
    int64_t n_u = 0;
    if (two) {
        PathSet& ps = bu.ps;
        hipStream_t su = bu.st;
        Scratch f2(c, (size_t)(ps.n > 0 ? ps.n : 1), su), off2(c, sizeof(int64_t) * (size_t)(ps.n > 0 ? ps.n : 1), su);
        if (ps.n > 0) {
            hipLaunchKernelGGL(k_u_flags<KM>, dim3(nblk(ps.n, 256)), dim3(256), 0, su, ps.recs.as<PathRec<KM>>(),
                               ps.valid.as<uint8_t>(), ps.n, f2.as<uint8_t>());
            HIP_CHECK(hipGetLastError());
        }
        scan_flags(c, f2.as<uint8_t>(), off2.as<int64_t>(), ps.n, bu.d_cnt, su);
        // rows for every geometric path (an upper bound of the valid ones)
        useq = Scratch(c, sizeof(int32_t) * useq_stride(KM) * (size_t)(ps.n > 0 ? ps.n : 1), su);
        if (ps.n > 0) {
            hipLaunchKernelGGL(k_u_compact<KM>, dim3(nblk(ps.n, 256)), dim3(256), 0, su, ps.recs.as<PathRec<KM>>(),
                               bu.cd.view(), f2.as<uint8_t>(), off2.as<int64_t>(), ps.n, useq.as<int32_t>());
            HIP_CHECK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_uptr_dev, dim3(nblk(R + 1, 128)), dim3(128), 0, su, ps.rstart.as<int64_t>(), ps.n,
                           off2.as<int64_t>(), bu.d_cnt, R, uptr.as<int64_t>());
        HIP_CHECK(hipGetLastError());
        if (keep_paths || keep_cir) n_u = read_i64(bu.d_cnt, su);
    }
    tm.mark();   // 3: the Tx branch's legs and field are queued on the caller's stream
    tm.mark();   // 4

    // The per-element kernel needs only the centre branch (its sequences per
    // receiver) and the field reaching the elements: it runs on the centre
    // branch's stream, beside the Tx branch's legs and field on the caller's
    // stream; the caller's stream joins it below.
    const hipStream_t sr = two ? bu.st : st;
    if (!a.ris) {
        ch.H = Scratch(c, 0, st);
        tm.mark();
        tm.mark();
    } else {
        HIP_CHECK(hipStreamWaitEvent(sr, in_ready.e, 0));   // the field reaching every element
        ch.H = Scratch(c, sizeof(float2) * (size_t)(R * M), sr);
        if (keep_paths) ch.ris_valid = Scratch(c, (size_t)((n_u + R) * M), sr);
        if (keep_paths || keep_cir) {
            ch.cir_amp = Scratch(c, sizeof(float2) * (size_t)((n_u + R) * M), sr);
            ch.cir_len = Scratch(c, sizeof(double) * (size_t)((n_u + R) * M), sr);
        }
        int n_mchunk = (int)((M + 63) / 64);
        int64_t waves = R * n_mchunk;
        int64_t threads = waves * 64;
        if (R >= ((int64_t)1 << 32)) throw inval_error("too many receivers");
        Scratch order(c, sizeof(uint64_t) * (size_t)(R > 0 ? R : 1), sr);
        if (R > 0) {
            Scratch cost(c, sizeof(uint64_t) * (size_t)R, sr);
            hipLaunchKernelGGL(k_ris_order<KM>, dim3(nblk(R, 256)), dim3(256), 0, sr, uptr.as<int64_t>(),
                               useq.as<int32_t>(), R, cost.as<uint64_t>());
            HIP_CHECK(hipGetLastError());
            // the keys come in receiver order and the sort is stable: the cost bits decide alone
            sort_keys(c, cost.as<uint64_t>(), order.as<uint64_t>(), R, 1, 32, 52, sr);
        }
        tm.mark(true, sr);   // 5
        if (threads > 0) {
            if (count_work && !brute && !keep_paths && !keep_cir) {
                SEL_STK(stk, hipLaunchKernelGGL((k_ris<false, false, STK, true, false, KM>), dim3(nblk(threads, RIS_B)),
                                                dim3(RIS_B), 0, sr, sv, a.tc, rv, txm.as<TxmRec>(), a.rx_dev, R,
                                                uptr.as<int64_t>(), useq.as<int32_t>(), order.as<uint64_t>(), n_mchunk, ch.H.as<float2>(),
                                                ch.ris_valid.as<uint8_t>(), (float2*)nullptr, (double*)nullptr, d_legs,
                                                d_work, d_ctr + 14));
            } else {
                SEL_BOOL(fresnel, FR, SEL_BOOL(brute, BR,
                         SEL_BOOL(keep_paths || keep_cir, KP,
                                  SEL_STK(stk, hipLaunchKernelGGL((k_ris<BR, KP, STK, false, FR, KM>),
                                                                  dim3(nblk(threads, RIS_B)), dim3(RIS_B), 0, sr, sv,
                                                                  a.tc, rv, txm.as<TxmRec>(), a.rx_dev, R,
                                                                  uptr.as<int64_t>(), useq.as<int32_t>(),
                                                                  order.as<uint64_t>(), n_mchunk, ch.H.as<float2>(),
                                                                  keep_paths ? ch.ris_valid.as<uint8_t>() : nullptr,
                                                                  ch.cir_amp.as<float2>(), ch.cir_len.as<double>(),
                                                                  d_legs, d_work, d_ctr + 14)))));
            }
        }
        HIP_CHECK(hipGetLastError());
        tm.mark(true, sr);   // 6
        if (keep_paths) {
            ch.n_u = n_u;
            ch.useq = std::move(useq);
        }
        if (keep_cir) ch.cir_uptr = std::move(uptr);
    }
    if (two) {   // the caller's stream joins the centre branch (and the per-element kernel)
        HIP_CHECK(hipEventRecord(join.e, sr));
        HIP_CHECK(hipStreamWaitEvent(st, join.e, 0));
    }
    ch.key_words = key_words(a.tc.K);
    ch.useq_stride = useq_stride(KM);
    if (keep_paths || keep_hits) {   // the candidate keys are small: kept with either flag
        ch.n_cand[0] = bt.cd.n;
        ch.cand_keys[0] = std::move(bt.cd.keys);
        if (two) {
            ch.n_cand[1] = bu.cd.n;
            ch.cand_keys[1] = std::move(bu.cd.keys);
        }
    }
    // temporaries of the centre branch are released on the main stream (after the join)
    if (two) {
        for (Scratch* p : {&bu.keys, &bu.cd.keys, &bu.cd.k, &bu.cd.seq, &bu.cd.img, &bu.ps.cells, &bu.ps.valid,
                           &bu.ps.amp, &bu.ps.len, &bu.ps.recs, &bu.ps.rstart})
            p->st = st;
        if (!keep_paths) useq.st = st;
    }
    int64_t h[24];
    read_i64s((const int64_t*)d_ctr, h, 24, st);
    tm.mark();   // 7
    out.disc_segments = h[0];
    out.leg_segments = h[1];
    out.segments = h[0] + h[1];
    out.n_env = h[13];
    out.n_u = h[5];
    out.n_slots = a.ris ? h[5] + R : 0;
    ch.n_env = out.n_env;
    ch.n_slots = out.n_slots;
    ch.keep_cir = keep_cir;
    for (int q = 0; q < 5; ++q) out.work[q] = h[8 + q];
    out.leg_walk_fallbacks = h[14];
    out.n_in_seq = incoming && a.ris ? h[16] : 0;
    out.n_in_paths = incoming && a.ris ? h[17] : 0;
    for (int q = 0; q < 6; ++q) out.disc_work[q] = h[18 + q];
    if (time_disc) {   // the repeats of phase A after a hash-set overflow are not timed separately
        HIP_CHECK(hipStreamSynchronize(st));
        auto el = [&](int i, int j) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev_d[i].e, ev_d[j].e) != hipSuccess) {
                (void)hipGetLastError();
                return -1.0f;
            }
            return ms;
        };
        out.ms_disc[0] = fmaxf(el(0, 1), 0.0f);
        if (two) {
            out.ms_disc[1] = fmaxf(el(2, 3), 0.0f);
            // span of both launches: from the earlier start to the later end (the two streams overlap)
            const float start_gap = el(0, 2);   // > 0: the Tx launch started first
            const float t_first = start_gap >= 0.0f ? 0.0f : -start_gap;
            const float end_tx = t_first + out.ms_disc[0];
            const float end_u = (start_gap >= 0.0f ? start_gap : 0.0f) + out.ms_disc[1];
            out.ms_disc[2] = fmaxf(end_tx, end_u);
        } else {
            out.ms_disc[2] = out.ms_disc[0];
        }
    }
    if (timing) {
        HIP_CHECK(hipStreamSynchronize(st));
        auto el = [&](int i, int j) {
            float ms = 0;
            if (tm.ev[i] && tm.ev[j]) HIP_CHECK(hipEventElapsedTime(&ms, tm.ev[i], tm.ev[j]));
            return ms;
        };
        out.ms[0] = el(0, 1);                  // setup
        out.ms[1] = el(1, 2);                  // discovery + dedupe (both sources)
        out.ms[2] = 0.0f;
        out.ms[3] = el(2, 3);                  // Tx branch: images, paths, legs, field
        out.ms[4] = 0.0f;
        out.ms[5] = a.ris ? el(5, 6) : 0.0f;   // per-element kernel (k_ris) alone, on its stream
        out.ms[6] = a.ris ? el(2, 5) : 0.0f;   // from the candidates to the start of the per-element kernel
        out.ms[7] = el(0, 7);                  // total
    }
    ch.last_stream = st;
}

void trace(Ctx& c, const TraceArgs& a, Channel& ch, TraceOut& out, bool timing, hipStream_t st)
{
    if (a.tc.K <= RT_KM_SMALL)
        trace_km<RT_KM_SMALL>(c, a, ch, out, timing, st);
    else
        trace_km<RT_MAX_K>(c, a, ch, out, timing, st);
}

// --------------------------------------------------------------------------
// Channel impulse response of one configuration (delay bins of width
// L_bin / c), bin = floor(length / L_bin): the gamma-weighted amplitudes of a
// receiver's paths summed per bin.
// --------------------------------------------------------------------------
constexpr int CIR_B = 256;
constexpr int CIR_G = 2048;   // bins per pass (two 64-bit LDS counters each)

// The records of one receiver in order: its environment paths, then its RIS
// paths slot by slot, element by element.  A thread visits records p, p +
// CIR_B, ...; the (slot, element) of a RIS record advances by a fixed step.
struct CirWalk {
    int64_t n_env, s0, M, dsl, dm, sl = -1, m = 0;
    __device__ void next(int64_t p)   // p = this thread's current record
    {
        if (sl >= 0) {
            sl += dsl;
            m += dm;
            if (m >= M) {
                m -= M;
                ++sl;
            }
        } else if (p >= n_env && M > 0) {
            const int64_t q = p - n_env;
            sl = s0 + q / M;
            m = q - (q / M) * M;
        }
    }
};

// Contribution of record p for configuration gamma: delay bin (-1: none or
// outside the window; with BIN false only whether the record is a path) and
// complex amplitude (FP64 of the FP32 inputs).
template <bool BIN>
__device__ __forceinline__ int64_t cir_term(int64_t p, const CirWalk& w, int64_t e0, int64_t n_path,
                                            const uint8_t* env_valid, const float2* env_amp, const double* env_len,
                                            const float2* camp, const double* clen, const float2* gamma,
                                            double l_bin, int64_t n_bins, double& ar, double& ai)
{
    double bin = -1.0;
    ar = 0.0;
    ai = 0.0;
    if (p < w.n_env) {
        const int64_t j = e0 + p;
        if (env_valid[j]) {
            const float2 a = env_amp[j];
            bin = BIN ? floor(env_len[j] / l_bin) : 0.0;
            ar = a.x;
            ai = a.y;
        }
    } else if (p < n_path) {
        const int64_t cell = w.sl * w.M + w.m;
        const float2 a = camp[cell];
        if (a.x != 0.0f || a.y != 0.0f) {
            const float2 g = gamma[w.m];
            bin = BIN ? floor(clen[cell] / l_bin) : 0.0;
            ar = (double)a.x * (double)g.x - (double)a.y * (double)g.y;
            ai = (double)a.x * (double)g.y + (double)a.y * (double)g.x;
        }
    }
    return bin >= 0.0 && bin < (double)n_bins ? (int64_t)bin : -1;
}

// One workgroup per receiver.  The bins are summed in fixed point: every
// term is rounded to a multiple of 2^-S, where 2^S scales the receiver's sum
// of |re| + |im| below 2^61, and added with 64-bit integer LDS atomics, so the
// result does not depend on the order of the additions (deterministic) and
// each term's rounding error is at most 2^-61 of that sum.
__global__ __launch_bounds__(CIR_B) void k_cir(const int64_t* env_rstart, const uint8_t* env_valid,
                                               const float2* env_amp, const double* env_len, const int64_t* uptr,
                                               const float2* camp, const double* clen, int64_t M, const float2* gamma,
                                               double l_bin, int64_t n_bins, float2* cir)
{
    __shared__ unsigned long long acc[2 * CIR_G];
    __shared__ double red[CIR_B];
    const int64_t r = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t e0 = env_rstart ? env_rstart[r] : 0, e1 = env_rstart ? env_rstart[r + 1] : 0;
    const int64_t s0 = uptr ? uptr[r] + r : 0, s1 = uptr ? uptr[r + 1] + r + 1 : 0;
    const int64_t n_env = e1 - e0, n_path = n_env + (s1 - s0) * M;
    const int64_t dsl = M > 0 ? CIR_B / M : 0, dm = M > 0 ? CIR_B - dsl * M : 0;
    // the scale: sum of |re| + |im| over the receiver's paths (inside the window or not), reduced in a
    // fixed order
    double sa = 0.0;
    {
        CirWalk w{n_env, s0, M, dsl, dm};
        for (int64_t p = tid; p < n_path; p += CIR_B) {
            w.next(p);
            double ar, ai;
            if (cir_term<false>(p, w, e0, n_path, env_valid, env_amp, env_len, camp, clen, gamma, l_bin, n_bins, ar,
                                ai) >= 0)
                sa += fabs(ar) + fabs(ai);
        }
    }
    red[tid] = sa;
    __syncthreads();
    for (int h = CIR_B / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    const double total = red[0];
    // total * 2^S < 2^61 (S kept in the range where 2^S is a finite double)
    const int S = total > 0.0 ? min(1000, max(-1000, 60 - ilogb(total))) : 0;
    const double scale = ldexp(1.0, S), unscale = ldexp(1.0, -S);
    for (int64_t g0 = 0; g0 < n_bins; g0 += CIR_G) {
        const int64_t gn = n_bins - g0 < CIR_G ? n_bins - g0 : CIR_G;
        for (int64_t i = tid; i < 2 * gn; i += CIR_B) acc[i] = 0ull;
        __syncthreads();
        CirWalk w{n_env, s0, M, dsl, dm};
        for (int64_t p = tid; p < n_path; p += CIR_B) {
            w.next(p);
            double ar, ai;
            const int64_t bin =
                cir_term<true>(p, w, e0, n_path, env_valid, env_amp, env_len, camp, clen, gamma, l_bin, n_bins, ar, ai);
            if (bin >= g0 && bin < g0 + gn) {
                atomicAdd(&acc[2 * (bin - g0)], (unsigned long long)(long long)rint(ar * scale));
                atomicAdd(&acc[2 * (bin - g0) + 1], (unsigned long long)(long long)rint(ai * scale));
            }
        }
        __syncthreads();
        for (int64_t i = tid; i < gn; i += CIR_B)
            cir[r * n_bins + g0 + i] = make_float2((float)((double)(long long)acc[2 * i] * unscale),
                                                   (float)((double)(long long)acc[2 * i + 1] * unscale));
        __syncthreads();
    }
}

void cir(Ctx& c, const Channel& ch, const float* gamma, double bin_s, int64_t n_bins, float* out, hipStream_t st)
{
    (void)c;
    if (ch.R == 0 || n_bins == 0) return;
    const double l_bin = 299792458.0 * bin_s;
    const bool ris = ch.M > 0 && ch.cir_uptr.bytes > 0;
    hipLaunchKernelGGL(k_cir, dim3((unsigned)ch.R), dim3(CIR_B), 0, st, ch.env_cells > 0 ? ch.env_rstart.as<int64_t>() : nullptr,
                       ch.env_valid.as<uint8_t>(), ch.env_amp.as<float2>(), ch.env_len.as<double>(),
                       ris ? ch.cir_uptr.as<int64_t>() : nullptr, ch.cir_amp.as<float2>(), ch.cir_len.as<double>(),
                       ris ? ch.M : 0, (const float2*)gamma, l_bin, n_bins, (float2*)out);
    HIP_CHECK(hipGetLastError());
}

}  // namespace rt
