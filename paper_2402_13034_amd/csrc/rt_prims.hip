// Sorting, de-duplication and scans of integer keys on the device, written
// for 64-wide wavefronts:
//
//  * LSD radix sort of keys of W 64-bit words (word 0 least significant) on a
//    bit range [begin, end), 8-bit digits, stable.  A key's rank among the
//    keys of its wave with the same digit comes from eight ballots (the lanes
//    that agree with it on every bit), so a workgroup places 1024 (or 256)
//    keys per round with no atomics.  Up to SMALL_CAP keys the whole sort runs
//    in one workgroup with the keys in LDS (one launch for all passes); larger
//    inputs take three launches per pass: per-tile digit counts, one exclusive
//    scan of the digit-major count table, and the scatter.
//  * unique of sorted keys: flag where a key differs from its predecessor,
//    scan, scatter.
//  * exclusive scans (uint8 flags or int64 values into int64, and the uint32
//    count table): per-tile sums, a scan of those (recursively), then each
//    tile scanned with its offset.
#include <cstring>

#include "rt_host.hpp"

namespace rt {

// device (or managed) memory, as opposed to host memory, pinned or not
bool is_device_ptr(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

static inline unsigned nblocks(int64_t n, int64_t b) { return (unsigned)((n + b - 1) / b); }

// --------------------------------------------------------------------------
// wave helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// 8-bit digit of a W-word key at bit `shift`, bits at or above `end` cleared
template <int W>
__device__ __forceinline__ unsigned key_digit(const uint64_t (&k)[W], int shift, int end)
{
    static_assert(W == 1 || W == 2, "keys of one or two words");
    const int off = shift & 63;
    // the word holding the digit's low bits and the next one (selected by value: no indexed registers)
    const bool upper = W == 2 && shift >= 64;
    const uint64_t lo = upper ? k[W - 1] : k[0];
    const uint64_t hi = (W == 2 && !upper) ? k[W - 1] : 0ull;
    uint64_t v = lo >> off;
    if (off > 56) v |= hi << (64 - off);
    const int width = end - shift < 8 ? end - shift : 8;
    return (unsigned)(v & ((1u << width) - 1u));
}

// Lanes of the wave holding the same digit as this lane (among `valid` lanes):
// this lane's rank among them (lower lanes first) and their count.
__device__ __forceinline__ void wave_multisplit(unsigned d, bool valid, unsigned& rank, unsigned& count)
{
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    const int lane = lane_id();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    rank = (unsigned)__popcll(peers & below);
    count = (unsigned)__popcll(peers);
}

template <class T>
__device__ __forceinline__ T wave_inclusive_add(T v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread over a workgroup of NT threads (NT/64
// waves); `wsum` is LDS for NT/64 values.  Returns the exclusive prefix and
// the workgroup total in *total.
template <class T, int NT>
__device__ __forceinline__ T block_exclusive_add(T v, T* wsum, T* total)
{
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    const T inc = wave_inclusive_add(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const T s = wsum[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// --------------------------------------------------------------------------
// scans
// --------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_IPT = 8, SCAN_TILE = SCAN_T * SCAN_IPT;

template <class In, class Out>
__global__ __launch_bounds__(SCAN_T) void k_scan_partials(const In* in, int64_t n, Out* part)
{
    __shared__ Out wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    Out s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j)
        if (base + j < n) s += (Out)in[base + j];
    Out tot;
    (void)block_exclusive_add<Out, SCAN_T>(s, wsum, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// out[i] = offset of the tile + exclusive prefix within it; the last tile
// writes the grand total to *total (if given)
template <class In, class Out>
__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(const In* in, int64_t n, const Out* tile_off, Out* out,
                                                       Out* total)
{
    __shared__ Out wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    Out v[SCAN_IPT];
    Out s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        v[j] = base + j < n ? (Out)in[base + j] : (Out)0;
        s += v[j];
    }
    Out tot;
    Out run = block_exclusive_add<Out, SCAN_T>(s, wsum, &tot) + (tile_off ? tile_off[blockIdx.x] : (Out)0);
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *total = (tile_off ? tile_off[blockIdx.x] : (Out)0) + tot;
}

template <class In, class Out>
static void scan_exclusive(Ctx& c, const In* in, Out* out, int64_t n, Out* d_total, hipStream_t st)
{
    if (n <= 0) {
        if (d_total) HIP_CHECK(hipMemsetAsync(d_total, 0, sizeof(Out), st));
        return;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL((k_scan_tiles<In, Out>), dim3(1), dim3(SCAN_T), 0, st, in, n, (const Out*)nullptr, out,
                           d_total);
        HIP_CHECK(hipGetLastError());
        return;
    }
    Scratch part(c, sizeof(Out) * (size_t)nb, st), off(c, sizeof(Out) * (size_t)nb, st);
    hipLaunchKernelGGL((k_scan_partials<In, Out>), dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, n, part.as<Out>());
    HIP_CHECK(hipGetLastError());
    scan_exclusive<Out, Out>(c, part.as<Out>(), off.as<Out>(), nb, (Out*)nullptr, st);
    hipLaunchKernelGGL((k_scan_tiles<In, Out>), dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, n,
                       (const Out*)off.as<Out>(), out, d_total);
    HIP_CHECK(hipGetLastError());
}

void scan_flags(Ctx& c, const uint8_t* flags, int64_t* offsets, int64_t n, int64_t* d_total, hipStream_t st)
{
    scan_exclusive<uint8_t, int64_t>(c, flags, offsets, n, d_total, st);
}

void scan_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n, hipStream_t st)
{
    scan_exclusive<int64_t, int64_t>(c, in, out, n, (int64_t*)nullptr, st);
}

// --------------------------------------------------------------------------
// radix sort, one workgroup, keys in LDS
// --------------------------------------------------------------------------
constexpr int SMALL_T = 1024;                    // threads (16 waves)
constexpr int SMALL_WORDS = 8192;                // 64-bit words per LDS buffer (64 KiB)

// A pass over a digit that every key shares is the identity (the sort is
// stable): the bits that vary (OR ^ AND over all keys) decide which passes run.
template <int W>
__global__ __launch_bounds__(SMALL_T) void k_sort_small(const uint64_t* in, uint64_t* out, int n, int begin, int end)
{
    __shared__ uint64_t buf[2][SMALL_WORDS];
    __shared__ unsigned wc[SMALL_T / 64][256];   // per wave and digit: count, then start
    __shared__ unsigned hist[256];
    __shared__ unsigned wsum[4];
    __shared__ uint64_t wor[SMALL_T / 64][W], wand[SMALL_T / 64][W];
    const int t = (int)threadIdx.x, wave = t >> 6;
    uint64_t vo[W], va[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        vo[j] = 0ull;
        va[j] = ~0ull;
    }
    for (int i = t; i < n; i += SMALL_T) {
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const uint64_t v = in[i * W + j];
            buf[0][i * W + j] = v;
            vo[j] |= v;
            va[j] &= v;
        }
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        for (int o = 32; o > 0; o >>= 1) {
            vo[j] |= (uint64_t)__shfl_xor((long long)vo[j], o, 64);
            va[j] &= (uint64_t)__shfl_xor((long long)va[j], o, 64);
        }
        if ((t & 63) == 0) {
            wor[wave][j] = vo[j];
            wand[wave][j] = va[j];
        }
    }
    __syncthreads();
    uint64_t vary[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        uint64_t o = 0ull, a = ~0ull;
        for (int w = 0; w < SMALL_T / 64; ++w) {
            o |= wor[w][j];
            a &= wand[w][j];
        }
        vary[j] = n > 0 ? (o ^ a) : 0ull;
    }
    int src = 0;
    for (int shift = begin; shift < end; shift += 8) {
        if (key_digit<W>(vary, shift, end) == 0u) continue;   // same on every thread
        if (t < 256) hist[t] = 0;
        __syncthreads();
        for (int i = t; i < n; i += SMALL_T) {
            uint64_t k[W];
#pragma unroll
            for (int j = 0; j < W; ++j) k[j] = buf[src][i * W + j];
            atomicAdd(&hist[key_digit<W>(k, shift, end)], 1u);
        }
        __syncthreads();
        // digit starts: exclusive scan of the 256 counts by the first four waves
        unsigned start = 0;
        if (t < 256) {
            const unsigned h = hist[t];
            const unsigned inc = wave_inclusive_add(h);
            if ((t & 63) == 63) wsum[t >> 6] = inc;
            start = inc - h;
        }
        __syncthreads();
        if (t < 256) {
            for (int w = 0; w < (t >> 6); ++w) start += wsum[w];
            hist[t] = start;   // running start of each digit
        }
        for (int c0 = 0; c0 < n; c0 += SMALL_T) {
            const int i = c0 + t;
            const bool valid = i < n;
            uint64_t k[W];
#pragma unroll
            for (int j = 0; j < W; ++j) k[j] = valid ? buf[src][i * W + j] : 0ull;
            const unsigned d = valid ? key_digit<W>(k, shift, end) : 0u;
            unsigned rank, cnt;
            wave_multisplit(d, valid, rank, cnt);
            for (int e = t; e < (SMALL_T / 64) * 256; e += SMALL_T) (&wc[0][0])[e] = 0;
            __syncthreads();
            if (valid && rank == 0) wc[wave][d] = cnt;
            __syncthreads();
            if (t < 256) {
                unsigned run = hist[t];
                for (int w = 0; w < SMALL_T / 64; ++w) {
                    const unsigned x = wc[w][t];
                    wc[w][t] = run;
                    run += x;
                }
                hist[t] = run;
            }
            __syncthreads();
            if (valid) {
                const unsigned pos = wc[wave][d] + rank;
#pragma unroll
                for (int j = 0; j < W; ++j) buf[src ^ 1][pos * W + j] = k[j];
            }
            __syncthreads();
        }
        src ^= 1;
    }
    __syncthreads();
    for (int i = t; i < n * W; i += SMALL_T) out[i] = buf[src][i];
}

// --------------------------------------------------------------------------
// radix sort, many workgroups
// --------------------------------------------------------------------------
constexpr int RS_T = 256, RS_KPT = 8, RS_TILE = RS_T * RS_KPT;

// digit counts of one tile into cnt[digit * n_tiles + tile]
template <int W>
__global__ __launch_bounds__(RS_T) void k_rs_count(const uint64_t* keys, int64_t n, int shift, int end,
                                                   unsigned* cnt, int n_tiles)
{
    __shared__ unsigned h[256];
    const int t = (int)threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int j = 0; j < RS_KPT; ++j) {
        const int64_t i = base + j * RS_T + t;
        if (i < n) {
            uint64_t k[W];
#pragma unroll
            for (int q = 0; q < W; ++q) k[q] = keys[i * W + q];
            atomicAdd(&h[key_digit<W>(k, shift, end)], 1u);
        }
    }
    __syncthreads();
    cnt[(int64_t)t * n_tiles + blockIdx.x] = h[t];
}

// keys of one tile to their places: start[digit * n_tiles + tile] (the scanned
// counts) plus the rank among the tile's earlier keys with that digit
template <int W>
__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint64_t* keys, uint64_t* out, int64_t n, int shift,
                                                     int end, const unsigned* start, int n_tiles)
{
    __shared__ unsigned wc[RS_T / 64][256];
    __shared__ unsigned run[256];
    const int t = (int)threadIdx.x, wave = t >> 6;
    run[t] = start[(int64_t)t * n_tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = 0; j < RS_KPT; ++j) {
        const int64_t i = base + j * RS_T + t;
        const bool valid = i < n;
        uint64_t k[W];
#pragma unroll
        for (int q = 0; q < W; ++q) k[q] = valid ? keys[i * W + q] : 0ull;
        const unsigned d = valid ? key_digit<W>(k, shift, end) : 0u;
        unsigned rank, c;
        wave_multisplit(d, valid, rank, c);
#pragma unroll
        for (int w = 0; w < RS_T / 64; ++w) wc[w][t] = 0;
        __syncthreads();
        if (valid && rank == 0) wc[wave][d] = c;
        __syncthreads();
        {
            unsigned r = run[t];
#pragma unroll
            for (int w = 0; w < RS_T / 64; ++w) {
                const unsigned x = wc[w][t];
                wc[w][t] = r;
                r += x;
            }
            run[t] = r;
        }
        __syncthreads();
        if (valid) {
            const int64_t pos = (int64_t)wc[wave][d] + rank;
#pragma unroll
            for (int q = 0; q < W; ++q) out[pos * W + q] = k[q];
        }
        __syncthreads();
    }
}

template <int W>
static void sort_keys_w(Ctx& c, uint64_t* in, uint64_t* out, int64_t n, int begin, int end, hipStream_t st)
{
    if (n <= 0) return;
    if (n == 1 || begin >= end) {
        if (in != out) HIP_CHECK(hipMemcpyAsync(out, in, sizeof(uint64_t) * W * (size_t)n, hipMemcpyDeviceToDevice, st));
        return;
    }
    if (n * W <= SMALL_WORDS) {
        hipLaunchKernelGGL((k_sort_small<W>), dim3(1), dim3(SMALL_T), 0, st, in, out, (int)n, begin, end);
        HIP_CHECK(hipGetLastError());
        return;
    }
    if (n >= ((int64_t)1 << 32)) throw inval_error("too many keys to sort");
    const int n_tiles = (int)((n + RS_TILE - 1) / RS_TILE);
    const int64_t table = (int64_t)256 * n_tiles;
    Scratch cnt(c, sizeof(unsigned) * (size_t)table, st), start(c, sizeof(unsigned) * (size_t)table, st);
    uint64_t* bufs[2] = {in, out};
    int src = 0;
    for (int shift = begin; shift < end; shift += 8) {
        hipLaunchKernelGGL((k_rs_count<W>), dim3((unsigned)n_tiles), dim3(RS_T), 0, st, bufs[src], n, shift, end,
                           cnt.as<unsigned>(), n_tiles);
        HIP_CHECK(hipGetLastError());
        scan_exclusive<unsigned, unsigned>(c, cnt.as<unsigned>(), start.as<unsigned>(), table, (unsigned*)nullptr, st);
        hipLaunchKernelGGL((k_rs_scatter<W>), dim3((unsigned)n_tiles), dim3(RS_T), 0, st, bufs[src], bufs[src ^ 1], n,
                           shift, end, (const unsigned*)start.as<unsigned>(), n_tiles);
        HIP_CHECK(hipGetLastError());
        src ^= 1;
    }
    if (bufs[src] != out)
        HIP_CHECK(hipMemcpyAsync(out, bufs[src], sizeof(uint64_t) * W * (size_t)n, hipMemcpyDeviceToDevice, st));
}

void sort_keys(Ctx& c, uint64_t* in, uint64_t* out, int64_t n, int words, int begin_bit, int end_bit, hipStream_t st)
{
    if (words == 1)
        sort_keys_w<1>(c, in, out, n, begin_bit, end_bit, st);
    else if (words == 2)
        sort_keys_w<2>(c, in, out, n, begin_bit, end_bit, st);
    else
        throw inval_error("keys of 1 or 2 words");
}

// keys_in sorted into keys_out (keys_in is left in an unspecified order)
void sort_u64_into(Ctx& c, uint64_t* keys_in, uint64_t* keys_out, int64_t n, int end_bit, hipStream_t st)
{
    sort_keys_w<1>(c, keys_in, keys_out, n, 0, end_bit, st);
}

void sort_u64(Ctx& c, uint64_t* keys, int64_t n, int end_bit, hipStream_t st)
{
    if (n <= 1) return;
    if (n <= SMALL_WORDS) {   // in place: the workgroup holds every key in LDS
        sort_keys_w<1>(c, keys, keys, n, 0, end_bit, st);
        return;
    }
    Scratch tmp(c, sizeof(uint64_t) * (size_t)n, st);
    sort_keys_w<1>(c, keys, tmp.as<uint64_t>(), n, 0, end_bit, st);
    HIP_CHECK(hipMemcpyAsync(keys, tmp.p, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
}

// --------------------------------------------------------------------------
// unique of sorted keys
// --------------------------------------------------------------------------
template <int W>
__global__ void k_unique_flags(const uint64_t* keys, int64_t n, uint8_t* flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool first = i == 0;
    if (!first)
#pragma unroll
        for (int q = 0; q < W; ++q) first |= keys[i * W + q] != keys[(i - 1) * W + q];
    flag[i] = first ? 1 : 0;
}

template <int W>
__global__ void k_unique_scatter(const uint64_t* keys, int64_t n, const uint8_t* flag, const int64_t* off,
                                 uint64_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
#pragma unroll
    for (int q = 0; q < W; ++q) out[off[i] * W + q] = keys[i * W + q];
}

void unique_keys(Ctx& c, const uint64_t* in, uint64_t* out, int64_t n, int words, int64_t* d_count, hipStream_t st)
{
    if (words != 1 && words != 2) throw inval_error("keys of 1 or 2 words");
    Scratch flag(c, (size_t)(n > 0 ? n : 1), st), off(c, sizeof(int64_t) * (size_t)(n > 0 ? n : 1), st);
    if (n > 0) {
        if (words == 1)
            hipLaunchKernelGGL(k_unique_flags<1>, dim3(nblocks(n, 256)), dim3(256), 0, st, in, n, flag.as<uint8_t>());
        else
            hipLaunchKernelGGL(k_unique_flags<2>, dim3(nblocks(n, 256)), dim3(256), 0, st, in, n, flag.as<uint8_t>());
        HIP_CHECK(hipGetLastError());
    }
    scan_flags(c, flag.as<uint8_t>(), off.as<int64_t>(), n, d_count, st);
    if (n > 0) {
        if (words == 1)
            hipLaunchKernelGGL(k_unique_scatter<1>, dim3(nblocks(n, 256)), dim3(256), 0, st, in, n,
                               (const uint8_t*)flag.as<uint8_t>(), (const int64_t*)off.as<int64_t>(), out);
        else
            hipLaunchKernelGGL(k_unique_scatter<2>, dim3(nblocks(n, 256)), dim3(256), 0, st, in, n,
                               (const uint8_t*)flag.as<uint8_t>(), (const int64_t*)off.as<int64_t>(), out);
        HIP_CHECK(hipGetLastError());
    }
}

void unique_u64(Ctx& c, const uint64_t* in, uint64_t* out, int64_t n, int64_t* d_count, hipStream_t st)
{
    unique_keys(c, in, out, n, 1, d_count, st);
}

}  // namespace rt
