// Coherent RIS sum over many configurations (eqs. (9)-(10)):
//   E[r, c] = E_env[r] + scale * sum_m H[r, m] Gamma[m, c],  P = |E|^2 / (2 eta0).
//
// RT_PREC_VALU_F32: FP32 complex multiply-add, LDS-tiled, vector ALUs.
// RT_PREC_MFMA_*:   the complex product as one real GEMM on the matrix cores:
//   rows 2r / 2r+1 of A give Re / Im of E[r, :];
//   real Gamma:    A[2r] = Re H[r, :],            A[2r+1] = Im H[r, :],           B = Re Gamma
//   complex Gamma: A[2r] = [Re H, -Im H],         A[2r+1] = [Im H, Re H],         B = [Re G; Im G]
//   H is split into hi + lo (hi = RNE(x), lo = RNE(x - hi)); Gamma into hi (and lo for X3);
//   products hi*hi + lo*hi (+ hi*lo) accumulate in FP32 on the matrix cores:
//   bf16 (v_mfma_f32_32x32x16_bf16), or fp16 (v_mfma_f32_32x32x16_f16) with
//   each receiver's two rows scaled by a power of two 2^s_r that brings their
//   largest magnitude into [2^14, 2^15) (fp16 has 5 exponent bits: unscaled
//   fields of 1e-6 V/m would be subnormal); the epilogue multiplies by 2^-s_r.
//   The epilogue adds E_env, scales, and writes E and/or P.
#include <algorithm>
#include <cstring>

#include "rt_host.hpp"

namespace rt {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

#define ETA0_F 376.99111843077515f  // 120 pi

// --------------------------------------------------------------------------
// VALU path
// --------------------------------------------------------------------------
constexpr int VT = 64;   // tile of receivers and of configurations
constexpr int VK = 16;   // k tile
constexpr int VN = 4;    // configurations of the narrow kernel (one per thread)

// One complex multiply-add of the VALU sums, as four explicit FMAs in a fixed
// order: both VALU kernels take it over the elements in increasing order, so
// an output does not depend on which kernel, tile or batch of configurations
// computed it.
__device__ __forceinline__ void cmac(float2 h, float2 g, float& ar, float& ai)
{
    ar = __builtin_fmaf(h.x, g.x, ar);
    ar = __builtin_fmaf(-h.y, g.y, ar);
    ai = __builtin_fmaf(h.x, g.y, ai);
    ai = __builtin_fmaf(h.y, g.x, ai);
}

__global__ __launch_bounds__(256) void k_sum_valu(const float2* H, const float2* G, const float2* Eenv, int64_t R,
                                                  int64_t M, int64_t C, float scale, float2* Eout, float* Pout)
{
    __shared__ float2 sh[VK][VT + 1];
    __shared__ float2 sg[VK][VT + 1];
    int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    int64_t r0 = (int64_t)blockIdx.y * VT, c0 = (int64_t)blockIdx.x * VT;
    float accr[4][4], acci[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) accr[i][j] = acci[i][j] = 0.0f;
    for (int64_t k0 = 0; k0 < M; k0 += VK) {
        for (int e = threadIdx.x; e < VK * VT; e += 256) {
            int kk = e / VT, rr = e % VT;
            int64_t r = r0 + rr, m = k0 + kk;
            sh[kk][rr] = (r < R && m < M) ? H[r * M + m] : make_float2(0.0f, 0.0f);
            int64_t cc = c0 + rr;
            sg[kk][rr] = (cc < C && m < M) ? G[m * C + cc] : make_float2(0.0f, 0.0f);
        }
        __syncthreads();
        for (int kk = 0; kk < VK; ++kk) {
            float2 h[4], g[4];
            for (int i = 0; i < 4; ++i) h[i] = sh[kk][ty * 4 + i];
            for (int j = 0; j < 4; ++j) g[j] = sg[kk][tx * 4 + j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) cmac(h[i], g[j], accr[i][j], acci[i][j]);
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i) {
        int64_t r = r0 + ty * 4 + i;
        if (r >= R) continue;
        float2 e0 = Eenv[r];
        for (int j = 0; j < 4; ++j) {
            int64_t c = c0 + tx * 4 + j;
            if (c >= C) continue;
            float er = e0.x + scale * accr[i][j];
            float ei = e0.y + scale * acci[i][j];
            if (Eout) Eout[r * C + c] = make_float2(er, ei);
            if (Pout) Pout[r * C + c] = (er * er + ei * ei) / (2.0f * ETA0_F);
        }
    }
}

// Few configurations (C <= VN): a block takes 64 receivers x VN configurations,
// one output per thread, so a one-configuration sum still spreads over R / 64
// blocks instead of filling 1/64 of a square tile.
__global__ __launch_bounds__(256) void k_sum_valu_narrow(const float2* H, const float2* G, const float2* Eenv,
                                                         int64_t R, int64_t M, int64_t C, float scale, float2* Eout,
                                                         float* Pout)
{
    __shared__ float2 sh[VK][VT + 1];
    __shared__ float2 sg[VK][VN];
    const int j = threadIdx.x & (VN - 1), i = threadIdx.x / VN;   // configuration, receiver in the tile
    const int64_t r0 = (int64_t)blockIdx.x * VT;
    float ar = 0.0f, ai = 0.0f;
    for (int64_t k0 = 0; k0 < M; k0 += VK) {
        for (int e = threadIdx.x; e < VK * VT; e += 256) {
            const int rr = e / VK, kk = e % VK;   // consecutive threads: consecutive elements of a row
            const int64_t r = r0 + rr, m = k0 + kk;
            sh[kk][rr] = (r < R && m < M) ? H[r * M + m] : make_float2(0.0f, 0.0f);
        }
        if (threadIdx.x < VK * VN) {
            const int kk = threadIdx.x / VN, cc = threadIdx.x % VN;
            const int64_t m = k0 + kk;
            sg[kk][cc] = (cc < C && m < M) ? G[m * C + cc] : make_float2(0.0f, 0.0f);
        }
        __syncthreads();
        for (int kk = 0; kk < VK; ++kk) cmac(sh[kk][i], sg[kk][j], ar, ai);
        __syncthreads();
    }
    const int64_t r = r0 + i;
    if (r < R && j < C) {
        const float2 e0 = Eenv[r];
        const float er = e0.x + scale * ar;
        const float ei = e0.y + scale * ai;
        if (Eout) Eout[r * C + j] = make_float2(er, ei);
        if (Pout) Pout[r * C + j] = (er * er + ei * ei) / (2.0f * ETA0_F);
    }
}

// --------------------------------------------------------------------------
// bf16 split helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f16_rne(float x)
{
    const _Float16 h = (_Float16)x;   // round to nearest even
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}
__device__ __forceinline__ float f16_to_f(uint16_t b)
{
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    return (float)h;
}

// fp16 split: per receiver, the power of two s_r with max |Re H|, |Im H| of the
// row times 2^s_r in [2^14, 2^15) (s_r = 0 for an all-zero row); one wave per receiver
__global__ void k_row_scale(const float2* H, int64_t R, int64_t M, int32_t* sexp)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (r >= R) return;
    const int lane = threadIdx.x & 63;
    float m = 0.0f;
    for (int64_t k = lane; k < M; k += 64) {
        const float2 h = H[r * M + k];
        m = fmaxf(m, fmaxf(fabsf(h.x), fabsf(h.y)));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (lane == 0) sexp[r] = m > 0.0f ? 14 - ilogbf(m) : 0;
}

// A [rows_p x kp] row-major (k fastest); layout 1 = real Gamma, 2 = complex Gamma;
// sexp: per-receiver scale exponents of the fp16 split (nullptr: bf16)
__global__ void k_split_A(const float2* H, int64_t R, int64_t M, int layout, int64_t rows_p, int64_t kp,
                          const int32_t* sexp, uint16_t* Ahi, uint16_t* Alo)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows_p * kp) return;
    int64_t row = idx / kp, k = idx - row * kp;
    int64_t r = row >> 1;
    int part = (int)(row & 1);
    float v = 0.0f;
    if (r < R) {
        if (layout == 1) {
            if (k < M) v = part == 0 ? H[r * M + k].x : H[r * M + k].y;
        } else {
            if (k < M) v = part == 0 ? H[r * M + k].x : H[r * M + k].y;
            else if (k < 2 * M) v = part == 0 ? -H[r * M + k - M].y : H[r * M + k - M].x;
        }
    }
    if (sexp) {
        v = r < R ? ldexpf(v, sexp[r]) : 0.0f;
        const uint16_t hi = f16_rne(v);
        Ahi[idx] = hi;
        Alo[idx] = f16_rne(v - f16_to_f(hi));
        return;
    }
    uint16_t hi = bf16_rne(v);
    Ahi[idx] = hi;
    Alo[idx] = bf16_rne(v - bf16_to_f(hi));
}

// Bt [cols_p x kp] (k fastest) from Gamma [M x C] (c fastest): a 64 x 64
// transpose through LDS per workgroup, so both the reads (along c) and the
// writes (along k) are contiguous
constexpr int SBT = 64;
__global__ __launch_bounds__(256) void k_split_B(const float2* G, int64_t M, int64_t C, int layout, int64_t cols_p,
                                                 int64_t kp, bool f16, uint16_t* Bhi, uint16_t* Blo)
{
    __shared__ float tile[SBT][SBT + 1];
    const int64_t c0 = (int64_t)blockIdx.x * SBT, k0 = (int64_t)blockIdx.y * SBT;
    for (int i = threadIdx.x; i < SBT * SBT; i += 256) {
        const int kk = i / SBT, cc = i % SBT;
        const int64_t k = k0 + kk, c = c0 + cc;
        float v = 0.0f;
        if (c < C) {
            if (k < M) v = G[k * C + c].x;
            else if (layout == 2 && k < 2 * M) v = G[(k - M) * C + c].y;
        }
        tile[kk][cc] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SBT * SBT; i += 256) {
        const int cc = i / SBT, kk = i % SBT;
        const int64_t k = k0 + kk, c = c0 + cc;
        if (c >= cols_p || k >= kp) continue;
        const float v = tile[kk][cc];
        const int64_t idx = c * kp + k;
        if (f16) {
            const uint16_t hi = f16_rne(v);
            Bhi[idx] = hi;
            if (Blo) Blo[idx] = f16_rne(v - f16_to_f(hi));
        } else {
            const uint16_t hi = bf16_rne(v);
            Bhi[idx] = hi;
            if (Blo) Blo[idx] = bf16_rne(v - bf16_to_f(hi));
        }
    }
}

// --------------------------------------------------------------------------
// MFMA GEMM: 128 x 128 tile, 4 waves (each 64 x 64 = 2 x 2 blocks of 32 x 32), BK = 32
// --------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int GBM = 128, GBN = 128, GBK = 32;
constexpr int LDA = GBK + 8;   // padded row (bf16 elements)

// one 32 x 32 x 16 product of 8-element operands, bf16 or fp16
template <bool F16>
__device__ __forceinline__ f32x16 mfma16(const uint16_t* a, const uint16_t* b, f32x16 acc)
{
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(*(const f16x8*)a, *(const f16x8*)b, acc, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)a, *(const bf16x8*)b, acc, 0, 0, 0);
}

// sexp: per-receiver scale exponents of the fp16 split (F16 only)
template <int NT, bool F16>
__global__ __launch_bounds__(256) void k_sum_mfma(const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo,
                                                  const uint16_t* __restrict__ Bhi, const uint16_t* __restrict__ Blo,
                                                  int64_t kp, const float2* __restrict__ Eenv,
                                                  const int32_t* __restrict__ sexp, int64_t R, int64_t C,
                                                  float scale, float2* Eout, float* Pout, int n_tiles_n)
{
    __shared__ __attribute__((aligned(16))) uint16_t sAh[GBM * LDA];
    __shared__ __attribute__((aligned(16))) uint16_t sAl[GBM * LDA];
    __shared__ __attribute__((aligned(16))) uint16_t sBh[GBN * LDA];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[(NT == 3 ? GBN : 1) * LDA];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t tile_m = blockIdx.x / n_tiles_n, tile_n = blockIdx.x % n_tiles_n;
    const int64_t row0 = tile_m * GBM, col0 = tile_n * GBN;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

    f32x16 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    // each thread moves 16 bf16 (two 16-byte vectors) of each 128 x 32 tile
    const int lrow = tid >> 1, lcol = (tid & 1) * 16;
    const uint4* gAh = (const uint4*)(Ahi + (row0 + lrow) * kp + lcol);
    const uint4* gAl = (const uint4*)(Alo + (row0 + lrow) * kp + lcol);
    const uint4* gBh = (const uint4*)(Bhi + (col0 + lrow) * kp + lcol);
    const uint4* gBl = NT == 3 ? (const uint4*)(Blo + (col0 + lrow) * kp + lcol) : nullptr;

    uint4 rAh0 = gAh[0], rAh1 = gAh[1], rAl0 = gAl[0], rAl1 = gAl[1], rBh0 = gBh[0], rBh1 = gBh[1];
    uint4 rBl0 = make_uint4(0, 0, 0, 0), rBl1 = rBl0;
    if (NT == 3) {
        rBl0 = gBl[0];
        rBl1 = gBl[1];
    }
    const int64_t nk = kp / GBK;
    for (int64_t kt = 0; kt < nk; ++kt) {
        *(uint4*)&sAh[lrow * LDA + lcol] = rAh0;
        *(uint4*)&sAh[lrow * LDA + lcol + 8] = rAh1;
        *(uint4*)&sAl[lrow * LDA + lcol] = rAl0;
        *(uint4*)&sAl[lrow * LDA + lcol + 8] = rAl1;
        *(uint4*)&sBh[lrow * LDA + lcol] = rBh0;
        *(uint4*)&sBh[lrow * LDA + lcol + 8] = rBh1;
        if (NT == 3) {
            *(uint4*)&sBl[lrow * LDA + lcol] = rBl0;
            *(uint4*)&sBl[lrow * LDA + lcol + 8] = rBl1;
        }
        __syncthreads();
        if (kt + 1 < nk) {
            const int64_t o = (kt + 1) * GBK / 8;   // in uint4 units
            rAh0 = gAh[o];
            rAh1 = gAh[o + 1];
            rAl0 = gAl[o];
            rAl1 = gAl[o + 1];
            rBh0 = gBh[o];
            rBh1 = gBh[o + 1];
            if (NT == 3) {
                rBl0 = gBl[o];
                rBl1 = gBl[o + 1];
            }
        }
        for (int ks = 0; ks < GBK; ks += 16) {
            const int kofs = ks + (lane >> 5) * 8;
            uint4 ah[2], al[2], bh[2], bl[2];
            for (int i = 0; i < 2; ++i) {
                const int r = wm + i * 32 + (lane & 31);
                ah[i] = *(const uint4*)&sAh[r * LDA + kofs];
                al[i] = *(const uint4*)&sAl[r * LDA + kofs];
            }
            for (int j = 0; j < 2; ++j) {
                const int cix = wn + j * 32 + (lane & 31);
                bh[j] = *(const uint4*)&sBh[cix * LDA + kofs];
                if (NT == 3) bl[j] = *(const uint4*)&sBl[cix * LDA + kofs];
            }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = mfma16<F16>((const uint16_t*)&ah[i], (const uint16_t*)&bh[j], acc[i][j]);
                    acc[i][j] = mfma16<F16>((const uint16_t*)&al[i], (const uint16_t*)&bh[j], acc[i][j]);
                    if (NT == 3) acc[i][j] = mfma16<F16>((const uint16_t*)&ah[i], (const uint16_t*)&bl[j], acc[i][j]);
                }
        }
        __syncthreads();
    }
    // epilogue: lane holds column (lane & 31); values e: row 8 (e / 4) + 4 (lane / 32) + (e % 4)
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int64_t c = col0 + wn + j * 32 + (lane & 31);
            for (int e = 0; e < 16; e += 2) {
                const int64_t row = row0 + wm + i * 32 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
                const int64_t r = row >> 1;
                if (r >= R || c >= C) continue;
                float2 e0 = Eenv[r];
                const float sr = F16 ? ldexpf(scale, -sexp[r]) : scale;   // exact: a power of two
                float er = e0.x + sr * acc[i][j][e];
                float ei = e0.y + sr * acc[i][j][e + 1];
                if (Eout) Eout[r * C + c] = make_float2(er, ei);
                if (Pout) Pout[r * C + c] = (er * er + ei * ei) / (2.0f * ETA0_F);
            }
        }
}

// Two-product split (H hi + lo against Gamma hi) on 256 x 256 tiles: 8 waves
// (4 x 2), each 64 x 128 outputs = 2 x 4 blocks of 32 x 32, so every A
// fragment (hi and lo) read from LDS feeds four blocks and every B fragment four.
//
// Operand tiles of K = 32 come straight from global memory into LDS
// (buffer_load_dwordx4 ... lds: no staging registers), three stages deep, so
// two tiles are in flight while one is multiplied.  An LDS row is 64 bytes
// (four 16-byte chunks); chunk c of row r sits at position c ^ swz(r), which
// keeps both the 64-lane fragment reads and the direct loads free of bank
// conflicts.  Within a tile the second half (k 16..31) is read from LDS while
// the first half's products run, and the next tile's first half is read right
// after the barrier, while the second half's products run.
//
// Persistent: one workgroup per CU walks tiles t = blockIdx.x + i * gridDim.x;
// the next tile's three stages are loaded during this tile's epilogue.
// XCD-aware order (gh > 0): workgroups are placed on the 8 XCDs round-robin
// by index, so tile t is given to XCD t % 8; each XCD owns a band of n_tm / 8
// tile rows and walks it in groups of gh tile rows, column by column, which
// keeps the A rows and B columns its CUs share in that XCD's L2.
constexpr int G2M = 256, G2N = 256, G2K = 32;
constexpr int G2R = 32;                 // LDS row length (elements)
constexpr int G2OP = G2M * G2R;         // elements of one operand tile in LDS
constexpr int G2_STAGE_WAIT_1 = 0x0076;   // s_waitcnt vmcnt(6) lgkmcnt(0): one later tile's loads may fly
constexpr int G2_STAGE_WAIT_0 = 0x0070;   // s_waitcnt vmcnt(0) lgkmcnt(0)
constexpr int G2_STAGE_WAIT_2 = 0x007C;   // s_waitcnt vmcnt(12) lgkmcnt(0): two later tiles' loads may fly
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int g2_swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// a barrier after an explicit wait: the direct loads are counted by vmcnt only,
// so the wait names how many of this wave's later loads may still be in flight
#define G2_SYNC(WAIT)                          \
    do {                                       \
        __builtin_amdgcn_s_waitcnt(WAIT);      \
        asm volatile("" ::: "memory");         \
        __builtin_amdgcn_s_barrier();          \
        asm volatile("" ::: "memory");         \
    } while (0)

template <bool F16>
__global__ __launch_bounds__(512) void k_sum_mfma_2x(const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo,
                                                     const uint16_t* __restrict__ Bhi, int64_t kp,
                                                     const float2* __restrict__ Eenv, const int32_t* __restrict__ sexp,
                                                     int64_t R, int64_t C, float scale, float2* Eout, float* Pout,
                                                     int n_tm, int n_tn, int gh)
{
    // three stages, each [A hi | A lo | B] of 256 rows x 32; separate arrays so
    // that a read of one stage never waits for the direct loads into another
    __shared__ __attribute__((aligned(1024))) uint16_t st0[3 * G2OP];
    __shared__ __attribute__((aligned(1024))) uint16_t st1[3 * G2OP];
    __shared__ __attribute__((aligned(1024))) uint16_t st2[3 * G2OP];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 128;
    const int T = n_tm * n_tn;
    const int64_t nk = kp / G2K;
    auto tile_of = [&](int t, int& tm, int& tn) {
        if (gh == 0) {
            tm = t / n_tn;
            tn = t % n_tn;
        } else {
            const int x = t & 7, l = t >> 3;
            const int g = l / (gh * n_tn), q = l % (gh * n_tn);
            tm = x * (n_tm >> 3) + g * gh + q % gh;
            tn = q / gh;
        }
    };
    // this lane's two 16-byte chunks of each operand tile: LDS chunk
    // p = wave * 128 + q * 64 + lane holds row p / 4, logical chunk (p % 4) ^ swz(row)
    int voff[2];
    for (int q = 0; q < 2; ++q) {
        const int p = wave * 128 + q * 64 + lane;
        const int r = p >> 2, c = (p & 3) ^ g2_swz(p >> 2);
        voff[q] = (int)((r * kp + c * 8) * 2);
    }
    const int tile_bytes = (int)(G2M * kp * 2);   // 256 rows of either operand
    __amdgpu_buffer_rsrc_t rAh, rAl, rB;
    auto set_tile = [&](int t) {
        int tm, tn;
        tile_of(t, tm, tn);
        rAh = __builtin_amdgcn_make_buffer_rsrc((void*)(Ahi + (int64_t)tm * G2M * kp), (short)0, tile_bytes, 0x00020000);
        rAl = __builtin_amdgcn_make_buffer_rsrc((void*)(Alo + (int64_t)tm * G2M * kp), (short)0, tile_bytes, 0x00020000);
        rB = __builtin_amdgcn_make_buffer_rsrc((void*)(Bhi + (int64_t)tn * G2N * kp), (short)0, tile_bytes, 0x00020000);
    };
    auto issue = [&](uint16_t* base, int64_t kt) {
        const int ko = (int)(kt * G2K * 2);
        for (int q = 0; q < 2; ++q) {
            const int lo = (wave * 128 + q * 64) * 8;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rAh, (lds_void*)(base + lo), 16, voff[q], ko, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rAl, (lds_void*)(base + G2OP + lo), 16, voff[q], ko, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rB, (lds_void*)(base + 2 * G2OP + lo), 16, voff[q], ko, 0, 0);
        }
    };
    f32x16 acc[2][4];
    uint4 xh[2], xl[2], xb[4], yh[2], yl[2], yb[4];
    // fragments of k half ks (0 or 16) of the tile in `base`
    auto frag = [&](const uint16_t* base, int ks, uint4* h, uint4* l, uint4* bb) {
        const int c = (ks >> 3) + (lane >> 5);
        for (int i = 0; i < 2; ++i) {
            const int r = wm + i * 32 + (lane & 31);
            const int o = r * G2R + ((c ^ g2_swz(r)) * 8);
            h[i] = *(const uint4*)&base[o];
            l[i] = *(const uint4*)&base[G2OP + o];
        }
        for (int j = 0; j < 4; ++j) {
            const int r = wn + j * 32 + (lane & 31);
            bb[j] = *(const uint4*)&base[2 * G2OP + r * G2R + ((c ^ g2_swz(r)) * 8)];
        }
    };
    auto mma = [&](const uint4* h, const uint4* l, const uint4* bb) {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma16<F16>((const uint16_t*)&h[i], (const uint16_t*)&bb[j], acc[i][j]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma16<F16>((const uint16_t*)&l[i], (const uint16_t*)&bb[j], acc[i][j]);
    };
    // Tile kt from stage `cur`; the next tile's first half from stage `nxt`.
    // Every body issues exactly one tile's loads (past the last tile: the last
    // tile again, never read), so the same wait, one later tile in flight,
    // holds everywhere and the compiler's own waits stay exact.
    // The scheduling fences keep each phase whole: one half's reads are all in
    // flight while the other half's products issue.
    auto body = [&](uint16_t* cur, const uint16_t* nxt, int64_t kt) {
        frag(cur, 16, yh, yl, yb);
        __builtin_amdgcn_sched_barrier(0);
        mma(xh, xl, xb);
        __builtin_amdgcn_sched_barrier(0);
        G2_SYNC(G2_STAGE_WAIT_1);                      // tile kt + 1 landed in every wave
        issue(cur, kt + 3 < nk ? kt + 3 : nk - 1);     // every wave has read tile kt
        frag(nxt, 0, xh, xl, xb);
        __builtin_amdgcn_sched_barrier(0);
        mma(yh, yl, yb);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto issue3 = [&]() {
        issue(st0, 0);
        issue(st1, nk > 1 ? 1 : nk - 1);
        issue(st2, nk > 2 ? 2 : nk - 1);
    };

    int t = blockIdx.x;
    if (t >= T) return;
    set_tile(t);
    issue3();
    for (; t < T; t += gridDim.x) {
        int tm, tn;
        tile_of(t, tm, tn);
        const int64_t row0 = (int64_t)tm * G2M, col0 = (int64_t)tn * G2N;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 4; ++j)
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
        G2_SYNC(G2_STAGE_WAIT_2);   // tile 0 landed
        frag(st0, 0, xh, xl, xb);
        int64_t kt = 0;
        for (; kt + 3 <= nk; kt += 3) {
            body(st0, st1, kt);
            body(st1, st2, kt + 1);
            body(st2, st0, kt + 2);
        }
        if (kt < nk) body(st0, st1, kt);
        if (kt + 1 < nk) body(st1, st2, kt + 1);
        // epilogue: lane holds column (lane & 31); values e: row 8 (e / 4) + 4 (lane / 32) + (e % 4),
        // receiver = row / 2.  E_env and the row scales are loaded ahead of the wait that ends
        // the tile's products, so that wait covers them and the stores wait for nothing
        // (loaded after the next tile's stages, the compiler's waits for them would also
        // hold back those stages, and its waits for the stage reads after the loop would
        // no longer be exact)
        float2 ev[2][4][2];
        int32_t sx[2][4][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int eb = 0; eb < 4; ++eb)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    int64_t r = (row0 + wm + i * 32 + 8 * eb + 4 * (lane >> 5) + 2 * h) >> 1;
                    r = r < R ? r : R - 1;
                    ev[i][eb][h] = Eenv[r];
                    sx[i][eb][h] = F16 ? sexp[r] : 0;
                }
        G2_SYNC(G2_STAGE_WAIT_0);   // the repeated loads and E_env landed, every LDS read is done
        asm volatile("" ::: "memory");
        const int t2 = t + (int)gridDim.x;
        if (t2 < T) {
            set_tile(t2);
            issue3();
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t c = col0 + wn + j * 32 + (lane & 31);
#pragma unroll
                for (int e = 0; e < 16; e += 2) {
                    const int64_t r = (row0 + wm + i * 32 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4)) >> 1;
                    if (r >= R || c >= C) continue;
                    const float2 e0 = ev[i][e / 4][(e % 4) / 2];
                    const float sr = F16 ? ldexpf(scale, -sx[i][e / 4][(e % 4) / 2]) : scale;   // exact: a power of two
                    const float er = e0.x + sr * acc[i][j][e];
                    const float ei = e0.y + sr * acc[i][j][e + 1];
                    // streaming stores: the outputs are not read again here, and they drain
                    // faster at the end of a tile without taking room in the L2s
                    if (Eout) __builtin_nontemporal_store(f32x2{er, ei}, (f32x2*)&Eout[r * C + c]);
                    if (Pout) __builtin_nontemporal_store((er * er + ei * ei) / (2.0f * ETA0_F), &Pout[r * C + c]);
                }
            }
    }
}
#undef G2_SYNC

// XCD-aware group height of the two-product kernel: tile rows per group, 0 for row-major order
static int g2_group_rows(int n_tm)
{
    if (n_tm % 8) return 0;
    const int band = n_tm / 8;
    for (int g : {8, 4, 2, 1})
        if (band % g == 0) return g;
    return 0;
}

static int cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

// Shapes of the matrix-core product of one sum (the split buffers' sizes).
struct SumShape {
    bool f16, three;
    int layout;      // cached split key: 1 / 2 bf16 real / complex Gamma, 3 / 4 fp16
    int lay;         // 1 real, 2 complex Gamma
    int64_t kp, rows_p, cols_p;
};

static SumShape sum_shape(int64_t R, int64_t M, int64_t C, bool gamma_real, int precision)
{
    SumShape sh;
    sh.f16 = precision == 3;
    sh.three = precision == 2;
    sh.lay = gamma_real ? 1 : 2;
    sh.layout = sh.lay + (sh.f16 ? 2 : 0);
    const int64_t kd = gamma_real ? M : 2 * M;
    sh.kp = round_up(kd > 0 ? kd : 1, GBK);
    sh.rows_p = round_up(2 * R, G2M);   // a multiple of both tile heights
    sh.cols_p = round_up(C, G2N);
    return sh;
}

// Split of H into a_hi / a_lo (and the fp16 row scales), on `st`.
static void launch_split_a(const Channel& ch, const SumShape& sh, uint16_t* a_hi, uint16_t* a_lo, int32_t* sexp,
                           hipStream_t st)
{
    const int64_t R = ch.R, M = ch.M;
    if (sh.f16) {
        hipLaunchKernelGGL(k_row_scale, dim3(nblk(R, 4)), dim3(256), 0, st, ch.H.as<float2>(), R, M, sexp);
        HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_split_A, dim3(nblk(sh.rows_p * sh.kp, 256)), dim3(256), 0, st, ch.H.as<float2>(), R, M,
                       sh.lay, sh.rows_p, sh.kp, sh.f16 ? (const int32_t*)sexp : (const int32_t*)nullptr, a_hi, a_lo);
    HIP_CHECK(hipGetLastError());
}

// Split of Gamma into b_hi (b_lo for three products) and the product itself, on `st`.
static void launch_product(const Channel& ch, const SumShape& sh, const float2* G, int64_t C, float scale,
                           const uint16_t* a_hi, const uint16_t* a_lo, const int32_t* sexp, uint16_t* b_hi,
                           uint16_t* b_lo, float* E_out, float* P_out, hipStream_t st)
{
    const int64_t R = ch.R, M = ch.M, kp = sh.kp;
    hipLaunchKernelGGL(k_split_B, dim3(nblk(sh.cols_p, SBT), nblk(kp, SBT)), dim3(256), 0, st, G, M, C, sh.lay, sh.cols_p, kp,
                       sh.f16, b_hi, sh.three ? b_lo : (uint16_t*)nullptr);
    HIP_CHECK(hipGetLastError());
    const int32_t* sx = sh.f16 ? sexp : nullptr;
    if (sh.three) {
        const int n_tn = (int)(sh.cols_p / GBN);
        const int64_t n_tiles = (sh.rows_p / GBM) * n_tn;
        hipLaunchKernelGGL((k_sum_mfma<3, false>), dim3((unsigned)n_tiles), dim3(256), 0, st, a_hi, a_lo, b_hi, b_lo,
                           kp, ch.E_env.as<float2>(), sx, R, C, scale, (float2*)E_out, P_out, n_tn);
    } else {
        const int n_tm = (int)(sh.rows_p / G2M), n_tn = (int)(sh.cols_p / G2N);
        const int64_t n_tiles = (int64_t)n_tm * n_tn;
        if (n_tiles >= ((int64_t)1 << 31) || (int64_t)G2M * kp * 2 >= ((int64_t)1 << 31))
            throw inval_error("sum too large for the matrix-core tiles");
        const int gh = g2_group_rows(n_tm);
        const unsigned grid = (unsigned)std::min<int64_t>(n_tiles, cu_count());   // one workgroup per CU
        if (sh.f16)
            hipLaunchKernelGGL((k_sum_mfma_2x<true>), dim3(grid), dim3(512), 0, st, a_hi, a_lo, b_hi, kp,
                               ch.E_env.as<float2>(), sx, R, C, scale, (float2*)E_out, P_out, n_tm, n_tn, gh);
        else
            hipLaunchKernelGGL((k_sum_mfma_2x<false>), dim3(grid), dim3(512), 0, st, a_hi, a_lo, b_hi, kp,
                               ch.E_env.as<float2>(), sx, R, C, scale, (float2*)E_out, P_out, n_tm, n_tn, gh);
    }
    HIP_CHECK(hipGetLastError());
}

static void launch_valu(const Channel& ch, const float2* G, int64_t C, float scale, float* E_out, float* P_out,
                        hipStream_t st)
{
    static_assert(VT * VN == 256, "one output per thread in the narrow kernel");
    if (C <= VN) {
        hipLaunchKernelGGL(k_sum_valu_narrow, dim3(nblk(ch.R, VT)), dim3(256), 0, st, ch.H.as<float2>(), G,
                           ch.E_env.as<float2>(), ch.R, ch.M, C, scale, (float2*)E_out, P_out);
    } else {
        dim3 grid(nblk(C, VT), nblk(ch.R, VT));
        hipLaunchKernelGGL(k_sum_valu, grid, dim3(256), 0, st, ch.H.as<float2>(), G, ch.E_env.as<float2>(), ch.R,
                           ch.M, C, scale, (float2*)E_out, P_out);
    }
    HIP_CHECK(hipGetLastError());
}

void ris_sum(Ctx& c, Channel& ch, const float* gamma, int64_t C, float scale, bool gamma_real, int precision,
             float* E_out, float* P_out, hipStream_t st)
{
    const int64_t R = ch.R, M = ch.M;
    const float2* G = (const float2*)gamma;
    if (R == 0 || C == 0) return;
    if (precision == 0) {
        launch_valu(ch, G, C, scale, E_out, P_out, st);
        return;
    }
    const SumShape sh = sum_shape(R, M, C, gamma_real, precision);
    if (ch.split_kind == sh.layout && ch.split_ev) HIP_CHECK(hipStreamWaitEvent(st, ch.split_ev, 0));
    if (ch.split_kind != sh.layout) {
        // the old split may still be read by sums queued on other streams: this
        // stream waits for all of them, then releases it in its own order
        for (const auto& rd : ch.split_readers)
            if (rd.first != st) HIP_CHECK(hipStreamWaitEvent(st, rd.second, 0));
        for (Scratch* p : {&ch.a_hi, &ch.a_lo, &ch.a_sexp}) p->st = st;
        ch.a_hi.release();
        ch.a_lo.release();
        ch.a_sexp.release();
        ch.a_hi = Scratch(c, sizeof(uint16_t) * (size_t)(sh.rows_p * sh.kp), st);
        ch.a_lo = Scratch(c, sizeof(uint16_t) * (size_t)(sh.rows_p * sh.kp), st);
        if (sh.f16) ch.a_sexp = Scratch(c, sizeof(int32_t) * (size_t)R, st);
        launch_split_a(ch, sh, ch.a_hi.as<uint16_t>(), ch.a_lo.as<uint16_t>(), ch.a_sexp.as<int32_t>(), st);
        ch.split_kind = sh.layout;
        ch.a_rows = sh.rows_p;
        ch.a_k = sh.kp;
        if (!ch.split_ev) HIP_CHECK(hipEventCreateWithFlags(&ch.split_ev, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(ch.split_ev, st));
    }
    Scratch bhi(c, sizeof(uint16_t) * (size_t)(sh.cols_p * sh.kp), st);
    Scratch blo;
    if (sh.three) blo = Scratch(c, sizeof(uint16_t) * (size_t)(sh.cols_p * sh.kp), st);
    launch_product(ch, sh, G, C, scale, ch.a_hi.as<uint16_t>(), ch.a_lo.as<uint16_t>(), ch.a_sexp.as<int32_t>(),
                   bhi.as<uint16_t>(), blo.as<uint16_t>(), E_out, P_out, st);
    // this stream has read the split up to here
    hipEvent_t* ev = nullptr;
    for (auto& rd : ch.split_readers)
        if (rd.first == st) ev = &rd.second;
    if (!ev) {
        ch.split_readers.emplace_back(st, nullptr);
        ev = &ch.split_readers.back().second;
        HIP_CHECK(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    }
    HIP_CHECK(hipEventRecord(*ev, st));
}

// The caller-provided scratch: [a_hi | a_lo | b_hi | b_lo | sexp], each part
// starting on a 256-byte boundary.
static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t ris_sum_scratch_bytes(int64_t R, int64_t M, int64_t C, bool gamma_real, int precision)
{
    if (precision == 0 || R == 0 || C == 0) return 0;
    const SumShape sh = sum_shape(R, M, C, gamma_real, precision);
    const size_t a = align256(sizeof(uint16_t) * (size_t)(sh.rows_p * sh.kp));
    const size_t b = align256(sizeof(uint16_t) * (size_t)(sh.cols_p * sh.kp));
    return 2 * a + (sh.three ? 2 : 1) * b + (sh.f16 ? align256(sizeof(int32_t) * (size_t)R) : 0);
}

void ris_sum_in(const Channel& ch, const float* gamma, int64_t C, float scale, bool gamma_real, int precision,
                float* E_out, float* P_out, void* scratch, hipStream_t st)
{
    const int64_t R = ch.R, M = ch.M;
    const float2* G = (const float2*)gamma;
    if (R == 0 || C == 0) return;
    if (precision == 0) {
        launch_valu(ch, G, C, scale, E_out, P_out, st);
        return;
    }
    const SumShape sh = sum_shape(R, M, C, gamma_real, precision);
    const size_t a = align256(sizeof(uint16_t) * (size_t)(sh.rows_p * sh.kp));
    const size_t b = align256(sizeof(uint16_t) * (size_t)(sh.cols_p * sh.kp));
    char* base = (char*)scratch;
    uint16_t* a_hi = (uint16_t*)base;
    uint16_t* a_lo = (uint16_t*)(base + a);
    uint16_t* b_hi = (uint16_t*)(base + 2 * a);
    uint16_t* b_lo = sh.three ? (uint16_t*)(base + 2 * a + b) : nullptr;
    int32_t* sexp = sh.f16 ? (int32_t*)(base + 2 * a + (sh.three ? 2 : 1) * b) : nullptr;
    // every element of the split buffers (padding included) is written before it is read
    launch_split_a(ch, sh, a_hi, a_lo, sexp, st);
    launch_product(ch, sh, G, C, scale, a_hi, a_lo, sexp, b_hi, b_lo, E_out, P_out, st);
}

}  // namespace rt
