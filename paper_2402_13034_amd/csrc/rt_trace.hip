// Tracing: discovery rays, candidate surface sequences, image-method paths,
// visibility legs, the per-element RIS expansion and the field.
//
// Stages (all on one stream; sizes are read back where buffers depend on them):
//  1. discovery  spherical-Fibonacci rays from the Tx (full sphere) and from
//                the RIS centre u (half-space in front of the RIS); closest
//                hit + specular bounce up to K times (stand-in for the
//                analytic first stage of the hybrid tracer, Section II).
//  2. dedupe     every prefix of every hit list, mapped to surfaces, packed
//                into a 64-bit key (21 bits per surface); sort + unique.
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

#include <cstring>
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

template <bool BRUTE, int STK>
__global__ __launch_bounds__(DISC_B) void k_discover(SceneView s, double sx, double sy, double sz, int hemi,
                                                     double hx, double hy, double hz, int64_t rows, int K,
                                                     int32_t* hits, unsigned long long* segs)
{
    __shared__ int stack[STK * DISC_B];
    int64_t i = (int64_t)blockIdx.x * DISC_B + threadIdx.x;
    unsigned nseg = 0;
    if (i < rows) {
        double d64[3];
        fib_dir(i, rows, d64);
        for (int b = 0; b < K; ++b) hits[i * K + b] = -1;
        bool go = true;
        if (hemi) go = (d64[0] * hx + d64[1] * hy + d64[2] * hz) > 0.0;
        if (go) {
            float ox = (float)sx, oy = (float)sy, oz = (float)sz;
            float dx = (float)d64[0], dy = (float)d64[1], dz = (float)d64[2];
            int skip = -1;
            for (int b = 0; b < K; ++b) {
                float t;
                int id;
                ++nseg;
                int slot = closest_hit<BRUTE>(s, ox, oy, oz, dx, dy, dz, (float)RT_EPS, skip,
                                              stack + threadIdx.x, DISC_B, t, id);
                if (slot < 0) break;
                hits[i * K + b] = id;
                float px = ox + t * dx, py = oy + t * dy, pz = oz + t * dz;
                reflect32(s.tri4[3 * slot + 1], s.tri4[3 * slot + 2], dx, dy, dz);
                ox = px;
                oy = py;
                oz = pz;
                skip = id;
            }
        }
    }
    wave_count_add(segs, nseg);
}

// --------------------------------------------------------------------------
// 2. keys of every prefix (surface ids + 1, 21 bits each); 0 = none
// --------------------------------------------------------------------------
__global__ void k_prefix_keys(const int32_t* hits, const int32_t* surf, int64_t rows, int K, uint64_t* keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    uint64_t acc = 0;
    bool alive = true;
    for (int b = 0; b < K; ++b) {
        int32_t h = hits[i * K + b];
        alive = alive && h >= 0;
        if (alive) acc |= (uint64_t)(surf[h] + 1) << (RT_KEY_BITS * b);
        keys[i * K + b] = alive ? acc : 0ull;
    }
}

// every sequence of <= K surfaces without immediate repeat, as keys (0 for skipped)
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
    uint64_t key = 0;
    int prev = -1;
    bool ok = true;
    for (int j = 0; j < k; ++j) {
        int sidx = (int)(r % n_surf);
        r /= n_surf;
        if (sidx == prev) ok = false;
        prev = sidx;
        key |= (uint64_t)(sidx + 1) << (RT_KEY_BITS * j);
    }
    keys[idx] = ok ? key : 0ull;
}

// --------------------------------------------------------------------------
// 3. candidates: decode keys, images of the source
// --------------------------------------------------------------------------
__global__ void k_cand_prep(const uint64_t* keys, int64_t n, SceneView s, double sx, double sy, double sz,
                            int32_t* ck, int32_t* cseq, double* cimg)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    uint64_t key = keys[c];
    int k = 0;
    int seq[RT_MAX_K];
    for (int j = 0; j < RT_MAX_K; ++j) {
        uint64_t v = (key >> (RT_KEY_BITS * j)) & ((1ull << RT_KEY_BITS) - 1);
        seq[j] = v ? (int)v - 1 : -1;
        if (v && k == j) k = j + 1;
    }
    ck[c] = k;
    double I[3] = {sx, sy, sz};
    for (int j = 0; j < RT_MAX_K; ++j) {
        cseq[3 * c + j] = seq[j];
        if (j < k) {
            double o[3];
            mirror(s.s_plane + 4 * seq[j], I, o);
            I[0] = o[0];
            I[1] = o[1];
            I[2] = o[2];
        }
        cimg[9 * c + 3 * j + 0] = I[0];
        cimg[9 * c + 3 * j + 1] = I[1];
        cimg[9 * c + 3 * j + 2] = I[2];
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

__device__ __forceinline__ bool geo_path(const SceneView& s, const CandView& cv, int64_t c, const double* S,
                                         const double* X, double (*P)[3], int* tri, int& k)
{
    k = cv.k[c];
    int seq[RT_MAX_K];
    double I[RT_MAX_K + 1][3];
    I[0][0] = S[0];
    I[0][1] = S[1];
    I[0][2] = S[2];
    for (int j = 0; j < RT_MAX_K; ++j) {
        seq[j] = cv.seq[3 * c + j];
        for (int q = 0; q < 3; ++q) I[j + 1][q] = cv.img[9 * c + 3 * j + q];
    }
    return image_backtrace(s, seq, k, I, X, P, tri);
}

// Append `value` of every lane with ok to out[0..cap) (one atomic per wave);
// the counter keeps counting past cap so the host can detect the overflow.
__device__ __forceinline__ void wave_append(bool ok, uint64_t value, uint64_t* out, int64_t cap,
                                            unsigned long long* counter)
{
    const int lane = threadIdx.x & 63;
    unsigned long long mask = __ballot(ok);
    if (mask == 0ull) return;
    const int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    const unsigned long long idx = base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
    if (ok && idx < (unsigned long long)cap) out[idx] = value;
}

__global__ __launch_bounds__(256) void k_geo_cells(SceneView s, CandView cv, double sx, double sy, double sz,
                                                   const double* rx, int64_t R, uint64_t* cells, int64_t cap,
                                                   unsigned long long* counter)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = false;
    if (i < R * cv.n) {
        int64_t r = i / cv.n, c = i - r * cv.n;
        double S[3] = {sx, sy, sz};
        double X[3] = {rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]};
        double P[RT_MAX_K][3];
        int tri[RT_MAX_K];
        int k;
        ok = geo_path(s, cv, c, S, X, P, tri, k);
    }
    wave_append(ok, (uint64_t)i, cells, cap, counter);
}

// --------------------------------------------------------------------------
// 5/6. legs and field of each geometric path, in (receiver, candidate) order
// --------------------------------------------------------------------------
constexpr int LEG_B = 128;

struct PathRec {
    int32_t rx, cand, k;
    int32_t tri[RT_MAX_K];
};

__device__ __forceinline__ double seg_len(const double* a, const double* b)
{
    double w0 = b[0] - a[0], w1 = b[1] - a[1], w2 = b[2] - a[2];
    return sqrt(w0 * w0 + w1 * w1 + w2 * w2);
}

template <bool BRUTE, bool FIELD, int STK>
__global__ __launch_bounds__(LEG_B) void k_paths(SceneView s, CandView cv, TraceConst tc, double sx, double sy,
                                                 double sz, const double* rx, const uint64_t* cells, int64_t n,
                                                 uint8_t* valid, float2* amp, double* len, PathRec* recs,
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
        double P[RT_MAX_K][3];
        int tri[RT_MAX_K] = {-1, -1, -1};
        int k;
        bool ok = geo_path(s, cv, c, S, X, P, tri, k);
        float Ft = 1.0f, Fr = 1.0f;
        if (FIELD && ok) {
            double v1[3], vl[3];
            const double* f = k ? P[0] : X;
            const double* l = k ? P[k - 1] : S;
            for (int q = 0; q < 3; ++q) {
                v1[q] = f[q] - S[q];
                vl[q] = l[q] - X[q];
            }
            Ft = pattern_f(tc.txa.pattern, (float)tc.txa.param, cos_between(v1, tc.txa.axis));
            Fr = pattern_f(tc.rxa.pattern, (float)tc.rxa.param, cos_between(vl, tc.rxa.axis));
            ok = Ft > 0.0f && Fr > 0.0f;
        }
        for (int j = 0; j <= k && ok; ++j) {
            const double* A = j == 0 ? S : P[j - 1];
            const double* B = j == k ? X : P[j];
            int sa = j == 0 ? -1 : cv.seq[3 * c + j - 1];
            int sb = j == k ? -1 : cv.seq[3 * c + j];
            ++nseg;
            if (leg_blocked<BRUTE>(s, A, B, sa, sb, stack + threadIdx.x, LEG_B)) ok = false;
        }
        valid[i] = ok ? 1 : 0;
        PathRec pr;
        pr.rx = (int32_t)r;
        pr.cand = (int32_t)c;
        pr.k = k;
        for (int j = 0; j < RT_MAX_K; ++j) pr.tri[j] = j < k ? tri[j] : -1;
        recs[i] = pr;
        if (FIELD) {
            double D = 0.0;
            for (int j = 0; j <= k; ++j) D += seg_len(j == 0 ? S : P[j - 1], j == k ? X : P[j]);
            float2 a = make_float2(0.0f, 0.0f);
            if (ok) {
                float ar = 1.0f, ai = 0.0f;
                for (int j = 0; j < k; ++j) {
                    float2 Rc = s.refl[tri[j]];
                    float nr = ar * Rc.x - ai * Rc.y;
                    float ni = ar * Rc.y + ai * Rc.x;
                    ar = nr;
                    ai = ni;
                }
                float mag = sqrtf((float)tc.two_eta0_pt_gt * Ft) * sqrtf((float)tc.rxa.gain * Fr) *
                            (float)(tc.lambda / (4.0 * 3.141592653589793 * D));
                float ph = (float)phase_of(D, tc.lambda);
                float cs, sn;
                sincosf(ph, &sn, &cs);
                a = make_float2(mag * (ar * cs - ai * sn), mag * (ar * sn + ai * cs));
            }
            amp[i] = a;
            len[i] = D;
        }
    }
    wave_count_add(segs, nseg);
}

// first record of each receiver (records sorted by cell = r * nc + c)
__global__ void k_rx_start(const uint64_t* cells, int64_t n, int64_t nc, int64_t R, int64_t* rstart)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > R) return;
    const uint64_t key = (uint64_t)r * (uint64_t)nc;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (cells[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    rstart[r] = lo;
}

// E_env[r] = sum of emitted paths of receiver r, in record order (FP64)
__global__ void k_env_reduce(const int64_t* rstart, int64_t R, const uint8_t* valid, const float2* amp, float2* E)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double er = 0.0, ei = 0.0;
    for (int64_t j = rstart[r]; j < rstart[r + 1]; ++j)
        if (valid[j]) {
            er += (double)amp[j].x;
            ei += (double)amp[j].y;
        }
    E[r] = make_float2((float)er, (float)ei);
}

// keep valid records: env path records for read-back
__global__ void k_env_compact(const PathRec* recs, CandView cv, const uint8_t* valid, const int64_t* off2,
                              const float2* amp, const double* len, int64_t n, EnvRec* out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !valid[i]) return;
    const PathRec& pr = recs[i];
    EnvRec e;
    e.rx = pr.rx;
    e.order = pr.k;
    for (int j = 0; j < 3; ++j) {
        e.seq[j] = cv.seq[3 * pr.cand + j];
        e.tri[j] = pr.tri[j];
    }
    e.length = len[i];
    e.amp[0] = amp[i].x;
    e.amp[1] = amp[i].y;
    out[off2[i]] = e;
}

// valid centre sequences of order >= 1
__global__ void k_u_flags(const PathRec* recs, const uint8_t* valid, int64_t n, uint8_t* f2)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    f2[i] = (valid[i] && recs[i].k >= 1) ? 1 : 0;
}

// rows of 8 ints: rx, surfaces s0..s2, triangles t0..t2 reached from the centre, 0
__global__ void k_u_compact(const PathRec* recs, CandView cv, const uint8_t* f2, const int64_t* off2, int64_t n,
                            int32_t* useq)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !f2[i]) return;
    int64_t o = off2[i];
    useq[8 * o + 0] = recs[i].rx;
    for (int j = 0; j < 3; ++j) {
        useq[8 * o + 1 + j] = cv.seq[3 * recs[i].cand + j];
        useq[8 * o + 4 + j] = recs[i].tri[j];
    }
    useq[8 * o + 7] = 0;
}

__global__ void k_uptr(const int64_t* rstart, int64_t n_rec, const int64_t* off2, int64_t total2, int64_t R,
                       int64_t* uptr)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > R) return;
    int64_t a = rstart[r];
    uptr[r] = (r < R && a < n_rec) ? off2[a] : total2;
}

// --------------------------------------------------------------------------
// 7. RIS
// --------------------------------------------------------------------------
struct TxmRec {
    float fac;     // A_t(Tx->m) sqrt(G F_in d_y d_z / 4pi) / d_t
    int ok;        // leg clear and F_t, F_in > 0
    double dt;
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
        float Ft = pattern_f(tc.txa.pattern, (float)tc.txa.param, cos_between(vt, tc.txa.axis));
        float Fin = pattern_f(1, (float)rv.q, cos_between(back, rv.normal));
        bool ok = Ft > 0.0f && Fin > 0.0f;
        if (ok) {
            ++nseg;
            ok = !leg_blocked<BRUTE>(s, tc.tx, e, -1, -1, stack + threadIdx.x, 64);
        }
        TxmRec r;
        r.ok = ok ? 1 : 0;
        r.dt = dt;
        r.fac = ok ? (float)(sqrt(tc.two_eta0_pt_gt * (double)Ft) *
                             sqrt(rv.gain * (double)Fin * rv.dy * rv.dz / (4.0 * 3.141592653589793)) / dt)
                   : 0.0f;
        out[m] = r;
    }
    wave_count_add(segs, nseg);
}

constexpr int RIS_B = 128;

// Back-trace like image_backtrace, but each reflection first tries the
// triangle the RIS-centre path used (hint); a point on a surface lies in
// exactly one of its triangles, so the result is the same as a full search.
template <bool CNT>
__device__ inline bool image_backtrace_hint(const SceneView& s, const int* seq, const int* hint, int k,
                                            const double (*I)[3], const double* X, double (*P)[3], int* tri,
                                            WorkCount* wc)
{
#pragma clang fp contract(off)
    double Q[3] = {X[0], X[1], X[2]};
    for (int i = k; i >= 1; --i) {
        const double* pl = s.s_plane + 4 * seq[i - 1];
        double w0 = Q[0] - I[i][0], w1 = Q[1] - I[i][1], w2 = Q[2] - I[i][2];
        double den = pl[0] * w0 + pl[1] * w1 + pl[2] * w2;
        if (den == 0.0) return false;
        double sp = (pl[3] - (pl[0] * I[i][0] + pl[1] * I[i][1] + pl[2] * I[i][2])) / den;
        if (!(sp > 0.0 && sp < 1.0)) return false;
        double p[3] = {I[i][0] + sp * w0, I[i][1] + sp * w1, I[i][2] + sp * w2};
        int h = hint[i - 1];
        if (CNT && h >= 0) wc->contain++;
        int t = (h >= 0 && contains64(s.v64 + 9 * h, p)) ? h : surface_contains<CNT>(s, seq[i - 1], p, wc);
        if (t < 0) return false;
        tri[i - 1] = t;
        P[i - 1][0] = p[0]; P[i - 1][1] = p[1]; P[i - 1][2] = p[2];
        Q[0] = p[0]; Q[1] = p[1]; Q[2] = p[2];
    }
    for (int i = 0; i < k; ++i) {
        const double* pl = s.s_plane + 4 * seq[i];
        const double* prev = (i == 0) ? I[0] : P[i - 1];
        const double* next = (i == k - 1) ? X : P[i + 1];
        double a = plane_side(pl, prev);
        double b = plane_side(pl, next);
        if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return false;
    }
    return true;
}

// CNT: counting build; work[0..4] += node visits, triangle tests,
// containment tests, (slot, element) pairs, legs.
template <bool BRUTE, bool KEEP, int STK, bool CNT>
__global__ __launch_bounds__(RIS_B) void k_ris(SceneView s, TraceConst tc, RisView rv, const TxmRec* txm,
                                               const double* rx, int64_t R, const int64_t* uptr,
                                               const int32_t* useq, int n_mchunk, float2* H, uint8_t* rvalid,
                                               unsigned long long* segs, unsigned long long* work)
{
    __shared__ int stack[STK * RIS_B];
    WorkCount wc;
    unsigned pairs = 0;
    int64_t w = ((int64_t)blockIdx.x * RIS_B + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    unsigned nseg = 0;
    if (w < R * n_mchunk) {
        int64_t r = w / n_mchunk;
        int m = (int)(w - r * n_mchunk) * 64 + lane;
        bool active = m < rv.M;
        int mm = active ? m : 0;
        const double* e = rv.elem + 3 * mm;
        double E[3] = {e[0], e[1], e[2]};
        TxmRec t = txm[mm];
        double X[3] = {rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]};
        int64_t u0 = uptr[r], u1 = uptr[r + 1];
        int64_t nsl = 1 + (u1 - u0);
        double acc_r = 0.0, acc_i = 0.0;
        for (int64_t sl = 0; sl < nsl; ++sl) {
            int seq[RT_MAX_K] = {-1, -1, -1};
            int hint[RT_MAX_K] = {-1, -1, -1};
            int k = 0;
            if (sl > 0) {
                const int32_t* row = useq + 8 * (u0 + sl - 1);
                for (int j = 0; j < RT_MAX_K; ++j) {
                    seq[j] = row[1 + j];
                    hint[j] = row[4 + j];
                    if (seq[j] >= 0) k = j + 1;
                }
            }
            bool ok = active && t.ok;
            double I[RT_MAX_K + 1][3];
            double P[RT_MAX_K][3];
            int tri[RT_MAX_K];
            I[0][0] = E[0];
            I[0][1] = E[1];
            I[0][2] = E[2];
            for (int j = 0; j < k; ++j) mirror(s.s_plane + 4 * seq[j], I[j], I[j + 1]);
            if (CNT && active) ++pairs;
            if (ok) ok = image_backtrace_hint<CNT>(s, seq, hint, k, I, X, P, tri, &wc);
            float Fout = 0.0f, Fr = 0.0f;
            if (ok) {
                const double* f = k ? P[0] : X;
                const double* l = k ? P[k - 1] : E;
                double v1[3] = {f[0] - E[0], f[1] - E[1], f[2] - E[2]};
                double vl[3] = {l[0] - X[0], l[1] - X[1], l[2] - X[2]};
                Fout = pattern_f(1, (float)rv.q, cos_between(v1, rv.normal));
                Fr = pattern_f(tc.rxa.pattern, (float)tc.rxa.param, cos_between(vl, tc.rxa.axis));
                ok = Fout > 0.0f && Fr > 0.0f;
            }
            for (int j = 0; j <= k; ++j) {
                if (!ok) break;
                const double* A = j == 0 ? E : P[j - 1];
                const double* B = j == k ? X : P[j];
                int sa = j == 0 ? -1 : seq[j - 1];
                int sb = j == k ? -1 : seq[j];
                ++nseg;
                if (leg_blocked<BRUTE, CNT>(s, A, B, sa, sb, stack + threadIdx.x, RIS_B, &wc)) ok = false;
            }
            if (ok) {
                double Dr = 0.0;
                for (int j = 0; j <= k; ++j) Dr += seg_len(j == 0 ? E : P[j - 1], j == k ? X : P[j]);
                float ar = 1.0f, ai = 0.0f;
                for (int j = 0; j < k; ++j) {
                    float2 Rc = s.refl[tri[j]];
                    float nr = ar * Rc.x - ai * Rc.y;
                    float ni = ar * Rc.y + ai * Rc.x;
                    ar = nr;
                    ai = ni;
                }
                float mag = t.fac * sqrtf(Fout) * sqrtf((float)tc.rxa.gain * Fr) *
                            (float)(tc.lambda / (4.0 * 3.141592653589793 * Dr));
                float ph = (float)phase_of(t.dt + Dr, tc.lambda);
                float cs, sn;
                sincosf(ph, &sn, &cs);
                acc_r += (double)(mag * (ar * cs - ai * sn));
                acc_i += (double)(mag * (ar * sn + ai * cs));
            }
            if (KEEP && active) rvalid[(u0 + r + sl) * rv.M + m] = ok ? 1 : 0;
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

static void make_candidates(Ctx& c, const SceneView& sv, int stk, const double* src, const double* hemi_n,
                            const TraceArgs& a, bool brute, bool exhaustive, bool keep_hits, Channel& ch,
                            int which, Cands& out, unsigned long long* d_segs, int64_t* d_cnt, hipStream_t st)
{
    const int K = a.tc.K;
    Scratch keys;
    int64_t nkeys = 0;
    if (exhaustive) {
        int64_t ns = sv.n_surf;
        int64_t total = 0, p = 1;
        for (int k = 1; k <= K; ++k) {
            p *= ns;
            total += p;
            if (total > (int64_t)1 << 26) throw inval_error("exhaustive candidate set too large");
        }
        nkeys = total + 1;
        keys = Scratch(c, sizeof(uint64_t) * (size_t)nkeys, st);
        HIP_CHECK(hipMemsetAsync(keys.p, 0, keys.bytes, st));
        if (total > 0)
            hipLaunchKernelGGL(k_exhaustive_keys, dim3(nblk(total, 256)), dim3(256), 0, st, ns, K, total,
                               keys.as<uint64_t>());
        HIP_CHECK(hipGetLastError());
    } else {
        int64_t rows = hemi_n ? 2 * a.n_rays : a.n_rays;
        Scratch hits(c, sizeof(int32_t) * (size_t)(rows * K), st);
        if (rows > 0) {
            SEL_BOOL(brute, BR,
                     SEL_STK(stk, hipLaunchKernelGGL((k_discover<BR, STK>), dim3(nblk(rows, DISC_B)), dim3(DISC_B),
                                                     0, st, sv, src[0], src[1], src[2], hemi_n ? 1 : 0,
                                                     hemi_n ? hemi_n[0] : 0.0, hemi_n ? hemi_n[1] : 0.0,
                                                     hemi_n ? hemi_n[2] : 0.0, rows, K, hits.as<int32_t>(), d_segs)));
            HIP_CHECK(hipGetLastError());
        }
        nkeys = rows * K + 1;
        keys = Scratch(c, sizeof(uint64_t) * (size_t)nkeys, st);
        HIP_CHECK(hipMemsetAsync(keys.as<uint64_t>() + rows * K, 0, sizeof(uint64_t), st));
        if (rows > 0 && sv.n_tri > 0) {
            hipLaunchKernelGGL(k_prefix_keys, dim3(nblk(rows, 256)), dim3(256), 0, st, hits.as<int32_t>(), sv.surf,
                               rows, K, keys.as<uint64_t>());
            HIP_CHECK(hipGetLastError());
        } else if (rows * K > 0) {
            HIP_CHECK(hipMemsetAsync(keys.p, 0, sizeof(uint64_t) * (size_t)(rows * K), st));
        }
        if (keep_hits) {
            ch.n_hits_rows[which] = rows;
            ch.hits[which] = std::move(hits);
        }
    }
    sort_u64(c, keys.as<uint64_t>(), nkeys, RT_KEY_BITS * K, st);
    Scratch uniq(c, sizeof(uint64_t) * (size_t)nkeys, st);
    unique_u64(c, keys.as<uint64_t>(), uniq.as<uint64_t>(), nkeys, d_cnt, st);
    int64_t n = read_i64(d_cnt, st);
    out.n = n;
    out.keys = Scratch(c, sizeof(uint64_t) * (size_t)n, st);
    HIP_CHECK(hipMemcpyAsync(out.keys.p, uniq.p, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
    out.k = Scratch(c, sizeof(int32_t) * (size_t)n, st);
    out.seq = Scratch(c, sizeof(int32_t) * 3 * (size_t)n, st);
    out.img = Scratch(c, sizeof(double) * 9 * (size_t)n, st);
    hipLaunchKernelGGL(k_cand_prep, dim3(nblk(n, 128)), dim3(128), 0, st, out.keys.as<uint64_t>(), n, sv, src[0],
                       src[1], src[2], out.k.as<int32_t>(), out.seq.as<int32_t>(), out.img.as<double>());
    HIP_CHECK(hipGetLastError());
}

struct PathSet {
    int64_t n = 0;
    Scratch cells, valid, amp, len, recs, rstart;
};

static void find_paths(Ctx& c, const SceneView& sv, int stk, const Cands& cd, const double* src,
                       const TraceArgs& a, bool brute, bool field, PathSet& ps, unsigned long long* d_segs,
                       unsigned long long* d_app, hipStream_t st)
{
    const int64_t R = a.R;
    const int64_t cells = R * cd.n;
    if (cells > ((int64_t)1 << 40)) throw inval_error("receivers x candidates too large for one call");
    CandView cv = cd.view();
    // worst case: every cell valid; the pool hands back pages that are never touched cheaply
    const int64_t cap = cells < ((int64_t)1 << 24) ? cells : ((int64_t)1 << 24);
    Scratch raw(c, sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1), st);
    HIP_CHECK(hipMemsetAsync(d_app, 0, sizeof(unsigned long long), st));
    int64_t n = 0;
    if (cells > 0) {
        hipLaunchKernelGGL(k_geo_cells, dim3(nblk(cells, 256)), dim3(256), 0, st, sv, cv, src[0], src[1], src[2],
                           a.rx_dev, R, raw.as<uint64_t>(), cap, d_app);
        HIP_CHECK(hipGetLastError());
        n = read_i64((const int64_t*)d_app, st);
        if (n > cap) throw inval_error("too many geometric paths for one call");
    }
    ps.n = n;
    int end_bit = 1;
    while (end_bit < 64 && ((uint64_t)1 << end_bit) < (uint64_t)(cells > 1 ? cells : 2)) ++end_bit;
    sort_u64(c, raw.as<uint64_t>(), n, end_bit, st);
    ps.cells = std::move(raw);
    ps.valid = Scratch(c, (size_t)(n > 0 ? n : 1), st);
    ps.recs = Scratch(c, sizeof(PathRec) * (size_t)(n > 0 ? n : 1), st);
    if (field) {
        ps.amp = Scratch(c, sizeof(float2) * (size_t)(n > 0 ? n : 1), st);
        ps.len = Scratch(c, sizeof(double) * (size_t)(n > 0 ? n : 1), st);
    }
    ps.rstart = Scratch(c, sizeof(int64_t) * (size_t)(R + 1), st);
    hipLaunchKernelGGL(k_rx_start, dim3(nblk(R + 1, 256)), dim3(256), 0, st, ps.cells.as<uint64_t>(), n, cd.n, R,
                       ps.rstart.as<int64_t>());
    HIP_CHECK(hipGetLastError());
    if (n == 0) return;
    SEL_BOOL(brute, BR,
             SEL_BOOL(field, FI,
                      SEL_STK(stk, hipLaunchKernelGGL((k_paths<BR, FI, STK>), dim3(nblk(n, LEG_B)), dim3(LEG_B), 0,
                                                      st, sv, cv, a.tc, src[0], src[1], src[2], a.rx_dev,
                                                      ps.cells.as<uint64_t>(), n, ps.valid.as<uint8_t>(),
                                                      ps.amp.as<float2>(), ps.len.as<double>(),
                                                      ps.recs.as<PathRec>(), d_segs))));
    HIP_CHECK(hipGetLastError());
}

struct StageTimer {
    bool on;
    hipStream_t st;
    std::vector<hipEvent_t> ev;
    StageTimer(bool o, hipStream_t s) : on(o), st(s) {}
    void mark() {
        if (!on) return;
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        HIP_CHECK(hipEventRecord(e, st));
        ev.push_back(e);
    }
    ~StageTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

void trace(Ctx& c, const TraceArgs& a, Channel& ch, TraceOut& out, bool timing, hipStream_t st)
{
    const SceneView sv = a.scene->view();
    const bool brute = (a.tc.flags & 4) != 0;
    const bool keep_hits = (a.tc.flags & 1) != 0;
    const bool keep_paths = (a.tc.flags & 2) != 0;
    const bool exhaustive = (a.tc.flags & 8) != 0;
    const bool count_work = (a.tc.flags & 16) != 0;
    const int stk = stack_depth_for(*a.scene, brute);
    const int64_t R = a.R;
    const int64_t M = a.ris ? a.ris->M : 0;
    ch.R = R;
    ch.M = M;
    ch.K = a.tc.K;
    StageTimer tm(timing, st);
    tm.mark();   // 0

    Scratch ctr(c, 128, st);
    HIP_CHECK(hipMemsetAsync(ctr.p, 0, 128, st));
    unsigned long long* d_disc = ctr.as<unsigned long long>();
    unsigned long long* d_legs = d_disc + 1;
    int64_t* d_cnt = (int64_t*)(d_disc + 2);
    unsigned long long* d_app = d_disc + 3;
    unsigned long long* d_work = d_disc + 8;   // 5 counters of the counting build
    tm.mark();   // 1

    // 1-3: candidates
    Cands ctx_tx, ctx_u;
    make_candidates(c, sv, stk, a.tc.tx, nullptr, a, brute, exhaustive, keep_hits, ch, 0, ctx_tx, d_disc, d_cnt, st);
    if (a.ris)
        make_candidates(c, sv, stk, a.ris->centre, a.ris->normal, a, brute, exhaustive, keep_hits, ch, 1, ctx_u,
                        d_disc, d_cnt, st);
    tm.mark();   // 2
    out.n_cand_tx = ctx_tx.n;
    out.n_cand_u = a.ris ? ctx_u.n : 0;

    // 4-6: environment paths
    ch.E_env = Scratch(c, sizeof(float2) * (size_t)R, st);
    {
        PathSet ps;
        find_paths(c, sv, stk, ctx_tx, a.tc.tx, a, brute, true, ps, d_legs, d_app, st);
        if (R > 0) {
            hipLaunchKernelGGL(k_env_reduce, dim3(nblk(R, 128)), dim3(128), 0, st, ps.rstart.as<int64_t>(), R,
                               ps.valid.as<uint8_t>(), ps.amp.as<float2>(), ch.E_env.as<float2>());
            HIP_CHECK(hipGetLastError());
        }
        Scratch off2(c, sizeof(int64_t) * (size_t)(ps.n > 0 ? ps.n : 1), st);
        scan_flags(c, ps.valid.as<uint8_t>(), off2.as<int64_t>(), ps.n, d_cnt, st);
        out.n_env = read_i64(d_cnt, st);
        ch.n_env = out.n_env;
        if (keep_paths) {
            ch.env = Scratch(c, sizeof(EnvRec) * (size_t)out.n_env, st);
            if (ps.n > 0) {
                hipLaunchKernelGGL(k_env_compact, dim3(nblk(ps.n, 128)), dim3(128), 0, st, ps.recs.as<PathRec>(),
                                   ctx_tx.view(), ps.valid.as<uint8_t>(), off2.as<int64_t>(), ps.amp.as<float2>(),
                                   ps.len.as<double>(), ps.n, ch.env.as<EnvRec>());
                HIP_CHECK(hipGetLastError());
            }
        }
    }
    tm.mark();   // 3

    if (!a.ris) {
        ch.H = Scratch(c, 0, st);
        tm.mark();
        tm.mark();
        tm.mark();
    } else {
        // centre sequences V(rx)
        Scratch uptr(c, sizeof(int64_t) * (size_t)(R + 1), st);
        Scratch useq;
        int64_t n_u = 0;
        {
            PathSet ps;
            find_paths(c, sv, stk, ctx_u, a.ris->centre, a, brute, false, ps, d_legs, d_app, st);
            Scratch f2(c, (size_t)(ps.n > 0 ? ps.n : 1), st), off2(c, sizeof(int64_t) * (size_t)(ps.n > 0 ? ps.n : 1), st);
            if (ps.n > 0) {
                hipLaunchKernelGGL(k_u_flags, dim3(nblk(ps.n, 256)), dim3(256), 0, st, ps.recs.as<PathRec>(),
                                   ps.valid.as<uint8_t>(), ps.n, f2.as<uint8_t>());
                HIP_CHECK(hipGetLastError());
            }
            scan_flags(c, f2.as<uint8_t>(), off2.as<int64_t>(), ps.n, d_cnt, st);
            n_u = read_i64(d_cnt, st);
            useq = Scratch(c, sizeof(int32_t) * 8 * (size_t)(n_u > 0 ? n_u : 1), st);
            if (ps.n > 0) {
                hipLaunchKernelGGL(k_u_compact, dim3(nblk(ps.n, 256)), dim3(256), 0, st, ps.recs.as<PathRec>(),
                                   ctx_u.view(), f2.as<uint8_t>(), off2.as<int64_t>(), ps.n, useq.as<int32_t>());
                HIP_CHECK(hipGetLastError());
            }
            hipLaunchKernelGGL(k_uptr, dim3(nblk(R + 1, 128)), dim3(128), 0, st, ps.rstart.as<int64_t>(), ps.n,
                               off2.as<int64_t>(), n_u, R, uptr.as<int64_t>());
            HIP_CHECK(hipGetLastError());
        }
        out.n_u = n_u;
        out.n_slots = n_u + R;
        ch.n_slots = out.n_slots;
        tm.mark();   // 4

        RisView rv;
        rv.M = (int32_t)M;
        rv.pad = 0;
        rv.elem = a.ris->elem.as<double>();
        for (int q = 0; q < 3; ++q) {
            rv.centre[q] = a.ris->centre[q];
            rv.normal[q] = a.ris->normal[q];
        }
        rv.dy = a.ris->dy;
        rv.dz = a.ris->dz;
        rv.gain = a.ris->gain > 0 ? a.ris->gain
                                  : 4.0 * 3.141592653589793 * a.ris->dy * a.ris->dz / (a.tc.lambda * a.tc.lambda);
        rv.q = a.ris->q;
        Scratch txm(c, sizeof(TxmRec) * (size_t)M, st);
        SEL_BOOL(brute, BR,
                 SEL_STK(stk, hipLaunchKernelGGL((k_txm<BR, STK>), dim3(nblk(M, 64)), dim3(64), 0, st, sv, a.tc, rv,
                                                 txm.as<TxmRec>(), d_legs)));
        HIP_CHECK(hipGetLastError());
        ch.H = Scratch(c, sizeof(float2) * (size_t)(R * M), st);
        if (keep_paths) ch.ris_valid = Scratch(c, (size_t)(out.n_slots * M), st);
        int n_mchunk = (int)((M + 63) / 64);
        int64_t waves = R * n_mchunk;
        int64_t threads = waves * 64;
        tm.mark();   // 5
        if (threads > 0) {
            if (count_work && !brute && !keep_paths) {
                SEL_STK(stk, hipLaunchKernelGGL((k_ris<false, false, STK, true>), dim3(nblk(threads, RIS_B)),
                                                dim3(RIS_B), 0, st, sv, a.tc, rv, txm.as<TxmRec>(), a.rx_dev, R,
                                                uptr.as<int64_t>(), useq.as<int32_t>(), n_mchunk, ch.H.as<float2>(),
                                                ch.ris_valid.as<uint8_t>(), d_legs, d_work));
            } else {
                SEL_BOOL(brute, BR,
                         SEL_BOOL(keep_paths, KP,
                                  SEL_STK(stk, hipLaunchKernelGGL((k_ris<BR, KP, STK, false>),
                                                                  dim3(nblk(threads, RIS_B)), dim3(RIS_B), 0, st, sv,
                                                                  a.tc, rv, txm.as<TxmRec>(), a.rx_dev, R,
                                                                  uptr.as<int64_t>(), useq.as<int32_t>(), n_mchunk,
                                                                  ch.H.as<float2>(), ch.ris_valid.as<uint8_t>(),
                                                                  d_legs, d_work))));
            }
        }
        HIP_CHECK(hipGetLastError());
        tm.mark();   // 6
        if (keep_paths) {
            ch.n_u = n_u;
            ch.useq = std::move(useq);
        }
    }
    if (keep_paths) {
        ch.n_cand[0] = ctx_tx.n;
        ch.cand_keys[0] = std::move(ctx_tx.keys);
        if (a.ris) {
            ch.n_cand[1] = ctx_u.n;
            ch.cand_keys[1] = std::move(ctx_u.keys);
        }
    }
    int64_t h[13];
    read_i64s((const int64_t*)d_disc, h, 13, st);
    tm.mark();   // 7
    out.disc_segments = h[0];
    out.leg_segments = h[1];
    for (int q = 0; q < 5; ++q) out.work[q] = h[8 + q];
    out.segments = h[0] + h[1];
    if (timing) {
        HIP_CHECK(hipStreamSynchronize(st));
        auto el = [&](int i, int j) {
            float ms = 0;
            HIP_CHECK(hipEventElapsedTime(&ms, tm.ev[i], tm.ev[j]));
            return ms;
        };
        out.ms[0] = el(0, 1);                  // setup
        out.ms[1] = el(1, 2);                  // discovery + dedupe + candidate images
        out.ms[2] = 0.0f;
        out.ms[3] = el(2, 3);                  // environment paths
        out.ms[4] = a.ris ? el(3, 4) : 0.0f;   // RIS-centre sequences
        out.ms[5] = a.ris ? el(5, 6) : 0.0f;   // per-element kernel (k_ris) alone
        out.ms[6] = a.ris ? el(4, 5) : 0.0f;   // Tx -> element legs
        out.ms[7] = el(0, 7);                  // total
    }
    ch.last_stream = st;
}

}  // namespace rt
