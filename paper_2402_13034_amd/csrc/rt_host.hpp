// Host-side objects of the risrt runtime: context, device allocations and the
// scene / RIS / channel objects behind the C ABI handles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>
#include <stdexcept>
#include <string>
#include <vector>

#include "rt_internal.hpp"

namespace rt {

struct nomem_error : std::runtime_error {
    explicit nomem_error(const std::string& s) : std::runtime_error(s) {}
};
struct inval_error : std::runtime_error {
    explicit inval_error(const std::string& s) : std::runtime_error(s) {}
};

// A device block held by the context's cache after its last stream-ordered use.
struct CachedBlock {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;   // stream of the last use
    hipEvent_t done = nullptr;  // recorded on `st` after the block was released (shared by a batch)
};

struct Ctx {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> in_use{0};   // bytes of live allocations (charged to the budget)
    std::mutex mu;
    // caching allocator: size class -> released blocks
    std::mutex alloc_mu;
    std::multimap<size_t, CachedBlock> cache;
    uint64_t cached_bytes = 0;
    std::vector<hipEvent_t> ev_pool;   // events of reused blocks, recorded again by later releases
    std::unordered_map<hipEvent_t, int> ev_refs;   // cached blocks per release event
    // side streams lent to calls that fork work (default priority, non-blocking)
    std::mutex pool_mu;
    std::vector<hipStream_t> side_pool;
    std::vector<hipStream_t> side_all;
    // launch order of the discovery rows (built on first use, freed at shutdown)
    std::mutex fib_mu;
    int32_t* fib_perm = nullptr;
    int32_t* fib_off = nullptr;
    // unique candidate counts of the last call per branch (Tx, RIS centre):
    // the first hash set of the next call is sized from them
    std::atomic<int64_t> cand_hint[2] = {0, 0};
    // device address of this device's copy of the library's static scratch array
    // (the allocation-free sum); looked up once, when the context is opened
    void* static_scratch = nullptr;
    size_t static_scratch_bytes = 0;
};

// Borrow a side stream of the context for the lifetime of the object.
struct SideStream {
    Ctx& c;
    hipStream_t s = nullptr;
    explicit SideStream(Ctx& ctx);
    ~SideStream();
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
};

// Stream-ordered device allocation charged to the context's budget.
void* dalloc(Ctx& c, size_t bytes, hipStream_t st);
void dfree(Ctx& c, void* p, size_t bytes, hipStream_t st);
void release_cache(Ctx& c);

// While one is alive on a thread, the blocks that thread releases to its
// context wait in the batch; at its end one event per stream covers them all
// (instead of one event per block).  Its streams must outlive it.
struct FreeBatch {
    struct Item {
        void* p;
        size_t cls;
        hipStream_t st;
    };
    Ctx& c;
    FreeBatch* prev;
    std::vector<Item> items;
    explicit FreeBatch(Ctx& ctx);
    ~FreeBatch();
    void flush();
    FreeBatch(const FreeBatch&) = delete;
    FreeBatch& operator=(const FreeBatch&) = delete;
};

// RAII scratch buffer on a stream.
struct Scratch {
    Ctx* c = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    Scratch() = default;
    Scratch(Ctx& ctx, size_t n, hipStream_t s) : c(&ctx), bytes(n), st(s) { p = n ? dalloc(ctx, n, s) : nullptr; }
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    Scratch(Scratch&& o) noexcept { *this = std::move(o); }
    Scratch& operator=(Scratch&& o) noexcept {
        release();
        c = o.c; p = o.p; bytes = o.bytes; st = o.st;
        o.p = nullptr; o.bytes = 0;
        return *this;
    }
    ~Scratch() { release(); }
    void release() {
        if (p) dfree(*c, p, bytes, st);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct Scene {
    hipEvent_t ready = nullptr;   // recorded after the build
    hipStream_t ready_st = nullptr;   // the stream `ready` was recorded on
    int64_t n_tri = 0, n_surf = 0;
    int32_t root = 0;
    int32_t max_depth = 0;
    Scratch tri4, nodes, node4, v64, refl, surf, s_ptr, s_tris, s_plane, s_box, t_proj, t_axes;
    Scratch mat;   // float2 per triangle (eps_r, sigma), empty until set
    Scratch nrm;   // 3 doubles per triangle: unit normal, computed with the materials
    Scratch g_axes, g_frame, g_cnt, g_tris;
    Scratch box;   // 6 floats: the vertices' lower and upper corner
    SceneView view() const {
        SceneView v;
        v.n_tri = (int32_t)n_tri;
        v.n_surf = (int32_t)n_surf;
        v.root = root;
        v.pad = 0;
        v.tri4 = tri4.as<float4>();
        v.nodes = nodes.as<float4>();
        v.node4 = node4.as<float4>();
        v.v64 = v64.as<double>();
        v.refl = refl.as<float2>();
        v.mat = mat.bytes ? mat.as<float2>() : nullptr;
        v.nrm = nrm.bytes ? nrm.as<double>() : nullptr;
        v.surf = surf.as<int32_t>();
        v.s_ptr = s_ptr.as<int32_t>();
        v.s_tris = s_tris.as<int32_t>();
        v.s_plane = s_plane.as<double>();
        v.s_box = s_box.as<double>();
        v.t_proj = t_proj.as<double>();
        v.t_axes = t_axes.as<int32_t>();
        v.g_axes = g_axes.as<int32_t>();
        v.g_frame = g_frame.as<double>();
        v.g_cnt = g_cnt.as<int32_t>();
        v.g_tris = g_tris.as<int32_t>();
        return v;
    }
};

struct RisObj {
    int64_t M = 0;
    double centre[3], normal[3];
    double dy = 0, dz = 0, gain = 0, q = 1;
    Scratch elem;   // double [M * 3]
    Scratch order;  // int32 [M]: the elements in Morton order of their in-plane coordinates
};

struct Channel {
    hipEvent_t ready = nullptr;      // recorded when H / E_env are complete
    hipStream_t ready_st = nullptr;  // the stream `ready` was recorded on
    hipEvent_t split_ev = nullptr;   // recorded after the split of H
    int64_t R = 0, M = 0, K = 0;
    Scratch H;          // float2 [R * M]
    Scratch E_env;      // float2 [R]
    // kept on request
    int64_t n_hits_rows[2] = {0, 0};
    Scratch hits[2];    // int32 [rows * K]
    int64_t n_cand[2] = {0, 0};
    Scratch cand_keys[2];  // uint64 [n_cand * key_words]
    int64_t n_env = 0;
    Scratch env;        // rt_env_path-like records (device EnvRec)
    int64_t n_u = 0;
    Scratch useq;       // int32 rows of useq_stride: rx, surfaces s_0..s_{KM-1}, triangles, 0
    int useq_stride = 8;
    int key_words = 1;  // 64-bit words per candidate key (2 for orders 4 and 5)
    int64_t n_slots = 0;
    Scratch ris_valid;  // uint8 [n_slots * M]
    // kept for the impulse response (RT_FLAG_KEEP_CIR): environment cells of
    // every receiver (offsets, validity, amplitude, length) and, per RIS slot
    // and element, amplitude (0: no path) and unfolded length; slot offsets
    bool keep_cir = false;
    int64_t env_cells = 0;
    Scratch env_rstart, env_valid, env_amp, env_len;
    Scratch cir_amp, cir_len, cir_uptr;
    // split of H, cached for matrix-core sums
    int split_kind = 0; // 0 none; bf16: 1 real-Gamma layout, 2 complex-Gamma layout; fp16: 3, 4
    Scratch a_hi, a_lo;
    Scratch a_sexp;     // int32 [R]: fp16 split, per-receiver power-of-two scale exponents
    int64_t a_rows = 0, a_k = 0;
    // every stream that has read the split, with an event recorded after its last
    // read: a rebuild (new layout or format) waits on them all before it releases
    // the old split, so no sum still running elsewhere reads a reused block
    std::vector<std::pair<hipStream_t, hipEvent_t>> split_readers;
    hipStream_t last_stream = nullptr;
};

// Device record of one environment path (layout shared with rt_env_path).
struct EnvRec {
    int32_t rx;
    int32_t order;
    int32_t seq[RT_MAX_K];
    int32_t tri[RT_MAX_K];
    double length;
    float amp[2];
};

// ---- primitives (rt_prims.hip) ----
bool is_device_ptr(const void* p);
// stable LSD radix sort of keys of `words` (1 or 2) 64-bit words on bits
// [begin_bit, end_bit); `in` may be clobbered, in == out allowed
void sort_keys(Ctx& c, uint64_t* in, uint64_t* out, int64_t n, int words, int begin_bit, int end_bit, hipStream_t st);
// unique of sorted keys of `words` words; count written to device int64
void unique_keys(Ctx& c, const uint64_t* in, uint64_t* out, int64_t n, int words, int64_t* d_count, hipStream_t st);
void sort_u64(Ctx& c, uint64_t* keys, int64_t n, int end_bit, hipStream_t st);
void sort_u64_into(Ctx& c, uint64_t* keys_in, uint64_t* keys_out, int64_t n, int end_bit, hipStream_t st);
// unique of sorted keys; count written to device int64
void unique_u64(Ctx& c, const uint64_t* in, uint64_t* out, int64_t n, int64_t* d_count, hipStream_t st);
// exclusive scan of uint8 flags into int64 offsets; total written to d_total
void scan_flags(Ctx& c, const uint8_t* flags, int64_t* offsets, int64_t n, int64_t* d_total,
                hipStream_t st);
// exclusive scan of int64 values
void scan_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n, hipStream_t st);

// ---- scene build ----
void build_scene(Ctx& c, Scene& s, const float* V, int64_t nv, const int32_t* T, int64_t nt,
                 const int32_t* surf, const float* rr, const float* ri, hipStream_t st);
// Unit normals of the scene's triangles (FP64) into s.nrm, on `st`.
void scene_normals(Ctx& c, Scene& s, hipStream_t st);

// ---- trace ----
struct TraceArgs {
    const Scene* scene;
    const RisObj* ris;       // may be null
    TraceConst tc;
    const double* rx_dev;    // device [R * 3]
    int64_t R;
    int64_t n_rays;
};
struct TraceOut {
    int64_t segments = 0, disc_segments = 0, leg_segments = 0;
    int64_t n_cand_tx = 0, n_cand_u = 0, n_env = 0, n_u = 0, n_slots = 0;
    float ms[8] = {0};
    int64_t work[5] = {0, 0, 0, 0, 0};
    int64_t leg_walk_fallbacks = 0;
    int64_t n_in_seq = 0, n_in_paths = 0;
    int64_t disc_work[6] = {0, 0, 0, 0, 0, 0};
    float ms_disc[3] = {0.0f, 0.0f, 0.0f};
};
void trace(Ctx& c, const TraceArgs& a, Channel& ch, TraceOut& out, bool timing, hipStream_t st);
// impulse response of one configuration from a channel traced with RT_FLAG_KEEP_CIR
void cir(Ctx& c, const Channel& ch, const float* gamma, double bin_s, int64_t n_bins, float* out, hipStream_t st);

// ---- RIS sum ----
void ris_sum(Ctx& c, Channel& ch, const float* gamma, int64_t C, float scale, bool gamma_real,
             int precision, float* E_out, float* P_out, hipStream_t st);
// The same sum with its split buffers in caller-provided device memory (no
// allocation, no cached split): bytes needed, and the sum itself.
size_t ris_sum_scratch_bytes(int64_t R, int64_t M, int64_t C, bool gamma_real, int precision);
void ris_sum_in(const Channel& ch, const float* gamma, int64_t C, float scale, bool gamma_real, int precision,
                float* E_out, float* P_out, void* scratch, hipStream_t st);

// pinned host staging for size read-backs
int64_t read_i64(const int64_t* d, hipStream_t st);
void read_i64s(const int64_t* d, int64_t* h, int n, hipStream_t st);

}  // namespace rt
