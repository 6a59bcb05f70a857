// C ABI of the risrt library: contexts, handles, memory budget, argument
// checks, and the calls declared in include/risrt.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/risrt.h"
#include "rt_host.hpp"

namespace rt {

static thread_local std::string g_err;

// ---- allocation ----
// Blocks are rounded to a size class and, when released, kept in the
// context's cache with the stream of their last use and an event recorded
// there.  A request reuses a cached block of its class: at once on the same
// stream (stream order) or once the event has completed, else after a wait
// on the event on the requesting stream.  Events are pooled; the blocks
// released during one API call share one event per stream (FreeBatch).  New
// blocks come from hipMalloc; cached blocks are returned to the device when
// live + cached bytes would exceed the budget, and at shutdown.
static size_t size_class(size_t bytes)
{
    if (bytes <= 256) return 256;
    if (bytes <= ((size_t)4 << 20)) {
        size_t c = 512;
        while (c < bytes) c <<= 1;
        return c;
    }
    const size_t g = (size_t)2 << 20;
    return (bytes + g - 1) / g * g;
}

// one cached block fewer uses event e: back to the pool (or destroyed) with its last block
static void drop_event_ref_locked(Ctx& c, hipEvent_t e, bool keep)
{
    auto it = c.ev_refs.find(e);
    if (it != c.ev_refs.end() && --it->second > 0) return;
    if (it != c.ev_refs.end()) c.ev_refs.erase(it);
    if (keep)
        c.ev_pool.push_back(e);
    else
        (void)hipEventDestroy(e);
}

static void trim_cache_locked(Ctx& c, uint64_t need)
{
    // drop cached blocks (largest first) until live + cached + need fits the budget
    if (c.in_use.load() + c.cached_bytes + need <= c.budget) return;
    HIP_CHECK(hipDeviceSynchronize());
    while (!c.cache.empty() && c.in_use.load() + c.cached_bytes + need > c.budget) {
        auto it = std::prev(c.cache.end());
        drop_event_ref_locked(c, it->second.done, false);
        (void)hipFree(it->second.p);
        c.cached_bytes -= it->second.bytes;
        c.cache.erase(it);
    }
}

void* dalloc(Ctx& c, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return nullptr;
    const size_t cls = size_class(bytes);
    uint64_t cur = c.in_use.load();
    while (true) {
        if (cur + cls > c.budget)
            throw nomem_error("memory budget exceeded (" + std::to_string(cur + cls) + " > " +
                              std::to_string(c.budget) + " bytes)");
        if (c.in_use.compare_exchange_weak(cur, cur + cls)) break;
    }
    CachedBlock b;
    bool found = false;
    {
        std::lock_guard<std::mutex> lk(c.alloc_mu);
        auto range = c.cache.equal_range(cls);
        auto pick = c.cache.end();
        for (auto it = range.first; it != range.second; ++it) {
            if (it->second.st == st) {
                pick = it;
                break;
            }
            if (pick == c.cache.end()) pick = it;
        }
        if (pick != c.cache.end()) {
            b = pick->second;
            c.cache.erase(pick);
            c.cached_bytes -= b.bytes;
            found = true;
        } else {
            trim_cache_locked(c, cls);
        }
    }
    if (found) {
        // the block is this caller's now; its event goes back to the pool after the wait is enqueued
        if (b.st != st) {
            const hipError_t q = hipEventQuery(b.done);
            if (q != hipSuccess) {
                if (q != hipErrorNotReady) (void)hipGetLastError();
                (void)hipStreamWaitEvent(st, b.done, 0);
            }
        }
        std::lock_guard<std::mutex> lk(c.alloc_mu);
        drop_event_ref_locked(c, b.done, true);
        return b.p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
        c.in_use -= cls;
        (void)hipGetLastError();
        if (e == hipErrorOutOfMemory) throw nomem_error("device out of memory");
        throw hip_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return p;
}

// Order `st` after an object's ready event; work on the stream that recorded
// it is in order already (a wait would only add a marker to the stream).
static void wait_ready(hipStream_t st, hipEvent_t ready, hipStream_t ready_st)
{
    if (ready && ready_st != st) HIP_CHECK(hipStreamWaitEvent(st, ready, 0));
}

static thread_local FreeBatch* tl_batch = nullptr;

// a released block into the cache behind event e (already recorded on its stream)
static void cache_block_locked(Ctx& c, void* p, size_t cls, hipStream_t st, hipEvent_t e)
{
    CachedBlock b;
    b.p = p;
    b.bytes = cls;
    b.st = st;
    b.done = e;
    c.cache.emplace(cls, b);
    ++c.ev_refs[e];
}

// an event from the pool, recorded on st (null if HIP refused)
static hipEvent_t record_release(Ctx& c, hipStream_t st)
{
    hipEvent_t e = nullptr;
    {
        std::lock_guard<std::mutex> lk(c.alloc_mu);
        if (!c.ev_pool.empty()) {
            e = c.ev_pool.back();
            c.ev_pool.pop_back();
        }
    }
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
    if (e && hipEventRecord(e, st) != hipSuccess) {
        (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (!e) (void)hipGetLastError();
    return e;
}

void dfree(Ctx& c, void* p, size_t bytes, hipStream_t st)
{
    if (!p) return;
    const size_t cls = size_class(bytes);
    if (tl_batch && &tl_batch->c == &c) {
        tl_batch->items.push_back({p, cls, st});
        std::lock_guard<std::mutex> lk(c.alloc_mu);
        c.cached_bytes += cls;   // counted as cached while it waits in the batch
        c.in_use -= cls;
        return;
    }
    hipEvent_t e = record_release(c, st);
    if (!e) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(p);
        c.in_use -= cls;
        return;
    }
    std::lock_guard<std::mutex> lk(c.alloc_mu);
    cache_block_locked(c, p, cls, st, e);
    c.cached_bytes += cls;
    c.in_use -= cls;
}

FreeBatch::FreeBatch(Ctx& ctx) : c(ctx), prev(tl_batch) { tl_batch = this; }

FreeBatch::~FreeBatch()
{
    flush();
    tl_batch = prev;
}

void FreeBatch::flush()
{
    size_t done = 0;
    while (done < items.size()) {
        const hipStream_t st = items[done].st;
        hipEvent_t e = record_release(c, st);
        std::lock_guard<std::mutex> lk(c.alloc_mu);
        for (size_t i = done; i < items.size(); ++i) {
            if (items[i].p == nullptr || items[i].st != st) continue;   // placed already, or another stream
            if (e) {
                cache_block_locked(c, items[i].p, items[i].cls, st, e);
            } else {   // no event: wait for the stream and give the block back
                (void)hipStreamSynchronize(st);
                (void)hipFree(items[i].p);
                c.cached_bytes -= items[i].cls;
            }
            items[i].p = nullptr;   // placed
        }
        while (done < items.size() && items[done].p == nullptr) ++done;
    }
    items.clear();
}

void release_cache(Ctx& c)
{
    std::lock_guard<std::mutex> lk(c.alloc_mu);
    for (auto& kv : c.cache) (void)hipFree(kv.second.p);
    c.cache.clear();
    c.cached_bytes = 0;
    for (auto& kv : c.ev_refs) (void)hipEventDestroy(kv.first);
    c.ev_refs.clear();
    for (hipEvent_t e : c.ev_pool) (void)hipEventDestroy(e);
    c.ev_pool.clear();
}

SideStream::SideStream(Ctx& ctx) : c(ctx)
{
    std::lock_guard<std::mutex> lk(c.pool_mu);
    if (!c.side_pool.empty()) {
        s = c.side_pool.back();
        c.side_pool.pop_back();
    } else {
        HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c.side_all.push_back(s);
    }
}

SideStream::~SideStream()
{
    std::lock_guard<std::mutex> lk(c.pool_mu);
    c.side_pool.push_back(s);
}

// ---- small read-backs through a pinned buffer ----
static int64_t* pinned_buf()
{
    static thread_local int64_t* buf = nullptr;
    if (!buf) HIP_CHECK(hipHostMalloc((void**)&buf, 64 * sizeof(int64_t), hipHostMallocDefault));
    return buf;
}

int64_t read_i64(const int64_t* d, hipStream_t st)
{
    int64_t* h = pinned_buf();
    HIP_CHECK(hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    return h[0];
}

void read_i64s(const int64_t* d, int64_t* out, int n, hipStream_t st)
{
    int64_t* h = pinned_buf();
    HIP_CHECK(hipMemcpyAsync(h, d, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) out[i] = h[i];
}

}  // namespace rt

using namespace rt;

// ---- handles ----
struct Obj {
    int kind = 0;   // 1 scene, 2 ris, 3 channel
    std::unique_ptr<Scene> scene;
    std::unique_ptr<RisObj> ris;
    std::unique_ptr<Channel> channel;
    std::vector<hipStream_t> users;
    std::mutex mu;   // serialises calls that update the object (bf16 split cache)
};

struct rt_ctx_s {
    Ctx c;
    hipStream_t free_stream = nullptr;
    uint64_t next = 1;
    std::map<uint64_t, std::shared_ptr<Obj>> objs;
};

static_assert(sizeof(EnvRec) == sizeof(rt_env_path), "path record layout");

// Scratch of the allocation-free sum (rt_ris_sum_noalloc): a fixed array that
// every device the library runs on holds until the process ends.  In host code
// its name is only a stand-in; rt_init looks up this device's copy with
// hipGetSymbolAddress and the calls pass that address to the kernels.
#define RT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) unsigned char scratch[RT_STATIC_SCRATCH_BYTES];

namespace {

rt_status fail(rt_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

template <class F>
rt_status guarded(rt_ctx ctx, F&& f, bool batch_frees = true)
{
    if (!ctx) return fail(RT_EINVAL, "null context");
    try {
        HIP_CHECK(hipSetDevice(ctx->c.device));
        std::unique_ptr<FreeBatch> batch;
        if (batch_frees) batch = std::make_unique<FreeBatch>(ctx->c);
        try {
            rt_status s = f();
            if (s == RT_OK) g_err.clear();
            return s;
        } catch (...) {
            // A call that fails part-way (out of budget in the middle of a trace, say) may have
            // queued work on several streams that still reads buffers its unwinding released;
            // they reach the cache (where any stream may take them) only after that work is done.
            (void)hipDeviceSynchronize();
            throw;
        }
    } catch (const nomem_error& e) {
        return fail(RT_ENOMEM, e.what());
    } catch (const inval_error& e) {
        return fail(RT_EINVAL, e.what());
    } catch (const hip_error& e) {
        return fail(RT_EDEVICE, e.what());
    } catch (const std::exception& e) {
        return fail(RT_EDEVICE, e.what());
    }
}

std::shared_ptr<Obj> find(rt_ctx ctx, uint64_t h, int kind)
{
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    auto it = ctx->objs.find(h);
    if (it == ctx->objs.end() || it->second->kind != kind) return nullptr;
    return it->second;
}

uint64_t insert(rt_ctx ctx, std::shared_ptr<Obj> o)
{
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    uint64_t h = ctx->next++;
    ctx->objs[h] = std::move(o);
    return h;
}

void note_user(rt_ctx ctx, Obj& o, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(ctx->c.mu);
    for (auto u : o.users)
        if (u == st) return;
    o.users.push_back(st);
}

void retarget(Scratch& s, hipStream_t st) { s.st = st; }

// Release an object's memory once all work enqueued on its user streams is done.
void release_obj(rt_ctx ctx, Obj& o)
{
    std::vector<hipEvent_t> evs;
    for (auto u : o.users) {
        hipEvent_t e;
        HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(e, u));
        HIP_CHECK(hipStreamWaitEvent(ctx->free_stream, e, 0));
        evs.push_back(e);
    }
    hipStream_t fs = ctx->free_stream;
    if (o.scene) {
        Scene& s = *o.scene;
        for (Scratch* p : {&s.tri4, &s.nodes, &s.node4, &s.v64, &s.refl, &s.surf, &s.s_ptr, &s.s_tris, &s.s_plane,
                           &s.s_box, &s.t_proj, &s.t_axes, &s.g_axes, &s.g_frame, &s.g_cnt, &s.g_tris, &s.mat,
                           &s.nrm})
            retarget(*p, fs);
    }
    if (o.ris) {
        retarget(o.ris->elem, fs);
        retarget(o.ris->order, fs);
    }
    if (o.channel) {
        Channel& ch = *o.channel;
        for (Scratch* p : {&ch.H, &ch.E_env, &ch.hits[0], &ch.hits[1], &ch.cand_keys[0], &ch.cand_keys[1], &ch.env,
                           &ch.useq, &ch.ris_valid, &ch.a_hi, &ch.a_lo, &ch.a_sexp, &ch.env_rstart, &ch.env_valid,
                           &ch.env_amp, &ch.env_len, &ch.cir_amp, &ch.cir_len, &ch.cir_uptr})
            retarget(*p, fs);
    }
    if (o.scene && o.scene->ready) (void)hipEventDestroy(o.scene->ready);
    if (o.channel) {
        if (o.channel->ready) (void)hipEventDestroy(o.channel->ready);
        if (o.channel->split_ev) (void)hipEventDestroy(o.channel->split_ev);
        for (auto& rd : o.channel->split_readers) (void)hipEventDestroy(rd.second);
    }
    o.scene.reset();
    o.ris.reset();
    o.channel.reset();
    for (auto e : evs) (void)hipEventDestroy(e);
}

}  // namespace

extern "C" {

const char* rt_last_error(void) { return g_err.c_str(); }

rt_status rt_init(int device, uint64_t mem_budget_bytes, rt_ctx* out)
{
    if (!out) return fail(RT_EINVAL, "null output");
    try {
        int n = 0;
        HIP_CHECK(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) return fail(RT_EINVAL, "no such device");
        HIP_CHECK(hipSetDevice(device));
        auto* ctx = new rt_ctx_s();
        ctx->c.device = device;
        size_t fr = 0, tot = 0;
        HIP_CHECK(hipMemGetInfo(&fr, &tot));
        ctx->c.budget = mem_budget_bytes ? mem_budget_bytes : (uint64_t)(0.9 * (double)fr);
        void* sp = nullptr;
        const hipError_t se = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        if (se != hipSuccess || !sp) {
            delete ctx;
            return fail(RT_EDEVICE, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                        hipGetErrorString(se));
        }
        ctx->c.static_scratch = sp;
        ctx->c.static_scratch_bytes = RT_STATIC_SCRATCH_BYTES;
        HIP_CHECK(hipStreamCreateWithFlags(&ctx->free_stream, hipStreamNonBlocking));
        *out = ctx;
        g_err.clear();
        return RT_OK;
    } catch (const std::exception& e) {
        return fail(RT_EDEVICE, e.what());
    }
}

rt_status rt_shutdown(rt_ctx ctx)
{
    if (!ctx) return fail(RT_EINVAL, "null context");
    rt_status s = guarded(ctx, [&] {
        HIP_CHECK(hipDeviceSynchronize());
        for (auto& kv : ctx->objs) release_obj(ctx, *kv.second);
        ctx->objs.clear();
        HIP_CHECK(hipStreamSynchronize(ctx->free_stream));
        HIP_CHECK(hipStreamDestroy(ctx->free_stream));
        if (ctx->c.fib_perm) (void)hipFree(ctx->c.fib_perm);
        if (ctx->c.fib_off) (void)hipFree(ctx->c.fib_off);
        for (hipStream_t s : ctx->c.side_all) (void)hipStreamDestroy(s);
        release_cache(ctx->c);
        return RT_OK;
    }, false);
    delete ctx;
    return s;
}

rt_status rt_mem_info(rt_ctx ctx, uint64_t* in_use, uint64_t* budget)
{
    return guarded(ctx, [&] {
        if (in_use) *in_use = ctx->c.in_use.load();
        if (budget) *budget = ctx->c.budget;
        return RT_OK;
    });
}

rt_status rt_scene_create(rt_ctx ctx, const float* vtx_xyz, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                          const int32_t* surf, const float* refl_re, const float* refl_im, void* stream,
                          uint64_t* scene)
{
    return guarded(ctx, [&]() -> rt_status {
        if (!scene || n_vtx < 0 || n_tri < 0) return fail(RT_EINVAL, "bad scene arguments");
        if (n_tri > 0 && (!vtx_xyz || !tri || !surf || !refl_re || !refl_im || n_vtx == 0))
            return fail(RT_EINVAL, "null scene array");
        hipStream_t st = (hipStream_t)stream;
        auto o = std::make_shared<Obj>();
        o->kind = 1;
        o->scene = std::make_unique<Scene>();
        build_scene(ctx->c, *o->scene, vtx_xyz, n_vtx, tri, n_tri, surf, refl_re, refl_im, st);
        HIP_CHECK(hipEventCreateWithFlags(&o->scene->ready, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(o->scene->ready, st));
        o->scene->ready_st = st;
        o->users.push_back(st);
        *scene = insert(ctx, o);
        return RT_OK;
    });
}

rt_status rt_scene_info(rt_ctx ctx, uint64_t scene, int64_t* n_tri, int64_t* n_surf, int32_t* bvh_depth,
                        uint64_t* bytes)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, scene, 1);
        if (!o) return fail(RT_ENOTFOUND, "unknown scene handle");
        const Scene& sc = *o->scene;
        if (n_tri) *n_tri = sc.n_tri;
        if (n_surf) *n_surf = sc.n_surf;
        if (bvh_depth) *bvh_depth = sc.max_depth;
        if (bytes) {
            uint64_t b = 0;
            for (const Scratch* p : {&sc.tri4, &sc.nodes, &sc.node4, &sc.v64, &sc.refl, &sc.surf, &sc.s_ptr,
                                     &sc.s_tris, &sc.s_plane, &sc.s_box, &sc.t_proj, &sc.t_axes, &sc.g_axes,
                                     &sc.g_frame, &sc.g_cnt, &sc.g_tris, &sc.mat, &sc.nrm})
                b += p->bytes;
            *bytes = b;
        }
        return RT_OK;
    });
}

rt_status rt_scene_set_materials(rt_ctx ctx, uint64_t scene, const float* eps_r, const float* sigma, void* stream)
{
    return guarded(ctx, [&]() -> rt_status {
        auto so = find(ctx, scene, 1);
        if (!so) return fail(RT_ENOTFOUND, "unknown scene handle");
        Scene& sc = *so->scene;
        if (sc.n_tri > 0 && (!eps_r || !sigma)) return fail(RT_EINVAL, "null material array");
        if (sc.n_tri == 0) return RT_OK;
        std::vector<float> er((size_t)sc.n_tri), sg((size_t)sc.n_tri);
        HIP_CHECK(hipMemcpy(er.data(), eps_r, sizeof(float) * er.size(), hipMemcpyDefault));
        HIP_CHECK(hipMemcpy(sg.data(), sigma, sizeof(float) * sg.size(), hipMemcpyDefault));
        std::vector<float> m(2 * (size_t)sc.n_tri);
        for (int64_t t = 0; t < sc.n_tri; ++t) {
            if (!(er[t] >= 1.0f) || !(sg[t] >= 0.0f) || !std::isfinite(er[t]) || !std::isfinite(sg[t]))
                return fail(RT_EINVAL, "materials need eps_r >= 1 and sigma >= 0, finite");
            m[2 * t] = er[t];
            m[2 * t + 1] = sg[t];
        }
        hipStream_t st = (hipStream_t)stream;
        wait_ready(st, sc.ready, sc.ready_st);
        Scratch mat(ctx->c, sizeof(float) * m.size(), st);
        HIP_CHECK(hipMemcpyAsync(mat.p, m.data(), mat.bytes, hipMemcpyHostToDevice, st));
        HIP_CHECK(hipStreamSynchronize(st));   // the host staging buffer goes out of scope
        sc.mat = std::move(mat);
        scene_normals(ctx->c, sc, st);
        if (sc.ready) {
            HIP_CHECK(hipEventRecord(sc.ready, st));
            sc.ready_st = st;
        }
        return RT_OK;
    });
}

// Elements sorted by the Morton code of their coordinates in the RIS plane
// (16 bits per axis over the elements' extent; equal codes keep their index
// order).  Consecutive runs of 64 are compact patches of the surface (8 x 8
// blocks of a square array), so the legs a wave of the per-element kernel
// tests together lie in a thin tube; the order changes no result.
static std::vector<int32_t> element_order(const std::vector<double>& xyz, const double c[3], const double n[3])
{
    const size_t M = xyz.size() / 3;
    // in-plane axes: a = n x up (up = z, or x for a horizontal RIS), b = n x a
    const double up[3] = {fabs(n[2]) > 0.9 ? 1.0 : 0.0, 0.0, fabs(n[2]) > 0.9 ? 0.0 : 1.0};
    double a[3] = {n[1] * up[2] - n[2] * up[1], n[2] * up[0] - n[0] * up[2], n[0] * up[1] - n[1] * up[0]};
    const double al = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (double& v : a) v /= al;
    const double b[3] = {n[1] * a[2] - n[2] * a[1], n[2] * a[0] - n[0] * a[2], n[0] * a[1] - n[1] * a[0]};
    std::vector<double> u(M), v(M);
    double u0 = 1e300, u1 = -1e300, v0 = 1e300, v1 = -1e300;
    for (size_t i = 0; i < M; ++i) {
        const double d[3] = {xyz[3 * i] - c[0], xyz[3 * i + 1] - c[1], xyz[3 * i + 2] - c[2]};
        u[i] = d[0] * a[0] + d[1] * a[1] + d[2] * a[2];
        v[i] = d[0] * b[0] + d[1] * b[1] + d[2] * b[2];
        u0 = fmin(u0, u[i]);
        u1 = fmax(u1, u[i]);
        v0 = fmin(v0, v[i]);
        v1 = fmax(v1, v[i]);
    }
    auto quant = [](double x, double lo, double hi) -> uint32_t {
        if (!(hi > lo)) return 0u;
        const double t = (x - lo) / (hi - lo) * 65535.0;
        return (uint32_t)fmin(fmax(t + 0.5, 0.0), 65535.0);
    };
    auto spread = [](uint32_t x) -> uint64_t {   // 16 bits to the even positions of 32
        uint64_t y = x & 0xFFFFu;
        y = (y | (y << 8)) & 0x00FF00FFull;
        y = (y | (y << 4)) & 0x0F0F0F0Full;
        y = (y | (y << 2)) & 0x33333333ull;
        y = (y | (y << 1)) & 0x55555555ull;
        return y;
    };
    std::vector<std::pair<uint64_t, int32_t>> key(M);
    for (size_t i = 0; i < M; ++i)
        key[i] = {spread(quant(u[i], u0, u1)) | (spread(quant(v[i], v0, v1)) << 1), (int32_t)i};
    std::sort(key.begin(), key.end());
    std::vector<int32_t> ord(M);
    for (size_t i = 0; i < M; ++i) ord[i] = key[i].second;
    return ord;
}

rt_status rt_ris_create(rt_ctx ctx, const double* elem_xyz, int64_t M, const double centre[3], const double normal[3],
                        double dy, double dz, double elem_gain, double pattern_q, uint64_t* ris)
{
    return guarded(ctx, [&]() -> rt_status {
        if (!ris || M <= 0 || !elem_xyz || !centre || !normal) return fail(RT_EINVAL, "bad RIS arguments");
        if (M > (1 << 24)) return fail(RT_EUNSUPPORTED, "too many RIS elements");
        if (!(dy > 0) || !(dz > 0) || !(pattern_q >= 0)) return fail(RT_EINVAL, "bad element size or pattern");
        double nn = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
        if (!(nn > 0)) return fail(RT_EINVAL, "zero RIS normal");
        auto o = std::make_shared<Obj>();
        o->kind = 2;
        o->ris = std::make_unique<RisObj>();
        RisObj& r = *o->ris;
        r.M = M;
        for (int k = 0; k < 3; ++k) {
            r.centre[k] = centre[k];
            r.normal[k] = normal[k] / nn;
        }
        r.dy = dy;
        r.dz = dz;
        r.gain = elem_gain;
        r.q = pattern_q;
        r.elem = Scratch(ctx->c, sizeof(double) * 3 * (size_t)M, nullptr);
        HIP_CHECK(hipMemcpyAsync(r.elem.p, elem_xyz, r.elem.bytes, hipMemcpyDefault, nullptr));
        // the order the per-element kernel takes the elements in, 64 per wave
        std::vector<double> xyz((size_t)3 * M);
        HIP_CHECK(hipMemcpyAsync(xyz.data(), r.elem.p, r.elem.bytes, hipMemcpyDeviceToHost, nullptr));
        HIP_CHECK(hipStreamSynchronize(nullptr));
        const std::vector<int32_t> ord = element_order(xyz, r.centre, r.normal);
        r.order = Scratch(ctx->c, sizeof(int32_t) * (size_t)M, nullptr);
        HIP_CHECK(hipMemcpyAsync(r.order.p, ord.data(), r.order.bytes, hipMemcpyHostToDevice, nullptr));
        HIP_CHECK(hipStreamSynchronize(nullptr));
        o->users.push_back(nullptr);
        *ris = insert(ctx, o);
        return RT_OK;
    });
}

static void fill_antenna(Antenna& a, const double* axis, double gain, int32_t pattern, double param)
{
    double n = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    for (int k = 0; k < 3; ++k) a.axis[k] = axis[k] / n;
    a.axis_norm = sqrt(a.axis[0] * a.axis[0] + a.axis[1] * a.axis[1] + a.axis[2] * a.axis[2]);
    a.gain = gain;
    a.pattern = pattern;
    a.param = param;
}

rt_status rt_trace(rt_ctx ctx, uint64_t scene, uint64_t ris, const rt_tx* tx, const double* rx_xyz, int64_t R,
                   const rt_rx* rx, const rt_params* params, void* stream, uint64_t* channel, rt_stats* stats)
{
    return guarded(ctx, [&]() -> rt_status {
        if (!tx || !rx || !params || !channel || R < 0 || (R > 0 && !rx_xyz)) return fail(RT_EINVAL, "bad trace arguments");
        if (params->flags & ~1023u) return fail(RT_EINVAL, "unknown flag");
        if ((params->flags & 256u) && (params->flags & 32u))
            return fail(RT_EINVAL, "the impulse response keeps the direct incoming leg only (no RT_FLAG_RIS_INCOMING)");
        if ((params->flags & 64u) && (params->flags & 128u)) return fail(RT_EINVAL, "Fresnel TE and TM both set");
        if ((params->flags & 192u) && (params->flags & 16u))
            return fail(RT_EINVAL, "the counting build has no Fresnel variant");
        if (params->max_order < 0 || params->max_order > RT_MAX_K)
            return fail(RT_EUNSUPPORTED, "max_order must be 0.." + std::to_string(RT_MAX_K));
        if (!(params->freq_hz > 0) || params->n_rays < 0) return fail(RT_EINVAL, "bad frequency or ray count");
        // the geometry kernel's grid covers the receivers in blocks of 64 (at most 65535 of them);
        // checked here, before any work is queued
        if (R > (int64_t)65535 * 64) return fail(RT_EUNSUPPORTED, "at most 65535 x 64 receivers per trace");
        for (int32_t p : {tx->pattern, rx->pattern})
            if (p < 0 || p > 2) return fail(RT_EINVAL, "unknown pattern kind");
        double ta = tx->axis[0] * tx->axis[0] + tx->axis[1] * tx->axis[1] + tx->axis[2] * tx->axis[2];
        double ra = rx->axis[0] * rx->axis[0] + rx->axis[1] * rx->axis[1] + rx->axis[2] * rx->axis[2];
        if (!(ta > 0) || !(ra > 0)) return fail(RT_EINVAL, "zero antenna axis");
        if (!(tx->power_w >= 0) || !(tx->gain >= 0) || !(rx->gain >= 0)) return fail(RT_EINVAL, "bad power or gain");
        auto so = find(ctx, scene, 1);
        if (!so) return fail(RT_ENOTFOUND, "unknown scene handle");
        std::shared_ptr<Obj> ro;
        if (ris) {
            ro = find(ctx, ris, 2);
            if (!ro) return fail(RT_ENOTFOUND, "unknown RIS handle");
        }
        hipStream_t st = (hipStream_t)stream;
        note_user(ctx, *so, st);
        if (ro) note_user(ctx, *ro, st);
        wait_ready(st, so->scene->ready, so->scene->ready_st);
        TraceArgs a;
        a.scene = so->scene.get();
        a.ris = ro ? ro->ris.get() : nullptr;
        a.R = R;
        a.n_rays = params->n_rays;
        TraceConst& tc = a.tc;
        tc.lambda = 299792458.0 / params->freq_hz;
        tc.inv_lambda = 1.0 / tc.lambda;
        tc.lam_4pi = (float)(tc.lambda / (4.0 * 3.141592653589793));
        tc.two_eta0_pt_gt = 2.0 * 120.0 * 3.141592653589793 * tx->power_w * tx->gain;
        for (int k = 0; k < 3; ++k) tc.tx[k] = tx->pos[k];
        fill_antenna(tc.txa, tx->axis, tx->gain, tx->pattern, tx->param);
        fill_antenna(tc.rxa, rx->axis, rx->gain, rx->pattern, rx->param);
        tc.K = params->max_order;
        tc.flags = (int32_t)params->flags;
        tc.fresnel = (params->flags & 64u) ? 1 : (params->flags & 128u) ? 2 : 0;
        tc.pad = 0;
        tc.sig_scale = 1.0 / (2.0 * 3.141592653589793 * params->freq_hz * 8.8541878128e-12);
        if (tc.fresnel && so->scene->n_tri > 0 && !so->scene->mat.bytes)
            return fail(RT_EINVAL, "Fresnel coefficients need the scene's materials (rt_scene_set_materials)");
        auto o = std::make_shared<Obj>();
        o->kind = 3;
        o->channel = std::make_unique<Channel>();
        // receivers in device memory are read in place (the call waits for its work before it returns)
        Scratch rxd;
        if (R > 0 && !is_device_ptr(rx_xyz)) {
            rxd = Scratch(ctx->c, sizeof(double) * 3 * (size_t)R, st);
            HIP_CHECK(hipMemcpyAsync(rxd.p, rx_xyz, rxd.bytes, hipMemcpyDefault, st));
        }
        a.rx_dev = rxd.p ? rxd.as<double>() : rx_xyz;
        TraceOut out;
        trace(ctx->c, a, *o->channel, out, stats != nullptr, st);
        HIP_CHECK(hipEventCreateWithFlags(&o->channel->ready, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(o->channel->ready, st));
        o->channel->ready_st = st;
        o->users.push_back(st);
        if (stats) {
            stats->segments = out.segments;
            stats->discovery_segments = out.disc_segments;
            stats->leg_segments = out.leg_segments;
            stats->n_cand_tx = out.n_cand_tx;
            stats->n_cand_u = out.n_cand_u;
            stats->n_env_paths = out.n_env;
            stats->n_u_paths = out.n_u;
            stats->n_ris_slots = out.n_slots;
            for (int k = 0; k < 8; ++k) stats->ms_stage[k] = out.ms[k];
            for (int k = 0; k < 5; ++k) stats->ris_work[k] = out.work[k];
            stats->leg_walk_fallbacks = out.leg_walk_fallbacks;
            stats->n_in_seq = out.n_in_seq;
            stats->n_in_paths = out.n_in_paths;
            for (int q = 0; q < 6; ++q) stats->discovery_work[q] = out.disc_work[q];
            for (int q = 0; q < 3; ++q) stats->ms_discovery[q] = out.ms_disc[q];
        }
        *channel = insert(ctx, o);
        return RT_OK;
    });
}

rt_status rt_channel_create(rt_ctx ctx, int64_t R, int64_t M, const float* E_env, const float* H, void* stream,
                            uint64_t* channel)
{
    return guarded(ctx, [&]() -> rt_status {
        if (!channel || R < 0 || M < 0 || (R > 0 && !E_env) || (R * M > 0 && !H))
            return fail(RT_EINVAL, "bad channel arguments");
        hipStream_t st = (hipStream_t)stream;
        auto o = std::make_shared<Obj>();
        o->kind = 3;
        o->channel = std::make_unique<Channel>();
        Channel& ch = *o->channel;
        ch.R = R;
        ch.M = M;
        ch.E_env = Scratch(ctx->c, sizeof(float2) * (size_t)R, st);
        ch.H = Scratch(ctx->c, sizeof(float2) * (size_t)(R * M), st);
        if (R > 0) HIP_CHECK(hipMemcpyAsync(ch.E_env.p, E_env, ch.E_env.bytes, hipMemcpyDefault, st));
        if (R * M > 0) HIP_CHECK(hipMemcpyAsync(ch.H.p, H, ch.H.bytes, hipMemcpyDefault, st));
        HIP_CHECK(hipStreamSynchronize(st));
        HIP_CHECK(hipEventCreateWithFlags(&ch.ready, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(ch.ready, st));
        ch.ready_st = st;
        o->users.push_back(st);
        *channel = insert(ctx, o);
        return RT_OK;
    });
}

rt_status rt_channel_info(rt_ctx ctx, uint64_t channel, int64_t* R, int64_t* M, int64_t* n_env, int64_t* n_slots)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        if (R) *R = o->channel->R;
        if (M) *M = o->channel->M;
        if (n_env) *n_env = o->channel->n_env;
        if (n_slots) *n_slots = o->channel->n_slots;
        return RT_OK;
    });
}

rt_status rt_channel_read(rt_ctx ctx, uint64_t channel, float* E_env, float* H, void* stream)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        hipStream_t st = (hipStream_t)stream;
        note_user(ctx, *o, st);
        Channel& ch = *o->channel;
        wait_ready(st, ch.ready, ch.ready_st);
        if (E_env && ch.R > 0) HIP_CHECK(hipMemcpyAsync(E_env, ch.E_env.p, ch.E_env.bytes, hipMemcpyDefault, st));
        if (H && ch.R * ch.M > 0) HIP_CHECK(hipMemcpyAsync(H, ch.H.p, ch.H.bytes, hipMemcpyDefault, st));
        HIP_CHECK(hipStreamSynchronize(st));
        return RT_OK;
    });
}

rt_status rt_hits_read(rt_ctx ctx, uint64_t channel, int32_t source, int32_t* hits, int64_t cap, int64_t* rows)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        if (source < 0 || source > 1) return fail(RT_EINVAL, "source must be 0 or 1");
        Channel& ch = *o->channel;
        if (ch.ready) HIP_CHECK(hipEventSynchronize(ch.ready));
        int64_t n = ch.n_hits_rows[source];
        if (!ch.hits[source].p && n * ch.K > 0) return fail(RT_EINVAL, "hits not kept");
        if (rows) *rows = n;
        if (hits) {
            if (cap < n * ch.K) return fail(RT_EINVAL, "capacity too small");
            if (n * ch.K > 0) HIP_CHECK(hipMemcpy(hits, ch.hits[source].p, sizeof(int32_t) * (size_t)(n * ch.K), hipMemcpyDefault));
        }
        return RT_OK;
    });
}

rt_status rt_paths_read(rt_ctx ctx, uint64_t channel, rt_env_path* env, int64_t cap_env, int64_t* n_env,
                        int32_t* useq, int64_t cap_u, int64_t* n_u, uint8_t* ris_valid, int64_t cap_slots,
                        int64_t* n_slots)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        Channel& ch = *o->channel;
        if (ch.ready) HIP_CHECK(hipEventSynchronize(ch.ready));
        if (n_env) *n_env = ch.n_env;
        if (n_u) *n_u = ch.n_u;
        if (n_slots) *n_slots = ch.n_slots;
        if (env) {
            if (!ch.env.p && ch.n_env > 0) return fail(RT_EINVAL, "paths not kept");
            if (cap_env < ch.n_env) return fail(RT_EINVAL, "capacity too small");
            if (ch.n_env) HIP_CHECK(hipMemcpy(env, ch.env.p, sizeof(EnvRec) * (size_t)ch.n_env, hipMemcpyDefault));
        }
        if (useq) {
            if (cap_u < ch.n_u) return fail(RT_EINVAL, "capacity too small");
            if (ch.n_u) {
                if (!ch.useq.p) return fail(RT_EINVAL, "paths not kept");
                // internal rows: rx, s_0..s_{KM-1}, triangles, 0; out: rx, s_0..s_4 (-1 padded)
                const int us = ch.useq_stride, km = (us - 2) / 2;
                std::vector<int32_t> rows((size_t)(us * ch.n_u));
                HIP_CHECK(hipMemcpy(rows.data(), ch.useq.p, sizeof(int32_t) * rows.size(), hipMemcpyDefault));
                for (int64_t i = 0; i < ch.n_u; ++i) {
                    useq[(1 + RT_MAX_K) * i] = rows[us * i];
                    for (int j = 0; j < RT_MAX_K; ++j)
                        useq[(1 + RT_MAX_K) * i + 1 + j] = j < km ? rows[us * i + 1 + j] : -1;
                }
            }
        }
        if (ris_valid) {
            if (cap_slots < ch.n_slots) return fail(RT_EINVAL, "capacity too small");
            if (ch.n_slots * ch.M) {
                if (!ch.ris_valid.p) return fail(RT_EINVAL, "paths not kept");
                HIP_CHECK(hipMemcpy(ris_valid, ch.ris_valid.p, (size_t)(ch.n_slots * ch.M), hipMemcpyDefault));
            }
        }
        return RT_OK;
    });
}

rt_status rt_ris_paths_read(rt_ctx ctx, uint64_t channel, float* amp, double* length, int64_t cap_cells,
                           int64_t* n_cells)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        Channel& ch = *o->channel;
        if (ch.ready) HIP_CHECK(hipEventSynchronize(ch.ready));
        const int64_t n = ch.n_slots * ch.M;
        if (n_cells) *n_cells = n;
        if (!amp && !length) return RT_OK;
        if (n > 0 && !ch.cir_amp.p) return fail(RT_EINVAL, "paths not kept");
        if (cap_cells < n) return fail(RT_EINVAL, "capacity too small");
        if (n > 0 && amp) HIP_CHECK(hipMemcpy(amp, ch.cir_amp.p, sizeof(float2) * (size_t)n, hipMemcpyDefault));
        if (n > 0 && length) HIP_CHECK(hipMemcpy(length, ch.cir_len.p, sizeof(double) * (size_t)n, hipMemcpyDefault));
        return RT_OK;
    });
}

rt_status rt_candidates_read(rt_ctx ctx, uint64_t channel, int32_t source, int32_t* seq, int64_t cap, int64_t* n)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        if (source < 0 || source > 1) return fail(RT_EINVAL, "source must be 0 or 1");
        Channel& ch = *o->channel;
        if (ch.ready) HIP_CHECK(hipEventSynchronize(ch.ready));
        int64_t nc = ch.n_cand[source];
        if (n) *n = nc;
        if (seq) {
            if (!ch.cand_keys[source].p && nc > 0) return fail(RT_EINVAL, "candidates not kept");
            if (cap < RT_MAX_K * nc) return fail(RT_EINVAL, "capacity too small");
            const int w = ch.key_words;
            std::vector<uint64_t> keys((size_t)(w * nc));
            if (nc) HIP_CHECK(hipMemcpy(keys.data(), ch.cand_keys[source].p, sizeof(uint64_t) * keys.size(), hipMemcpyDefault));
            for (int64_t i = 0; i < nc; ++i)
                for (int j = 0; j < RT_MAX_K; ++j) {
                    // surfaces 0-2 in word 0, 3-4 in word 1 (two-word keys), 21 bits each
                    const uint64_t word = j < 3 ? keys[w * i] : (w == 2 ? keys[w * i + 1] : 0ull);
                    const uint64_t v = (word >> (RT_KEY_BITS * (j < 3 ? j : j - 3))) & ((1ull << RT_KEY_BITS) - 1);
                    const bool alive = v != 0 && (j == 0 || seq[RT_MAX_K * i + j - 1] >= 0);
                    seq[RT_MAX_K * i + j] = alive ? (int32_t)v - 1 : -1;
                }
        }
        return RT_OK;
    });
}

rt_status rt_ris_sum(rt_ctx ctx, uint64_t channel, const float* gamma, int64_t C, float gamma_scale,
                     int32_t gamma_is_real, int32_t precision, float* E_out, float* P_out, void* stream)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        if (C < 0 || precision < 0 || precision > 3) return fail(RT_EINVAL, "bad configuration count or precision");
        Channel& ch = *o->channel;
        if (C > 0 && ch.M > 0 && !is_device_ptr(gamma)) return fail(RT_EINVAL, "gamma must be device memory");
        if ((E_out && !is_device_ptr(E_out)) || (P_out && !is_device_ptr(P_out)))
            return fail(RT_EINVAL, "outputs must be device memory");
        if (C > ((int64_t)1 << 31) - 1) return fail(RT_EUNSUPPORTED, "too many configurations");
        hipStream_t st = (hipStream_t)stream;
        note_user(ctx, *o, st);
        std::lock_guard<std::mutex> lk(o->mu);
        wait_ready(st, ch.ready, ch.ready_st);
        ris_sum(ctx->c, ch, gamma, C, gamma_scale, gamma_is_real != 0, precision, E_out, P_out, st);
        return RT_OK;
    });
}

rt_status rt_ris_sum_noalloc(rt_ctx ctx, uint64_t channel, const float* gamma, int64_t C, float gamma_scale,
                            int32_t gamma_is_real, int32_t precision, float* E_out, float* P_out, void* stream)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        if (C < 0 || precision < 0 || precision > 3) return fail(RT_EINVAL, "bad configuration count or precision");
        const Channel& ch = *o->channel;
        if (C > 0 && ch.M > 0 && !is_device_ptr(gamma)) return fail(RT_EINVAL, "gamma must be device memory");
        if ((E_out && !is_device_ptr(E_out)) || (P_out && !is_device_ptr(P_out)))
            return fail(RT_EINVAL, "outputs must be device memory");
        if (C > ((int64_t)1 << 31) - 1) return fail(RT_EUNSUPPORTED, "too many configurations");
        const size_t need = ris_sum_scratch_bytes(ch.R, ch.M, C, gamma_is_real != 0, precision);
        if (need > ctx->c.static_scratch_bytes)
            return fail(RT_EUNSUPPORTED, "the sum needs " + std::to_string(need) + " bytes of scratch; the static "
                                         "scratch holds " + std::to_string(ctx->c.static_scratch_bytes) +
                                         " (use rt_ris_sum)");
        hipStream_t st = (hipStream_t)stream;
        note_user(ctx, *o, st);
        wait_ready(st, ch.ready, ch.ready_st);
        ris_sum_in(ch, gamma, C, gamma_scale, gamma_is_real != 0, precision, E_out, P_out, ctx->c.static_scratch, st);
        return RT_OK;
    }, false);
}

rt_status rt_cir(rt_ctx ctx, uint64_t channel, const float* gamma, double bin_s, int64_t n_bins, float* cir_out,
                 void* stream)
{
    return guarded(ctx, [&]() -> rt_status {
        auto o = find(ctx, channel, 3);
        if (!o) return fail(RT_ENOTFOUND, "unknown channel handle");
        Channel& ch = *o->channel;
        if (!ch.keep_cir) return fail(RT_EINVAL, "the channel was not traced with RT_FLAG_KEEP_CIR");
        if (!(bin_s > 0.0) || !std::isfinite(bin_s) || n_bins < 0 || n_bins > ((int64_t)1 << 24))
            return fail(RT_EINVAL, "bad delay bins");
        if (ch.R > 0 && n_bins > 0 && (!cir_out || !is_device_ptr(cir_out)))
            return fail(RT_EINVAL, "the output must be device memory");
        if (ch.R > 0 && ch.M > 0 && n_bins > 0 && (!gamma || !is_device_ptr(gamma)))
            return fail(RT_EINVAL, "gamma must be device memory");
        if (ch.R >= ((int64_t)1 << 31)) return fail(RT_EUNSUPPORTED, "too many receivers");
        hipStream_t st = (hipStream_t)stream;
        note_user(ctx, *o, st);
        std::lock_guard<std::mutex> lk(o->mu);
        wait_ready(st, ch.ready, ch.ready_st);
        cir(ctx->c, ch, gamma, bin_s, n_bins, cir_out, st);
        return RT_OK;
    });
}

rt_status rt_keys_sort(rt_ctx ctx, uint64_t* keys, int64_t n, int32_t words, int32_t begin_bit, int32_t end_bit,
                       int32_t unique, int64_t* n_out, void* stream)
{
    return guarded(ctx, [&]() -> rt_status {
        if (n < 0 || (words != 1 && words != 2) || begin_bit < 0 || end_bit > 64 * words || begin_bit > end_bit)
            return fail(RT_EINVAL, "bad key count, width or bit range");
        if (n > 0 && !is_device_ptr(keys)) return fail(RT_EINVAL, "keys must be device memory");
        if (n >= ((int64_t)1 << 32)) return fail(RT_EUNSUPPORTED, "too many keys");
        hipStream_t st = (hipStream_t)stream;
        Scratch tmp(ctx->c, sizeof(uint64_t) * (size_t)words * (size_t)(n > 0 ? n : 1), st);
        sort_keys(ctx->c, keys, tmp.as<uint64_t>(), n, words, begin_bit, end_bit, st);
        int64_t count = n;
        if (unique) {
            Scratch cnt(ctx->c, sizeof(int64_t), st);
            unique_keys(ctx->c, tmp.as<uint64_t>(), keys, n, words, cnt.as<int64_t>(), st);
            count = read_i64(cnt.as<int64_t>(), st);
        } else if (n > 0) {
            HIP_CHECK(hipMemcpyAsync(keys, tmp.p, sizeof(uint64_t) * (size_t)words * (size_t)n,
                                     hipMemcpyDeviceToDevice, st));
        }
        if (n_out) *n_out = count;
        return RT_OK;
    });
}

rt_status rt_destroy(rt_ctx ctx, uint64_t handle)
{
    return guarded(ctx, [&]() -> rt_status {
        std::shared_ptr<Obj> o;
        {
            std::lock_guard<std::mutex> lk(ctx->c.mu);
            auto it = ctx->objs.find(handle);
            if (it == ctx->objs.end()) return fail(RT_ENOTFOUND, "unknown handle");
            o = it->second;
            ctx->objs.erase(it);
        }
        release_obj(ctx, *o);
        return RT_OK;
    });
}

}  // extern "C"
