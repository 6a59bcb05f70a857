// Scene upload and linear BVH build on the device.
//
// LBVH after Karras, "Maximizing Parallelism in the Construction of BVHs,
// Octrees, and k-d Trees" (HPG 2012): 30-bit Morton codes of triangle
// centroids with the triangle index appended (unique 62-bit keys), radix
// sort, one thread per internal node finds its key range and split, then a
// bottom-up refit in which the second thread to reach a node writes it.
// Node boxes are inflated so that the FP32 slab test is conservative with
// respect to the exact ray/triangle formula.
//
// Layouts (leaf slot = rank of the triangle's key):
//   tri4  [3 * n]: (v0.xyz, id), (e1.xyz, surface), (e2.xyz, 0)
//   nodes [4 * (n - 1)]: (loL.xyz, childL), (hiL.xyz, childR), (loR.xyz, -), (hiR.xyz, -)
//   child >= 0: internal node; child < 0: leaf slot ~child.
// Surfaces: s_tris groups triangle indices by surface (ascending), s_ptr the
// CSR offsets, s_plane the plane of each surface's lowest-numbered triangle.
#pragma clang fp contract(off)

#include <cstring>
#include <vector>

#include "rt_host.hpp"
#include "rt_lbvh_core.hpp"

namespace rt {

__device__ __forceinline__ unsigned f2ord(float f)
{
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// bounds[0..2] min centroid, [3..5] max centroid, [6..8] min vertex, [9..11] max vertex
__device__ __forceinline__ unsigned wave_umin(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, (unsigned)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ unsigned wave_umax(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
    return v;
}

// FP64 vertices and their 2-D projection, reflection coefficients, surface
// ids, centroids; bounds of the centroids and of the vertices (order-preserving
// unsigned keys, reduced per wave, one atomic per wave and value).
__global__ void k_scene_prep(const float* V, const int32_t* T, const int32_t* surf_in, const float* rr,
                             const float* ri, int64_t nv, int64_t nt, double* v64, float2* refl,
                             int32_t* surf, float4* cent, unsigned* bounds, int32_t* bad, double* proj, int32_t* axes)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t < nt;
    float c[3] = {0, 0, 0};
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    if (live) {
        for (int j = 0; j < 3; ++j) {
            int32_t vi = T[3 * t + j];
            if (vi < 0 || vi >= nv) {
                atomicOr(bad, 1);
                vi = 0;
            }
            for (int k = 0; k < 3; ++k) {
                float x = V[3 * (int64_t)vi + k];
                if (!(x == x) || fabsf(x) > 1e6f) atomicOr(bad, 2);
                v64[9 * t + 3 * j + k] = (double)x;
                c[k] += x;
                lo[k] = fminf(lo[k], x);
                hi[k] = fmaxf(hi[k], x);
            }
        }
        triangle_projection(v64 + 9 * t, proj + 6 * t, axes + t);
        refl[t] = make_float2(rr[t], ri[t]);
        surf[t] = surf_in[t];
        if (surf_in[t] < 0) atomicOr(bad, 4);
        for (int k = 0; k < 3; ++k) c[k] = c[k] / 3.0f;
        cent[t] = make_float4(c[0], c[1], c[2], 0.0f);
    }
    const bool lead = (threadIdx.x & 63) == 0;
    for (int k = 0; k < 3; ++k) {
        const unsigned cmin = wave_umin(live ? f2ord(c[k]) : 0xffffffffu);
        const unsigned cmax = wave_umax(live ? f2ord(c[k]) : 0u);
        const unsigned vmin = wave_umin(live ? f2ord(lo[k]) : 0xffffffffu);
        const unsigned vmax = wave_umax(live ? f2ord(hi[k]) : 0u);
        if (lead) {
            atomicMin(&bounds[k], cmin);
            atomicMax(&bounds[3 + k], cmax);
            atomicMin(&bounds[6 + k], vmin);
            atomicMax(&bounds[9 + k], vmax);
        }
    }
}

// spread the low 21 bits of v to every third bit of 63 (bit i -> bit 3 i)
__device__ __forceinline__ uint64_t expand21(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

// Two-word sort keys: word 0 the triangle index, word 1 the 63-bit Morton code
// of the centroid (21 bits per axis over the scene bounds); sorted on word 1,
// stably, so equal codes stay in index order (the tie-break of the unique keys).
__global__ void k_morton(const float4* cent, const unsigned* bounds, int64_t nt, uint64_t* keys)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    float lo[3], ext[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = ord2f(bounds[k]);
        float hi = ord2f(bounds[3 + k]);
        ext[k] = hi - lo[k];
    }
    float4 c = cent[t];
    float cc[3] = {c.x, c.y, c.z};
    uint64_t q[3];
    for (int k = 0; k < 3; ++k) {
        float u = ext[k] > 0.0f ? (cc[k] - lo[k]) / ext[k] : 0.5f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        q[k] = (uint64_t)fminf(u * 2097152.0f, 2097151.0f);
    }
    keys[2 * t] = (uint64_t)t;
    keys[2 * t + 1] = (expand21(q[0]) << 2) | (expand21(q[1]) << 1) | expand21(q[2]);
}

struct Box6 {
    float lo[3], hi[3];
};

__device__ __forceinline__ int64_t clamp_index(int32_t v, int64_t n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Leaf data in sorted order.  Box padding: 1e-5 of the scene extent + 1e-6 m
// + 1e-5 |x| (indices are clamped: malformed input is reported after the build).
__global__ void k_leaves(const uint64_t* keys, const float* V, const int32_t* T, const int32_t* surf, int64_t nv,
                         int64_t nt, const unsigned* bounds, float4* tri4, float* lbox)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    float ext = 0.0f;
    for (int k = 0; k < 3; ++k) ext = fmaxf(ext, ord2f(bounds[9 + k]) - ord2f(bounds[6 + k]));
    const float pad = 1e-5f * ext + 1e-6f;
    int32_t t = (int32_t)keys[2 * i];   // word 0 of the sorted key: the triangle index
    const float* a = V + 3 * clamp_index(T[3 * t + 0], nv);
    const float* b = V + 3 * clamp_index(T[3 * t + 1], nv);
    const float* c = V + 3 * clamp_index(T[3 * t + 2], nv);
    tri4[3 * i + 0] = make_float4(a[0], a[1], a[2], __int_as_float(t));
    tri4[3 * i + 1] = make_float4(b[0] - a[0], b[1] - a[1], b[2] - a[2], __int_as_float(surf[t]));
    tri4[3 * i + 2] = make_float4(c[0] - a[0], c[1] - a[1], c[2] - a[2], 0.0f);
    for (int k = 0; k < 3; ++k) {
        float lo = fminf(a[k], fminf(b[k], c[k]));
        float hi = fmaxf(a[k], fmaxf(b[k], c[k]));
        float p = pad + 1e-5f * fmaxf(fabsf(lo), fabsf(hi));
        lbox[6 * i + k] = lo - p;
        lbox[6 * i + 3 + k] = hi + p;
    }
}

__global__ void k_karras(const uint64_t* keys, int64_t n, int32_t* child, int32_t* parent_int,
                         int32_t* parent_leaf)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    if (i == 0) parent_int[0] = -1;   // the root; every other node and every leaf gets its parent below
    int32_t cl, cr;
    lbvh_node<2>(keys, n, i, &cl, &cr);
    if (cl < 0) parent_leaf[~cl] = (int32_t)i;
    else parent_int[cl] = (int32_t)i;
    if (cr < 0) parent_leaf[~cr] = (int32_t)i;
    else parent_int[cr] = (int32_t)i;
    child[2 * i] = cl;
    child[2 * i + 1] = cr;
}

__device__ __forceinline__ void load_box(int32_t c, const float* lbox, const float* ibox, float* b)
{
    const volatile float* src = c < 0 ? (const volatile float*)(lbox + 6 * (int64_t)(~c))
                                      : (const volatile float*)(ibox + 6 * (int64_t)c);
    for (int k = 0; k < 6; ++k) b[k] = src[k];
}

__global__ void k_refit(const int32_t* child, const int32_t* parent_int, const int32_t* parent_leaf,
                        const float* lbox, float* ibox, int32_t* flags, float4* nodes, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p = parent_leaf[i];
    while (p >= 0 && p < n - 1) {
        __threadfence();
        int old = __hip_atomic_fetch_add(&flags[p], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0) return;
        int32_t cl = child[2 * p], cr = child[2 * p + 1];
        float bl[6], br[6];
        load_box(cl, lbox, ibox, bl);
        load_box(cr, lbox, ibox, br);
        nodes[4 * p + 0] = make_float4(bl[0], bl[1], bl[2], __int_as_float(cl));
        nodes[4 * p + 1] = make_float4(bl[3], bl[4], bl[5], __int_as_float(cr));
        nodes[4 * p + 2] = make_float4(br[0], br[1], br[2], 0.0f);
        nodes[4 * p + 3] = make_float4(br[3], br[4], br[5], 0.0f);
        volatile float* dst = ibox + 6 * (int64_t)p;
        for (int k = 0; k < 3; ++k) {
            dst[k] = fminf(bl[k], br[k]);
            dst[3 + k] = fmaxf(bl[3 + k], br[3 + k]);
        }
        __threadfence();
        p = parent_int[p];
    }
}

// Refit of a small tree in one workgroup, the leaf-to-root walk of the
// atomic refit with every shared word in LDS.  A walker carries the box of
// the node it comes from in registers and leaves it in the parent's slot for
// that side; per node one word holds the parent link (plus one, low 29
// bits) with the arrival count above it, so one LDS atomic per level both
// counts the arrival and yields the next node.  The first arrival at a node
// stops; the second has both boxes and takes the union.  A node that does
// not see exactly two arrivals marks the tree inconsistent (flag 8).
constexpr int RT_REFIT_SMALL = 2048;   // leaves
constexpr uint32_t RT_UP_LINK = (1u << 29) - 1;
__global__ __launch_bounds__(1024) void k_refit_small(const int32_t* child, const int32_t* parent_int,
                                                      const int32_t* parent_leaf, const float* lbox, float4* nodes,
                                                      int64_t n, int32_t* bad)
{
    __shared__ float side[(RT_REFIT_SMALL - 1) * 12];   // [node][left, right][lo xyz, hi xyz]
    __shared__ int32_t ch[2 * (RT_REFIT_SMALL - 1)];
    __shared__ uint32_t up[RT_REFIT_SMALL - 1];
    const int ni = (int)n - 1;
    for (int p = threadIdx.x; p < ni; p += blockDim.x) {
        ch[2 * p] = child[2 * p];
        ch[2 * p + 1] = child[2 * p + 1];
        const int32_t q = parent_int[p];
        up[p] = q >= -1 && q < ni ? (uint32_t)(q + 1) : RT_UP_LINK;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (int)n; i += blockDim.x) {
        float b[6];
        for (int k = 0; k < 6; ++k) b[k] = lbox[6 * (int64_t)i + k];
        int32_t from = ~i;
        int32_t p = parent_leaf[i];
        while (p >= 0 && p < ni) {
            const int32_t cl = ch[2 * p], cr = ch[2 * p + 1];
            const int me = from == cl ? 0 : 1;
            if (me == 1 && from != cr) {
                atomicOr(bad, 8);
                break;
            }
            float* mine = side + 12 * p + 6 * me;
            for (int k = 0; k < 6; ++k) mine[k] = b[k];
            const uint32_t old =
                __hip_atomic_fetch_add(&up[p], 1u << 29, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if ((old >> 29) == 0) break;   // first arrival: the other child completes p
            const float* l = side + 12 * p;
            const float* r = l + 6;
            nodes[4 * p + 0] = make_float4(l[0], l[1], l[2], __int_as_float(cl));
            nodes[4 * p + 1] = make_float4(l[3], l[4], l[5], __int_as_float(cr));
            nodes[4 * p + 2] = make_float4(r[0], r[1], r[2], 0.0f);
            nodes[4 * p + 3] = make_float4(r[3], r[4], r[5], 0.0f);
            for (int k = 0; k < 3; ++k) {
                b[k] = fminf(l[k], r[k]);
                b[3 + k] = fmaxf(l[3 + k], r[3 + k]);
            }
            from = p;
            p = (int32_t)(old & RT_UP_LINK) - 1;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < ni; p += blockDim.x)
        if ((up[p] >> 29) != 2) atomicOr(bad, 8);
}

// 4-wide nodes: every internal node of even depth lists its grandchildren
// (a leaf child stands for itself).  Boxes are copied from the binary nodes.
// Also the tree depth: the deepest leaf lies one below the deepest internal
// node (a broken parent chain gives 2^20).
__global__ void k_node4(const int32_t* child, const int32_t* parent_int, const float4* nodes, const float4* tri4,
                        int64_t ni, float4* node4, int32_t* maxd)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = n < ni;
    int d = 0;
    int32_t p = live ? parent_int[n] : -1;
    for (; p >= 0 && p < ni && d < 4096; p = parent_int[p]) ++d;
    const unsigned dl = !live ? 0u : (p != -1 ? (1u << 20) : (unsigned)d + 1u);
    const unsigned dm = wave_umax(dl);
    if ((threadIdx.x & 63) == 0 && dm > 0) atomicMax(maxd, (int32_t)dm);
    if (!live || (d & 1)) return;
    float lo[4][3], hi[4][3];
    int32_t ref[4];
    int cnt = 0;
    for (int side = 0; side < 2; ++side) {
        const int32_t c = child[2 * n + side];
        const float4 l = nodes[4 * n + 2 * side], h = nodes[4 * n + 2 * side + 1];
        if (c < 0) {
            lo[cnt][0] = l.x; lo[cnt][1] = l.y; lo[cnt][2] = l.z;
            hi[cnt][0] = h.x; hi[cnt][1] = h.y; hi[cnt][2] = h.z;
            ref[cnt++] = c;
        } else {
            for (int g = 0; g < 2; ++g) {
                const float4 gl = nodes[4 * c + 2 * g], gh = nodes[4 * c + 2 * g + 1];
                lo[cnt][0] = gl.x; lo[cnt][1] = gl.y; lo[cnt][2] = gl.z;
                hi[cnt][0] = gh.x; hi[cnt][1] = gh.y; hi[cnt][2] = gh.z;
                ref[cnt++] = child[2 * c + g];
            }
        }
    }
    for (int j = cnt; j < 4; ++j) {
        lo[j][0] = lo[j][1] = lo[j][2] = 0.0f;   // masked out by the reference
        hi[j][0] = hi[j][1] = hi[j][2] = 0.0f;
        ref[j] = 0x7fffffff;
    }
    float4* q = node4 + 8 * n;
    for (int a = 0; a < 3; ++a) {
        q[2 * a] = make_float4(lo[0][a], lo[1][a], lo[2][a], lo[3][a]);
        q[2 * a + 1] = make_float4(hi[0][a], hi[1][a], hi[2][a], hi[3][a]);
    }
    q[6] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]),
                       __int_as_float(ref[3]));
    // surface of each leaf entry (-1 for inner and unused entries): walks that ignore a surface
    // drop its leaves without visiting them
    int lsf[4];
    for (int j = 0; j < 4; ++j)
        lsf[j] = (ref[j] < 0 && ref[j] != 0x7fffffff) ? __float_as_int(tri4[3 * (int64_t)(~ref[j]) + 1].w) : -1;
    q[7] = make_float4(__int_as_float(lsf[0]), __int_as_float(lsf[1]), __int_as_float(lsf[2]), __int_as_float(lsf[3]));
}

// every internal node reached by exactly two children during the refit
__global__ void k_check_refit(const int32_t* flags, int64_t ni, int32_t* bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ni && flags[i] != 2) atomicOr(bad, 8);
}

// surfaces
// surface ids are clamped to 0..nt-1 (larger ones are reported as invalid)
__global__ void k_surf_keys(const int32_t* surf, int64_t nt, uint64_t* keys, int32_t* n_surf, int32_t* bad)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int32_t s = surf[t];
    if (s < 0 || s >= nt) {
        atomicOr(bad, 4);
        s = s < 0 ? 0 : (int32_t)(nt - 1);
    }
    keys[t] = ((uint64_t)(uint32_t)s << 32) | (uint64_t)t;
    atomicMax(n_surf, s + 1);
}

// CSR over surfaces from the sorted (surface, triangle) keys; an unused id
// gets an empty range (and is reported as invalid).
__global__ void k_surf_csr(const uint64_t* keys, int64_t nt, const int32_t* n_surf_p, int32_t* s_ptr, int32_t* s_tris,
                           int32_t* seen)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const int32_t n_surf = *n_surf_p;
    int32_t s = (int32_t)(keys[i] >> 32);
    s_tris[i] = (int32_t)(keys[i] & 0xffffffffu);
    int32_t prev = i == 0 ? -1 : (int32_t)(keys[i - 1] >> 32);
    if (prev != s) {
        atomicAdd(seen, 1);
        for (int32_t q = prev + 1; q <= s; ++q) s_ptr[q] = (int32_t)i;
    }
    if (i == nt - 1)
        for (int32_t q = s + 1; q <= n_surf; ++q) s_ptr[q] = (int32_t)nt;
}

// A surface's plane is that of its lowest-numbered triangle; every vertex of
// the surface must lie within RT_EPS (0.1 mm) of it (bad |= 16), and that
// triangle must not be degenerate (bad |= 32): the image method mirrors in
// this one plane for the whole surface.
__global__ void k_surf_plane(const int32_t* s_ptr, const int32_t* s_tris, const double* v64, const int32_t* n_surf_p,
                             double* s_plane, double* s_box, int32_t* bad)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= *n_surf_p) return;
    if (s_ptr[s] >= s_ptr[s + 1]) {
        for (int k = 0; k < 4; ++k) s_plane[4 * s + k] = 0.0;
        for (int k = 0; k < 3; ++k) {
            s_box[6 * s + k] = 1e300;
            s_box[6 * s + 3 + k] = -1e300;
        }
        return;
    }
    const double* v = v64 + 9 * (int64_t)s_tris[s_ptr[s]];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = v[3 + k] - v[k];
        e2[k] = v[6 + k] - v[k];
    }
    double n0 = e1[1] * e2[2] - e1[2] * e2[1];
    double n1 = e1[2] * e2[0] - e1[0] * e2[2];
    double n2 = e1[0] * e2[1] - e1[1] * e2[0];
    s_plane[4 * s + 0] = n0;
    s_plane[4 * s + 1] = n1;
    s_plane[4 * s + 2] = n2;
    const double dpl = n0 * v[0] + n1 * v[1] + n2 * v[2];
    s_plane[4 * s + 3] = dpl;
    const double nlen = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    if (!(nlen > 0.0)) atomicOr(bad, 32);
    const double tol = RT_EPS * nlen;
    int off_plane = 0;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int j = s_ptr[s]; j < s_ptr[s + 1]; ++j) {
        const double* w = v64 + 9 * (int64_t)s_tris[j];
        for (int a = 0; a < 3; ++a) {
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], w[3 * a + k]);
                hi[k] = fmax(hi[k], w[3 * a + k]);
            }
            const double dist = n0 * w[3 * a] + n1 * w[3 * a + 1] + n2 * w[3 * a + 2] - dpl;
            off_plane |= !(fabs(dist) <= tol);
        }
    }
    if (off_plane) atomicOr(bad, 16);
    for (int k = 0; k < 3; ++k) {
        s_box[6 * s + k] = lo[k] - 1e-9;
        s_box[6 * s + 3 + k] = hi[k] + 1e-9;
    }
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Containment grid: one thread per (surface, cell).  A surface gets a grid
// only if all its non-degenerate triangles use the same projection; a
// triangle is listed in every cell its projected box, grown by a margin that
// covers the rounding of the FP64 edge tests (relative to the coordinates and
// inversely to the shortest edge), overlaps.  Lists keep the surface's
// triangle order.
__global__ void k_surf_grid(const int32_t* s_ptr, const int32_t* s_tris, const double* t_proj,
                            const int32_t* t_axes, const double* s_box, const int32_t* n_surf_p, int32_t* g_axes,
                            double* g_frame, int32_t* g_cnt, int32_t* g_tris)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_surf = *n_surf_p;
    if (id >= n_surf * RT_SGRID_CELLS) return;
    const int sf = (int)(id / RT_SGRID_CELLS), cell = (int)(id % RT_SGRID_CELLS);
    const int b = s_ptr[sf], e = s_ptr[sf + 1];
    int ax = -1;
    bool same = true;
    for (int j = b; j < e; ++j) {
        const int a = t_axes[s_tris[j]];
        if (a & 16) continue;
        if (ax < 0) ax = a;
        else if (a != ax) same = false;
    }
    if (!same || ax < 0) {
        if (cell == 0) g_axes[sf] = -1;
        g_cnt[id] = 0;
        return;
    }
    const int i0 = ax & 3, i1 = (ax >> 2) & 3;
    const double* bx = s_box + 6 * sf;
    const double u0 = bx[i0], v0 = bx[i1];
    const double eu = bx[3 + i0] - u0, ev = bx[3 + i1] - v0;
    const double pu = eu > 0.0 ? (double)RT_SGRID / eu : 0.0, pv = ev > 0.0 ? (double)RT_SGRID / ev : 0.0;
    if (cell == 0) {
        g_axes[sf] = ax;
        g_frame[4 * sf + 0] = u0;
        g_frame[4 * sf + 1] = v0;
        g_frame[4 * sf + 2] = pu;
        g_frame[4 * sf + 3] = pv;
    }
    const int ci = cell / RT_SGRID, cj = cell % RT_SGRID;
    const int64_t base = (int64_t)b * RT_SGRID_CELLS + (int64_t)cell * (e - b);
    int n = 0;
    for (int j = b; j < e; ++j) {
        const int t = s_tris[j];
        if (t_axes[t] & 16) continue;   // contains nothing
        const double* q = t_proj + 6 * (int64_t)t;
        const double umin = fmin(q[0], fmin(q[2], q[4])), umax = fmax(q[0], fmax(q[2], q[4]));
        const double vmin = fmin(q[1], fmin(q[3], q[5])), vmax = fmax(q[1], fmax(q[3], q[5]));
        const double C = fmax(fmax(fabs(umin), fabs(umax)), fmax(fabs(vmin), fabs(vmax)));
        const double l0 = hypot(q[2] - q[0], q[3] - q[1]), l1 = hypot(q[4] - q[2], q[5] - q[3]),
                     l2 = hypot(q[0] - q[4], q[1] - q[5]);
        const double lmin = fmax(fmin(l0, fmin(l1, l2)), 1e-300);
        const double m = 1e-13 * (C * C / lmin) + 1e-9 * C + 1e-12;
        const int c0 = sgrid_index(umin - m, u0, pu), c1 = sgrid_index(umax + m, u0, pu);
        const int d0 = sgrid_index(vmin - m, v0, pv), d1 = sgrid_index(vmax + m, v0, pv);
        if (ci >= c0 && ci <= c1 && cj >= d0 && cj <= d1) g_tris[base + n++] = t;
    }
    g_cnt[id] = n;
}



// the scene's vertex bounds as floats (lower x y z, upper x y z)
__global__ void k_scene_box(const unsigned* bounds, float* box)
{
    const int i = threadIdx.x;
    if (i < 6) box[i] = ord2f(bounds[6 + i]);
}

__global__ void k_ctl_init(unsigned* ctl)
{
    int i = threadIdx.x;
    if (i >= 64) return;
    unsigned v = 0u;
    if (i < 3 || (i >= 6 && i < 9)) v = 0xffffffffu;   // running minima
    ctl[i] = v;
}

// unit normal of e1 x e2 per triangle (0 for a degenerate triangle)
__global__ void k_unit_normals(const double* v64, int64_t nt, double* nrm)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const double* v = v64 + 9 * t;
    const double ex = v[3] - v[0], ey = v[4] - v[1], ez = v[5] - v[2];
    const double fx = v[6] - v[0], fy = v[7] - v[1], fz = v[8] - v[2];
    const double nx = ey * fz - ez * fy, ny = ez * fx - ex * fz, nz = ex * fy - ey * fx;
    const double l = sqrt(nx * nx + ny * ny + nz * nz);
    const double il = l > 0.0 ? 1.0 / l : 0.0;
    nrm[3 * t + 0] = nx * il;
    nrm[3 * t + 1] = ny * il;
    nrm[3 * t + 2] = nz * il;
}

void scene_normals(Ctx& c, Scene& s, hipStream_t st)
{
    if (s.n_tri == 0 || s.nrm.bytes) return;
    s.nrm = Scratch(c, sizeof(double) * 3 * (size_t)s.n_tri, st);
    hipLaunchKernelGGL(k_unit_normals, dim3(blocks_for(s.n_tri, 256)), dim3(256), 0, st, s.v64.as<double>(), s.n_tri,
                       s.nrm.as<double>());
    HIP_CHECK(hipGetLastError());
}

void build_scene(Ctx& c, Scene& s, const float* V, int64_t nv, const int32_t* T, int64_t nt,
                 const int32_t* surf, const float* rr, const float* ri, hipStream_t st)
{
    s.n_tri = nt;
    if (nt == 0) {
        s.n_surf = 0;
        s.root = 0;
        return;
    }
    if (nt >= (int64_t)1 << 29) throw inval_error("too many triangles (at most 2^29 - 1)");
    // inputs in device memory are read in place (the build is complete before the call returns);
    // host arrays are staged
    Scratch stage_buf[5];
    auto input = [&](const void* p, size_t bytes, int slot) -> const void* {
        if (bytes == 0 || is_device_ptr(p)) return p;
        stage_buf[slot] = Scratch(c, bytes, st);
        HIP_CHECK(hipMemcpyAsync(stage_buf[slot].p, p, bytes, hipMemcpyDefault, st));
        return stage_buf[slot].p;
    };
    const float* dV = (const float*)input(V, sizeof(float) * 3 * (size_t)nv, 0);
    const int32_t* dT = (const int32_t*)input(T, sizeof(int32_t) * 3 * (size_t)nt, 1);
    const int32_t* dS = (const int32_t*)input(surf, sizeof(int32_t) * (size_t)nt, 2);
    const float* dR = (const float*)input(rr, sizeof(float) * (size_t)nt, 3);
    const float* dI = (const float*)input(ri, sizeof(float) * (size_t)nt, 4);

    s.v64 = Scratch(c, sizeof(double) * 9 * (size_t)nt, st);
    s.t_proj = Scratch(c, sizeof(double) * 6 * (size_t)nt, st);
    s.t_axes = Scratch(c, sizeof(int32_t) * (size_t)nt, st);
    s.refl = Scratch(c, sizeof(float2) * (size_t)nt, st);
    s.surf = Scratch(c, sizeof(int32_t) * (size_t)nt, st);
    s.tri4 = Scratch(c, sizeof(float4) * 3 * (size_t)nt, st);
    Scratch cent(c, sizeof(float4) * (size_t)nt, st);
    // control block: bounds[12] unsigned, bad, maxdepth, n_surf, seen
    Scratch ctl(c, 64 * sizeof(int32_t), st);
    unsigned* bounds = ctl.as<unsigned>();
    int32_t* bad = ctl.as<int32_t>() + 12;
    int32_t* maxd = ctl.as<int32_t>() + 13;
    int32_t* nsurf = ctl.as<int32_t>() + 14;
    int32_t* seen = ctl.as<int32_t>() + 15;
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, bounds);
    HIP_CHECK(hipGetLastError());
    const int B = 256;
    hipLaunchKernelGGL(k_scene_prep, dim3(blocks_for(nt, B)), dim3(B), 0, st, dV, dT, dS, dR, dI, nv, nt,
                       s.v64.as<double>(), s.refl.as<float2>(), s.surf.as<int32_t>(), cent.as<float4>(), bounds, bad,
                       s.t_proj.as<double>(), s.t_axes.as<int32_t>());
    HIP_CHECK(hipGetLastError());
    s.box = Scratch(c, 6 * sizeof(float), st);
    hipLaunchKernelGGL(k_scene_box, dim3(1), dim3(64), 0, st, bounds, s.box.as<float>());
    HIP_CHECK(hipGetLastError());
    Scratch keys_raw(c, 2 * sizeof(uint64_t) * (size_t)nt, st), keys(c, 2 * sizeof(uint64_t) * (size_t)nt, st);
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(nt, B)), dim3(B), 0, st, cent.as<float4>(), bounds, nt,
                       keys_raw.as<uint64_t>());
    HIP_CHECK(hipGetLastError());
    sort_keys(c, keys_raw.as<uint64_t>(), keys.as<uint64_t>(), nt, 2, 64, 127, st);
    Scratch lbox(c, sizeof(float) * 6 * (size_t)nt, st);
    hipLaunchKernelGGL(k_leaves, dim3(blocks_for(nt, B)), dim3(B), 0, st, keys.as<uint64_t>(), dV, dT,
                       s.surf.as<int32_t>(), nv, nt, bounds, s.tri4.as<float4>(), lbox.as<float>());
    HIP_CHECK(hipGetLastError());

    if (nt >= 2) {
        int64_t ni = nt - 1;
        s.nodes = Scratch(c, sizeof(float4) * 4 * (size_t)ni, st);
        Scratch child(c, sizeof(int32_t) * 2 * (size_t)ni, st), pint(c, sizeof(int32_t) * (size_t)ni, st),
            pleaf(c, sizeof(int32_t) * (size_t)nt, st), ibox(c, sizeof(float) * 6 * (size_t)ni, st),
            flags(c, sizeof(int32_t) * (size_t)ni, st);
        const bool small = nt <= RT_REFIT_SMALL;
        if (!small) HIP_CHECK(hipMemsetAsync(flags.p, 0, flags.bytes, st));
        hipLaunchKernelGGL(k_karras, dim3(blocks_for(ni, B)), dim3(B), 0, st, keys.as<uint64_t>(), nt,
                           child.as<int32_t>(), pint.as<int32_t>(), pleaf.as<int32_t>());
        HIP_CHECK(hipGetLastError());
        if (small)
            hipLaunchKernelGGL(k_refit_small, dim3(1), dim3(1024), 0, st, child.as<int32_t>(), pint.as<int32_t>(),
                               pleaf.as<int32_t>(), lbox.as<float>(), s.nodes.as<float4>(), nt, bad);
        else
            hipLaunchKernelGGL(k_refit, dim3(blocks_for(nt, B)), dim3(B), 0, st, child.as<int32_t>(),
                               pint.as<int32_t>(), pleaf.as<int32_t>(), lbox.as<float>(), ibox.as<float>(),
                               flags.as<int32_t>(), s.nodes.as<float4>(), nt);
        HIP_CHECK(hipGetLastError());
        s.node4 = Scratch(c, sizeof(float4) * 8 * (size_t)ni, st);
        hipLaunchKernelGGL(k_node4, dim3(blocks_for(ni, B)), dim3(B), 0, st, child.as<int32_t>(), pint.as<int32_t>(),
                           s.nodes.as<float4>(), s.tri4.as<float4>(), ni, s.node4.as<float4>(), maxd);
        HIP_CHECK(hipGetLastError());
        if (!small) {
            hipLaunchKernelGGL(k_check_refit, dim3(blocks_for(ni, B)), dim3(B), 0, st, flags.as<int32_t>(), ni, bad);
            HIP_CHECK(hipGetLastError());
        }
        s.root = 0;
    } else {
        s.root = ~0;
    }

    // surfaces (tables sized for the largest valid count, n_surf <= n_tri)
    Scratch skeys(c, sizeof(uint64_t) * (size_t)nt, st);
    hipLaunchKernelGGL(k_surf_keys, dim3(blocks_for(nt, B)), dim3(B), 0, st, s.surf.as<int32_t>(), nt,
                       skeys.as<uint64_t>(), nsurf, bad);
    HIP_CHECK(hipGetLastError());
    {
        Scratch sorted(c, sizeof(uint64_t) * (size_t)nt, st);
        sort_u64_into(c, skeys.as<uint64_t>(), sorted.as<uint64_t>(), nt, 64, st);
        std::swap(skeys, sorted);
    }
    s.s_ptr = Scratch(c, sizeof(int32_t) * (size_t)(nt + 1), st);
    s.s_tris = Scratch(c, sizeof(int32_t) * (size_t)nt, st);
    s.s_plane = Scratch(c, sizeof(double) * 4 * (size_t)nt, st);
    s.s_box = Scratch(c, sizeof(double) * 6 * (size_t)nt, st);
    hipLaunchKernelGGL(k_surf_csr, dim3(blocks_for(nt, B)), dim3(B), 0, st, skeys.as<uint64_t>(), nt, nsurf,
                       s.s_ptr.as<int32_t>(), s.s_tris.as<int32_t>(), seen);
    HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_surf_plane, dim3(blocks_for(nt, 64)), dim3(64), 0, st, s.s_ptr.as<int32_t>(),
                       s.s_tris.as<int32_t>(), s.v64.as<double>(), nsurf, s.s_plane.as<double>(),
                       s.s_box.as<double>(), bad);
    HIP_CHECK(hipGetLastError());
    s.g_axes = Scratch(c, sizeof(int32_t) * (size_t)nt, st);
    s.g_frame = Scratch(c, sizeof(double) * 4 * (size_t)nt, st);
    s.g_cnt = Scratch(c, sizeof(int32_t) * RT_SGRID_CELLS * (size_t)nt, st);
    s.g_tris = Scratch(c, sizeof(int32_t) * RT_SGRID_CELLS * (size_t)nt, st);
    hipLaunchKernelGGL(k_surf_grid, dim3(blocks_for(nt * RT_SGRID_CELLS, 128)), dim3(128), 0, st,
                       s.s_ptr.as<int32_t>(), s.s_tris.as<int32_t>(), s.t_proj.as<double>(), s.t_axes.as<int32_t>(),
                       s.s_box.as<double>(), nsurf, s.g_axes.as<int32_t>(), s.g_frame.as<double>(),
                       s.g_cnt.as<int32_t>(), s.g_tris.as<int32_t>());
    HIP_CHECK(hipGetLastError());
    // one read-back: input checks, tree checks, surface count
    int64_t hq[2];
    read_i64s((const int64_t*)(ctl.as<int32_t>() + 12), hq, 2, st);
    const int32_t badv = (int32_t)(hq[0] & 0xffffffff), depth = (int32_t)(hq[0] >> 32);
    const int32_t n_surf = (int32_t)(hq[1] & 0xffffffff), n_seen = (int32_t)(hq[1] >> 32);
    if (badv & 1) throw inval_error("triangle vertex index out of range");
    if (badv & 2) throw inval_error("vertex coordinate not finite or |x| > 1e6");
    if (badv & 4) throw inval_error("surface id outside 0..n_tri-1");
    if (badv & 8) throw hip_error("BVH build produced an inconsistent tree");
    if (depth > RT_STACK - 1) throw inval_error("BVH deeper than the traversal stack");
    if (n_seen != n_surf) throw inval_error("surface ids must be 0..n_surf-1, each used");
    if (n_surf > (1 << RT_KEY_BITS) - 1)   // a candidate key holds surface id + 1 in 21 bits
        throw inval_error("at most 2^21 - 1 surfaces");
    if (badv & 32) throw inval_error("the lowest-numbered triangle of a surface is degenerate (no plane)");
    if (badv & 16) throw inval_error("the triangles of a surface are not coplanar (a vertex lies more than "
                                     "0.1 mm from the plane of the surface's first triangle)");
    s.max_depth = depth;
    s.n_surf = n_surf;
}

}  // namespace rt
