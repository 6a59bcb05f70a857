// Internal declarations of the risrt library (gfx950).
//
// Geometry decisions follow fixed formulas so that results are reproducible:
//   * ray/triangle: Moller-Trumbore in FP32, left-to-right sums, no fused
//     multiply-add, one correctly rounded division (1 / det);
//   * specular bounce: d' = d - (2 (d.n) / (n.n)) n, n = e1 x e2, FP32;
//   * image method, containment, side tests, lengths and phase: FP64 without
//     fused multiply-add.
// Files that include this header compile with contraction off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

#define RT_MAX_K 5            // largest reflection order (keys of two 64-bit words above 3)
#define RT_KM_SMALL 3        // orders up to this use one-word keys and the smaller kernel instances
#define RT_STACK 64          // BVH traversal stack entries per lane (LDS)
#define RT_EPS 1e-4          // metres: legs and bounces ignore hits closer than this
#define RT_KEY_BITS 21

namespace rt {

struct hip_error : std::runtime_error {
    explicit hip_error(const std::string& s) : std::runtime_error(s) {}
};

#define HIP_CHECK(x)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess)                                                               \
            throw ::rt::hip_error(std::string(#x) + ": " + hipGetErrorString(e_));           \
    } while (0)

// --------------------------------------------------------------------------
// Device views
// --------------------------------------------------------------------------
struct SceneView {
    int32_t n_tri;
    int32_t n_surf;
    int32_t root;          // >= 0 internal node, < 0 leaf ~slot; unused if n_tri == 0
    int32_t pad;
    const float4* tri4;    // 3 per leaf slot: (v0, id), (e1, surf), (e2, 0)
    const float4* nodes;   // 4 per internal node: (loL, cL), (hiL, cR), (loR, -), (hiR, -)
    const float4* node4;   // 8 per internal node of even depth (4-wide collapse), see RT_NODE4
    const double* v64;     // 9 per triangle (original order)
    const float2* refl;    // per triangle
    const float2* mat;     // per triangle: relative permittivity, conductivity S/m (null: none set)
    const double* nrm;     // per triangle unit normal e1 x e2 / |e1 x e2| (FP64), set with the materials
    const int32_t* surf;   // per triangle
    const int32_t* s_ptr;  // n_surf + 1
    const int32_t* s_tris; // triangles grouped by surface, ascending
    const double* s_plane; // 4 per surface: n (not unit), c = n . v0 of its first triangle
    const double* s_box;   // 6 per surface: lo, hi (inflated by 1e-9 m)
    const double* t_proj;  // 6 per triangle: a, b, c projected (counter-clockwise), see contains_proj
    const int32_t* t_axes; // per triangle: i0 | i1 << 2, 16 if degenerate
    // containment grid per surface (RT_SGRID x RT_SGRID cells over the surface box in the
    // projection all its triangles share; g_axes -1: no grid, scan every triangle)
    const int32_t* g_axes;   // per surface
    const double* g_frame;   // 4 per surface: u0, v0, cells per unit along u and v
    const int32_t* g_cnt;    // per (surface, cell): triangles listed
    const int32_t* g_tris;   // cell (c) of surface sf lists from s_ptr[sf] * cells + c * n_tris(sf)
};

#define RT_SGRID 4
#define RT_SGRID_CELLS (RT_SGRID * RT_SGRID)

// Grid cell coordinate of x (monotone in x, clamped to the grid)
__host__ __device__ __forceinline__ int sgrid_index(double x, double origin, double per_unit)
{
    double y = (x - origin) * per_unit;
    y = fmin(fmax(y, 0.0), (double)(RT_SGRID - 1));
    return (int)y;
}

struct Antenna {
    double axis[3];
    double axis_norm;      // |axis| in FP64
    double gain;
    int32_t pattern;
    double param;
};

struct TraceConst {
    double lambda;
    double two_eta0_pt_gt;   // 2 eta0 P_t G_t
    double tx[3];
    Antenna txa;
    Antenna rxa;
    int32_t K;
    int32_t flags;
    int32_t fresnel;       // 0: fixed coefficients; 1 TE, 2 TM Fresnel coefficients of the materials
    int32_t pad;
    double sig_scale;      // 1 / (omega eps0): eps = eps_r - j sigma sig_scale
    double inv_lambda;     // 1 / lambda (phase in turns = length x this)
    float lam_4pi;         // lambda / (4 pi) in FP32 (free-space amplitude factor over the length)
    int32_t pad2;
};

struct RisView {
    int32_t M;
    int32_t pad;
    const double* elem;    // 3 per element
    const int32_t* order;  // elements in the order the per-element kernel groups them (64 per wave)
    double centre[3];
    double normal[3];      // unit
    double normal_norm;    // |normal| in FP64
    double dy, dz, gain, q;
};

// --------------------------------------------------------------------------
// FP32 ray / triangle (same formula as the definition, no contraction)
// --------------------------------------------------------------------------
__device__ __forceinline__ bool mt_hit(float ox, float oy, float oz, float dx, float dy, float dz,
                                       float4 a, float4 b, float4 c, float tmin, float tmax,
                                       float& t_out)
{
#pragma clang fp contract(off)
    const float e1x = b.x, e1y = b.y, e1z = b.z;
    const float e2x = c.x, e2y = c.y, e2z = c.z;
    float px = dy * e2z - dz * e2y;
    float py = dz * e2x - dx * e2z;
    float pz = dx * e2y - dy * e2x;
    float det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0f) return false;
    float inv = 1.0f / det;
    float sx = ox - a.x;
    float sy = oy - a.y;
    float sz = oz - a.z;
    float u = (sx * px + sy * py + sz * pz) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    float qx = sy * e1z - sz * e1y;
    float qy = sz * e1x - sx * e1z;
    float qz = sx * e1y - sy * e1x;
    float v = (dx * qx + dy * qy + dz * qz) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
    if (!(t > tmin && t < tmax)) return false;
    t_out = t;
    return true;
}

__device__ __forceinline__ void reflect32(float4 b, float4 c, float& dx, float& dy, float& dz)
{
#pragma clang fp contract(off)
    float nx = b.y * c.z - b.z * c.y;
    float ny = b.z * c.x - b.x * c.z;
    float nz = b.x * c.y - b.y * c.x;
    float dn = dx * nx + dy * ny + dz * nz;
    float nn = nx * nx + ny * ny + nz * nz;
    float k = (2.0f * dn) / nn;
    dx = dx - k * nx;
    dy = dy - k * ny;
    dz = dz - k * nz;
}

// Work counters of the counting build of a kernel (node visits, triangle
// tests, FP64 containment tests).
struct WorkCount {
    uint32_t nodes = 0, tris = 0, contain = 0;
};

// --------------------------------------------------------------------------
// BVH walk.  Boxes are inflated at build time, so the slab test may use FMA:
// it never rejects a box holding a triangle the exact-formula test accepts.
// --------------------------------------------------------------------------
struct RayBox {
    float ix, iy, iz;     // 1 / d (zeros nudged to +-1e-30)
    float oix, oiy, oiz;  // o / d
};

__device__ __forceinline__ RayBox make_raybox(float ox, float oy, float oz, float dx, float dy, float dz)
{
    RayBox r;
    float sx = fabsf(dx) < 1e-30f ? copysignf(1e-30f, dx) : dx;
    float sy = fabsf(dy) < 1e-30f ? copysignf(1e-30f, dy) : dy;
    float sz = fabsf(dz) < 1e-30f ? copysignf(1e-30f, dz) : dz;
    r.ix = 1.0f / sx;
    r.iy = 1.0f / sy;
    r.iz = 1.0f / sz;
    r.oix = ox * r.ix;
    r.oiy = oy * r.iy;
    r.oiz = oz * r.iz;
    return r;
}

__device__ __forceinline__ bool slab(const RayBox& r, float4 lo, float4 hi, float tmin, float tmax,
                                     float& tn)
{
    float t0x = __builtin_fmaf(lo.x, r.ix, -r.oix), t1x = __builtin_fmaf(hi.x, r.ix, -r.oix);
    float t0y = __builtin_fmaf(lo.y, r.iy, -r.oiy), t1y = __builtin_fmaf(hi.y, r.iy, -r.oiy);
    float t0z = __builtin_fmaf(lo.z, r.iz, -r.oiz), t1z = __builtin_fmaf(hi.z, r.iz, -r.oiz);
    float a = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
    float b = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tn = a;
    return a <= b;
}

// Closest hit: lowest (t, triangle id) among triangles other than skip_tri
// with tmin < t < tmax.  Returns the leaf slot or -1.  `stack` points at this
// lane's column of an LDS array laid out [RT_STACK][stride].
// CNT: count the binary nodes visited and the triangles tested in *wc.
template <bool BRUTE, bool CNT = false>
__device__ int closest_hit(const SceneView& s, float ox, float oy, float oz, float dx, float dy,
                           float dz, float tmin, int skip_tri, int* stack, int stride, float& t_best,
                           int& id_best, WorkCount* wc = nullptr)
{
    t_best = __builtin_inff();
    id_best = 0x7fffffff;
    int slot_best = -1;
    if (s.n_tri == 0) return -1;
    if (BRUTE) {
        for (int i = 0; i < s.n_tri; ++i) {
            float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            int id = __float_as_int(a.w);
            if (id == skip_tri) continue;
            float t;
            if (mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, __builtin_inff(), t)) {
                if (t < t_best || (t == t_best && id < id_best)) {
                    t_best = t;
                    id_best = id;
                    slot_best = i;
                }
            }
        }
        return slot_best;
    }
    RayBox rb = make_raybox(ox, oy, oz, dx, dy, dz);
    int sp = 0;
    int node = s.root;
    while (true) {
        if (node >= 0) {
            if (CNT) wc->nodes++;
            const float4* nd = s.nodes + 4 * node;
            float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
            float tl, tr;
            bool hl = slab(rb, n0, n1, tmin, t_best, tl);
            bool hr = slab(rb, n2, n3, tmin, t_best, tr);
            int cl = __float_as_int(n0.w), cr = __float_as_int(n1.w);
            if (hl && hr) {
                int nearc = tl <= tr ? cl : cr;
                int farc = tl <= tr ? cr : cl;
                stack[sp * stride] = farc;
                ++sp;
                node = nearc;
                continue;
            } else if (hl) {
                node = cl;
                continue;
            } else if (hr) {
                node = cr;
                continue;
            }
        } else {
            int i = ~node;
            if (CNT) wc->tris++;
            float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            int id = __float_as_int(a.w);
            float t;
            if (id != skip_tri && mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, __builtin_inff(), t)) {
                if (t < t_best || (t == t_best && id < id_best)) {
                    t_best = t;
                    id_best = id;
                    slot_best = i;
                }
            }
        }
        if (sp == 0) break;
        --sp;
        node = stack[sp * stride];
    }
    return slot_best;
}

// Any hit of a triangle not on surface skip_a / skip_b with tmin < t < tmax.
template <bool BRUTE, bool CNT = false>
__device__ bool any_hit(const SceneView& s, float ox, float oy, float oz, float dx, float dy, float dz,
                        float tmin, float tmax, int skip_a, int skip_b, int* stack, int stride,
                        WorkCount* wc = nullptr)
{
    if (s.n_tri == 0) return false;
    if (BRUTE) {
        for (int i = 0; i < s.n_tri; ++i) {
            float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            int sf = __float_as_int(b.w);
            if (sf == skip_a || sf == skip_b) continue;
            float t;
            if (CNT) wc->tris++;
            if (mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, tmax, t)) return true;
        }
        return false;
    }
    RayBox rb = make_raybox(ox, oy, oz, dx, dy, dz);
    int sp = 0;
    int node = s.root;
    while (true) {
        if (node >= 0) {
            if (CNT) wc->nodes++;
            const float4* nd = s.nodes + 4 * node;
            float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
            float tl, tr;
            bool hl = slab(rb, n0, n1, tmin, tmax, tl);
            bool hr = slab(rb, n2, n3, tmin, tmax, tr);
            int cl = __float_as_int(n0.w), cr = __float_as_int(n1.w);
            if (hl && hr) {
                stack[sp * stride] = cr;
                ++sp;
                node = cl;
                continue;
            } else if (hl) {
                node = cl;
                continue;
            } else if (hr) {
                node = cr;
                continue;
            }
        } else {
            int i = ~node;
            float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            int sf = __float_as_int(b.w);
            float t;
            if (CNT && sf != skip_a && sf != skip_b) wc->tris++;
            if (sf != skip_a && sf != skip_b &&
                mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, tmax, t))
                return true;
        }
        if (sp == 0) break;
        --sp;
        node = stack[sp * stride];
    }
    return false;
}

// Leg A -> B blocked?  FP32 ray from fl(A) along fl((B - A) x (1 / L)), EPS < t < L - EPS,
// ignoring the surfaces sa, sb of its end points.
template <bool BRUTE, bool CNT = false>
__device__ bool leg_blocked(const SceneView& s, const double* A, const double* B, int sa, int sb,
                            int* stack, int stride, WorkCount* wc = nullptr)
{
#pragma clang fp contract(off)
    double w0 = B[0] - A[0], w1 = B[1] - A[1], w2 = B[2] - A[2];
    double L = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    float tmin = (float)RT_EPS;
    float tmax = (float)(L - RT_EPS);
    if (!(tmax > tmin)) return false;
    const double il = 1.0 / L;
    return any_hit<BRUTE, CNT>(s, (float)A[0], (float)A[1], (float)A[2], (float)(w0 * il), (float)(w1 * il),
                               (float)(w2 * il), tmin, tmax, sa, sb, stack, stride, wc);
}

// --------------------------------------------------------------------------
// Wave-coherent any hit.  The lanes of one wave walk the BVH together: a
// child is entered when its box test succeeds for any lane still searching;
// node index and stack are wave-uniform (one LDS stack per wave).  Each lane
// tests its own ray against every leaf reached, so its answer is exactly the
// per-lane any-hit answer (which does not depend on the nodes visited).
// Call from wave-uniform control flow; `searching` masks lanes out.
// --------------------------------------------------------------------------
template <bool CNT>
__device__ bool any_hit_wave(const SceneView& s, bool searching, float ox, float oy, float oz, float dx, float dy,
                             float dz, float tmin, float tmax, int skip_a, int skip_b, int* wstack,
                             WorkCount* wc)
{
    bool hit = false;
    if (s.n_tri == 0 || __ballot(searching) == 0ull) return false;
    RayBox rb = make_raybox(ox, oy, oz, dx, dy, dz);
    int sp = 0;
    int node = s.root;
    while (true) {
        if (node >= 0) {
            const float4* nd = s.nodes + 4 * node;
            float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
            float tl, tr;
            bool hl = searching && slab(rb, n0, n1, tmin, tmax, tl);
            bool hr = searching && slab(rb, n2, n3, tmin, tmax, tr);
            const unsigned long long bl = __ballot(hl), br = __ballot(hr);
            const int cl = __builtin_amdgcn_readfirstlane(__float_as_int(n0.w));
            const int cr = __builtin_amdgcn_readfirstlane(__float_as_int(n1.w));
            if (CNT) {
                if (hl && cl >= 0) wc->nodes++;
                if (hr && cr >= 0) wc->nodes++;
            }
            if (bl && br) {
                wstack[sp] = cr;
                ++sp;
                node = cl;
                continue;
            } else if (bl) {
                node = cl;
                continue;
            } else if (br) {
                node = cr;
                continue;
            }
        } else {
            const int i = ~node;
            float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            const int sf = __float_as_int(b.w);
            if (sf != skip_a && sf != skip_b && searching) {
                float t;
                if (CNT) wc->tris++;
                if (mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, tmax, t)) {
                    hit = true;
                    searching = false;
                }
            }
            if (__ballot(searching) == 0ull) break;
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(wstack[sp]);
    }
    return hit;
}

// 4-wide collapse of the binary tree, used by the wave-coherent walk: the
// node of every internal node n of even depth lists the grandchildren of n
// (or a child itself where that child is a leaf), with the boxes the binary
// nodes hold, so the boxes and the conservativeness of the test are the same.
// Layout per node (8 float4): lo.x, hi.x, lo.y, hi.y, lo.z, hi.z of the four
// entries, the four references (>= 0 node, < 0 ~leaf slot, RT_NODE4_EMPTY
// unused), and the surface of each leaf entry (-1 otherwise).  Node indices are those of the binary tree.  An
// unused entry has a zero box and is masked out by its reference.
#define RT_NODE4_EMPTY 0x7fffffff
#define RT_STACK4 (3 * (RT_STACK / 2) + 4)

__device__ __forceinline__ bool slab1(float lx, float hx, float ly, float hy, float lz, float hz, const RayBox& r,
                                      float tmin, float tmax)
{
    float t0x = __builtin_fmaf(lx, r.ix, -r.oix), t1x = __builtin_fmaf(hx, r.ix, -r.oix);
    float t0y = __builtin_fmaf(ly, r.iy, -r.oiy), t1y = __builtin_fmaf(hy, r.iy, -r.oiy);
    float t0z = __builtin_fmaf(lz, r.iz, -r.oiz), t1z = __builtin_fmaf(hz, r.iz, -r.oiz);
    float a = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
    float b = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    return a <= b;
}

// any_hit_wave over the 4-wide nodes (same answer per lane).  `wstack` holds
// RT_STACK4 entries for the wave.
__device__ bool any_hit_wave4(const SceneView& s, bool searching, float ox, float oy, float oz, float dx, float dy,
                              float dz, float tmin, float tmax, int skip_a, int skip_b, int* wstack)
{
    bool hit = false;
    if (s.n_tri == 0 || __ballot(searching) == 0ull) return false;
    const RayBox rb = make_raybox(ox, oy, oz, dx, dy, dz);
    int sp = 0;
    int node = s.root;
    while (true) {
        if (node >= 0) {
            const float4* q = s.node4 + 8 * node;
            const float4 lx = q[0], hx = q[1], ly = q[2], hy = q[3], lz = q[4], hz = q[5], cf = q[6], sfs = q[7];
            const int c0 = __float_as_int(cf.x), c1 = __float_as_int(cf.y);
            const int c2 = __float_as_int(cf.z), c3 = __float_as_int(cf.w);
            // unused entries and leaves of an ignored surface are masked after the ballot, without a branch
            const int f0 = __float_as_int(sfs.x), f1 = __float_as_int(sfs.y);
            const int f2 = __float_as_int(sfs.z), f3 = __float_as_int(sfs.w);
            const unsigned long long m0 = __ballot(slab1(lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, rb, tmin, tmax) & searching) &
                                          ((f0 >= 0 && (f0 == skip_a || f0 == skip_b)) ? 0ull : ~0ull);
            const unsigned long long m1 = __ballot(slab1(lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, rb, tmin, tmax) & searching) &
                                          ((f1 >= 0 && (f1 == skip_a || f1 == skip_b)) ? 0ull : ~0ull);
            const unsigned long long m2 = __ballot(slab1(lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, rb, tmin, tmax) & searching) &
                                          ((c2 == RT_NODE4_EMPTY || (f2 >= 0 && (f2 == skip_a || f2 == skip_b))) ? 0ull : ~0ull);
            const unsigned long long m3 = __ballot(slab1(lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, rb, tmin, tmax) & searching) &
                                          ((c3 == RT_NODE4_EMPTY || (f3 >= 0 && (f3 == skip_a || f3 == skip_b))) ? 0ull : ~0ull);
            // visit the first entry hit, push the others (last pushed = next visited)
            int next = RT_NODE4_EMPTY;
            if (m3) next = c3;
            if (m2) {
                if (next != RT_NODE4_EMPTY) wstack[sp++] = next;
                next = c2;
            }
            if (m1) {
                if (next != RT_NODE4_EMPTY) wstack[sp++] = next;
                next = c1;
            }
            if (m0) {
                if (next != RT_NODE4_EMPTY) wstack[sp++] = next;
                next = c0;
            }
            if (next != RT_NODE4_EMPTY) {
                node = next;
                continue;
            }
        } else {
            const int i = ~node;
            float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            const int sf = __float_as_int(b.w);
            if (sf != skip_a && sf != skip_b && searching) {
                float t;
                if (mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, tmax, t)) {
                    hit = true;
                    searching = false;
                }
            }
            if (__ballot(searching) == 0ull) break;
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(wstack[sp]);
    }
    return hit;
}

__device__ __forceinline__ bool slab1t(float lx, float hx, float ly, float hy, float lz, float hz, const RayBox& r,
                                       float tmin, float tmax, float& tn)
{
    float t0x = __builtin_fmaf(lx, r.ix, -r.oix), t1x = __builtin_fmaf(hx, r.ix, -r.oix);
    float t0y = __builtin_fmaf(ly, r.iy, -r.oiy), t1y = __builtin_fmaf(hy, r.iy, -r.oiy);
    float t0z = __builtin_fmaf(lz, r.iz, -r.oiz), t1z = __builtin_fmaf(hz, r.iz, -r.oiz);
    float a = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
    float b = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tn = a;
    return a <= b;
}

// Closest hit for a wave: the lanes walk the 4-wide nodes together (node
// data in scalar registers), each lane pruning boxes with its own best
// distance; the entries of a node are visited nearest first as seen by the
// first searching lane.  A lane's answer is the lowest (t, triangle id) over
// every triangle but skip_tri with tmin < t, as in closest_hit: a triangle
// is tested by every lane whenever some lane's ray reaches its box, and a
// lane only prunes boxes it cannot improve on.  wstack: RT_STACK4 entries.
__device__ int closest_hit_wave4(const SceneView& s, bool active, float ox, float oy, float oz, float dx, float dy,
                                 float dz, float tmin, int skip_tri, int* wstack, float& t_best, int& id_best)
{
    const float inf = __builtin_inff();
    t_best = inf;
    id_best = 0x7fffffff;
    int slot_best = -1;
    const unsigned long long act = __ballot(active);
    if (s.n_tri == 0 || act == 0ull) return -1;
    const int lead = __ffsll((long long)act) - 1;
    const RayBox rb = make_raybox(ox, oy, oz, dx, dy, dz);
    int sp = 0;
    int node = s.root;
    while (true) {
        if (node >= 0) {
            const float4* q = s.node4 + 8 * node;
            const float4 lx = q[0], hx = q[1], ly = q[2], hy = q[3], lz = q[4], hz = q[5], cf = q[6];
            int c0 = __float_as_int(cf.x), c1 = __float_as_int(cf.y);
            int c2 = __float_as_int(cf.z), c3 = __float_as_int(cf.w);
            float t0, t1, t2, t3;
            const bool h0 = slab1t(lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, rb, tmin, t_best, t0) & active;
            const bool h1 = slab1t(lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, rb, tmin, t_best, t1) & active;
            const bool h2 = slab1t(lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, rb, tmin, t_best, t2) & active;
            const bool h3 = slab1t(lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, rb, tmin, t_best, t3) & active;
            const bool v0 = __ballot(h0) != 0ull, v1 = __ballot(h1) != 0ull;
            const bool v2 = c2 != RT_NODE4_EMPTY && __ballot(h2) != 0ull;
            const bool v3 = c3 != RT_NODE4_EMPTY && __ballot(h3) != 0ull;
            // sort keys: the lead lane's entry distance; entries it misses after those it hits,
            // entries no lane hits (dropped) last
            const float big = 3.0e38f;
            float k0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h0 ? t0 : big), lead));
            float k1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h1 ? t1 : big), lead));
            float k2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h2 ? t2 : big), lead));
            float k3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h3 ? t3 : big), lead));
            k0 = v0 ? k0 : inf;
            k1 = v1 ? k1 : inf;
            k2 = v2 ? k2 : inf;
            k3 = v3 ? k3 : inf;
            c0 = v0 ? c0 : RT_NODE4_EMPTY;
            c1 = v1 ? c1 : RT_NODE4_EMPTY;
            c2 = v2 ? c2 : RT_NODE4_EMPTY;
            c3 = v3 ? c3 : RT_NODE4_EMPTY;
#define RT_CSWAP(ka, ca, kb, cb)                  \
    {                                             \
        const bool sw = kb < ka;                  \
        const float tk = sw ? kb : ka;            \
        kb = sw ? ka : kb;                        \
        ka = tk;                                  \
        const int tc = sw ? cb : ca;              \
        cb = sw ? ca : cb;                        \
        ca = tc;                                  \
    }
            RT_CSWAP(k0, c0, k1, c1)
            RT_CSWAP(k2, c2, k3, c3)
            RT_CSWAP(k0, c0, k2, c2)
            RT_CSWAP(k1, c1, k3, c3)
            RT_CSWAP(k1, c1, k2, c2)
#undef RT_CSWAP
            // the order is wave-uniform: keep it in scalar registers
            c0 = __builtin_amdgcn_readfirstlane(c0);
            c1 = __builtin_amdgcn_readfirstlane(c1);
            c2 = __builtin_amdgcn_readfirstlane(c2);
            c3 = __builtin_amdgcn_readfirstlane(c3);
            if (c3 != RT_NODE4_EMPTY) wstack[sp++] = c3;
            if (c2 != RT_NODE4_EMPTY) wstack[sp++] = c2;
            if (c1 != RT_NODE4_EMPTY) wstack[sp++] = c1;
            if (c0 != RT_NODE4_EMPTY) {
                node = c0;
                continue;
            }
        } else {
            const int i = ~node;
            const float4 a = s.tri4[3 * i], b = s.tri4[3 * i + 1], c = s.tri4[3 * i + 2];
            const int id = __float_as_int(a.w);
            if (active && id != skip_tri) {
                float t;
                if (mt_hit(ox, oy, oz, dx, dy, dz, a, b, c, tmin, inf, t)) {
                    if (t < t_best || (t == t_best && id < id_best)) {
                        t_best = t;
                        id_best = id;
                        slot_best = i;
                    }
                }
            }
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(wstack[sp]);
    }
    return slot_best;
}

// --------------------------------------------------------------------------
// Tube walk for a wave of nearly parallel segments (the legs of one slot for
// 64 RIS elements).  Every lane's tested segment o + t d, t in [tmin, tmax],
// lies within r of the central segment cA -> cB (the distance between points
// of equal parameter is at most the larger end-point distance), so a
// triangle the lane's own test can accept has its (inflated) leaf box within
// r of the central segment.  The wave walks the 4-wide nodes breadth first
// with only the central segment against boxes grown by r (+ a margin for the
// FP32 representation of the lanes' rays, the triangle test and the slab
// test), one entry per lane, collecting candidate leaves; then every lane
// tests its own ray against the candidates with the exact triangle test.
// The result per lane is the any-hit answer of the lane's ray (a superset of
// the triangles it could hit is tested with the same test).  If the frontier
// or the candidate list outgrows its LDS space, the wave falls back to the
// 4-wide wave walk.
// --------------------------------------------------------------------------
#define RT_TUBE_FRONT 128
#define RT_TUBE_CAND 128

// Maximum over the 64 lanes of a wave (every lane active), with DPP lane
// moves: butterflies inside rows of 16, then the row broadcasts of the
// 64-wide wave; lane 63 ends with the maximum.
__device__ __forceinline__ float wave_max(float v)
{
    int x = __float_as_int(v);
    x = __float_as_int(fmaxf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false))));
    x = __float_as_int(fmaxf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false))));
    x = __float_as_int(fmaxf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x124, 0xF, 0xF, false))));
    x = __float_as_int(fmaxf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x128, 0xF, 0xF, false))));
    x = __float_as_int(fmaxf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x142, 0xA, 0xF, false))));
    x = __float_as_int(fmaxf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x143, 0xC, 0xF, false))));
    return __int_as_float(__builtin_amdgcn_readlane(x, 63));
}

// All legs of one slot at once: one tube per leg, frontier and candidate
// entries tagged with their leg (3 bits above a 29-bit node or slot index),
// so the wave walks the levels of the tree once for up to KM + 1 legs.
// lb: the wave's leg rays in LDS, [leg][7][64] = ox, oy, oz, dx, dy, dz, tmax;
// tube: 8 floats per leg in LDS; front: 2 x RT_TUBE_FRONT ints, cand:
// RT_TUBE_CAND ints, wstack: RT_STACK4 ints (fallback), all per wave;
// seq: the slot's surfaces (wave-uniform), k its order; ok: the lane's path
// is still valid.  Returns the lane's bit set of blocked legs, plus
// RT_TUBE_FELL_BACK if the lists overflowed and the legs were walked one by
// one.
#define RT_TUBE_FELL_BACK 256u
#define RT_TUBE_TAG_SHIFT 29
#define RT_TUBE_IDX_MASK 0x1fffffffu
// a frontier or candidate entry: node or leaf slot index (< 2^29) and leg j (3 bits), as int
__device__ __forceinline__ int tube_entry(int idx, int j)
{
    return (int)((unsigned)idx | ((unsigned)j << RT_TUBE_TAG_SHIFT));
}
// surface at the start (a) or end (b) of leg j of a slot of order k (-1: a
// source or receiver), selected by value (j differs between lanes)
template <int KM>
__device__ __forceinline__ int leg_surface_a(const int* seq, int j)
{
    int v = -1;
#pragma unroll
    for (int q = 0; q < KM; ++q) v = (j == q + 1) ? seq[q] : v;
    return v;
}
template <int KM>
__device__ __forceinline__ int leg_surface_b(const int* seq, int j, int k)
{
    int v = -1;
#pragma unroll
    for (int q = 0; q < KM; ++q) v = (j == q && j != k) ? seq[q] : v;
    return v;
}

template <int KM>
__device__ __forceinline__ unsigned legs_blocked_tube(const SceneView& s, bool ok, int k, const int* seq,
                                                      const float* lb, float* tube, int* front, int* cand,
                                                      int* wstack)
{
    static_assert(KM + 1 <= 8, "three bits of leg index");
    const int lane = threadIdx.x & 63;
    const float tmin = (float)RT_EPS;
    unsigned blocked = 0;
    if (s.n_tri == 0 || __ballot(ok) == 0ull) return 0;
    const unsigned exact = 1u << 16;   // a tube radius not representable: exact walk
    unsigned live = 0;   // legs with a searching lane (uniform)
#pragma unroll
    for (int j = 0; j <= KM; ++j) {
        if (j > k) break;
        const float* r0 = lb + j * 7 * 64 + lane;
        const float ox = r0[0], oy = r0[64], oz = r0[128], dx = r0[192], dy = r0[256], dz = r0[320], tmax = r0[384];
        const bool searching = ok && tmax > tmin;
        const unsigned long long act = __ballot(searching);
        if (act == 0ull) continue;
        live |= 1u << j;
        // end points and distances in FP32: their rounding (a few 1e-7 relative) is far inside
        // the margin (1e-4 relative on r, 1e-4 m + 4e-6 x the coordinates' scale)
        const float ax = __builtin_fmaf(tmin, dx, ox), ay = __builtin_fmaf(tmin, dy, oy), az = __builtin_fmaf(tmin, dz, oz);
        const float bx = __builtin_fmaf(tmax, dx, ox), by = __builtin_fmaf(tmax, dy, oy), bz = __builtin_fmaf(tmax, dz, oz);
        const int lead = __ffsll((long long)act) - 1;
        const float cax = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ax), lead));
        const float cay = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ay), lead));
        const float caz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(az), lead));
        const float cbx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bx), lead));
        const float cby = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(by), lead));
        const float cbz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bz), lead));
        const float da = sqrtf((ax - cax) * (ax - cax) + (ay - cay) * (ay - cay) + (az - caz) * (az - caz));
        const float db = sqrtf((bx - cbx) * (bx - cbx) + (by - cby) * (by - cby) + (bz - cbz) * (bz - cbz));
        const float scale = fmaxf(fmaxf(fabsf(cax), fmaxf(fabsf(cay), fabsf(caz))),
                                  fmaxf(fabsf(cbx), fmaxf(fabsf(cby), fabsf(cbz)))) + fabsf(tmax);
        const float r = wave_max(searching ? fmaxf(da, db) * 1.0001f + 1e-4f + 4e-6f * scale : 0.0f);
        // central ray with hardware reciprocals (1 ulp): their error is inside the margin too
        RayBox crb;
        {
            float ex = cbx - cax, ey = cby - cay, ez = cbz - caz;
            ex = fabsf(ex) < 1e-30f ? copysignf(1e-30f, ex) : ex;
            ey = fabsf(ey) < 1e-30f ? copysignf(1e-30f, ey) : ey;
            ez = fabsf(ez) < 1e-30f ? copysignf(1e-30f, ez) : ez;
            crb.ix = __builtin_amdgcn_rcpf(ex);
            crb.iy = __builtin_amdgcn_rcpf(ey);
            crb.iz = __builtin_amdgcn_rcpf(ez);
            crb.oix = cax * crb.ix;
            crb.oiy = cay * crb.iy;
            crb.oiz = caz * crb.iz;
        }
        if (!(r < 1e30f)) live |= exact;   // not representable: exact walk below
        if (lane == 0) {
            float* t = tube + 8 * j;
            t[0] = crb.ix;
            t[1] = crb.iy;
            t[2] = crb.iz;
            t[3] = crb.oix;
            t[4] = crb.oiy;
            t[5] = crb.oiz;
            t[6] = r;
        }
    }
    if (live == 0) return 0;
    int nc = 0;
    bool overflow = (live & exact) != 0;
    if (!overflow) {
        if (s.root < 0) {
            for (int j = 0; j <= k; ++j)
                if (live & (1u << j)) {
                    if (lane == 0) cand[nc] = tube_entry(~s.root, j);
                    ++nc;
                }
        } else {
            int nf = 0, cur = 0;
            for (int j = 0; j <= k; ++j)
                if (live & (1u << j)) {
                    if (lane == 0) front[nf] = tube_entry(s.root, j);
                    ++nf;
                }
            while (nf > 0) {
                int nn = 0;
                int* fin = front + cur * RT_TUBE_FRONT;
                int* fout = front + (cur ^ 1) * RT_TUBE_FRONT;
                for (int base = 0; base < nf; base += 16) {
                    const int slot = base + (lane >> 2), e = lane & 3;
                    const bool valid = slot < nf;
                    const unsigned v = valid ? (unsigned)fin[slot] : 0u;
                    const int n = (int)(v & RT_TUBE_IDX_MASK), j = (int)(v >> RT_TUBE_TAG_SHIFT);
                    const float* t = tube + 8 * j;
                    RayBox crb;
                    crb.ix = t[0];
                    crb.iy = t[1];
                    crb.iz = t[2];
                    crb.oix = t[3];
                    crb.oiy = t[4];
                    crb.oiz = t[5];
                    const float r = t[6];
                    const float* q = (const float*)(s.node4 + 8 * n);
                    const int ref = __float_as_int(q[24 + e]);
                    // a leaf of one of the leg's end-point surfaces is never a candidate of that leg
                    const int lsf = __float_as_int(q[28 + e]);
                    const int sa = leg_surface_a<KM>(seq, j);
                    const int sb = leg_surface_b<KM>(seq, j, k);
                    const bool skip = lsf >= 0 && (lsf == sa || lsf == sb);
                    const bool hit = valid && ref != RT_NODE4_EMPTY && !skip &&
                                     slab1(q[e] - r, q[4 + e] + r, q[8 + e] - r, q[12 + e] + r, q[16 + e] - r,
                                           q[20 + e] + r, crb, -1e-3f, 1.001f);
                    const unsigned long long lt = (1ull << lane) - 1ull;
                    const unsigned long long mi = __ballot(hit && ref >= 0);
                    const unsigned long long ml = __ballot(hit && ref < 0);
                    if (hit && ref >= 0) {
                        const int idx = nn + __popcll(mi & lt);
                        if (idx < RT_TUBE_FRONT) fout[idx] = tube_entry(ref, j);
                    }
                    if (hit && ref < 0) {
                        const int idx = nc + __popcll(ml & lt);
                        if (idx < RT_TUBE_CAND) cand[idx] = tube_entry(~ref, j);
                    }
                    nn += __popcll(mi);
                    nc += __popcll(ml);
                }
                if (nn > RT_TUBE_FRONT || nc > RT_TUBE_CAND) {
                    overflow = true;
                    break;
                }
                nf = nn;
                cur ^= 1;
            }
        }
    }
    if (overflow) {   // exact walk of every leg
        blocked = RT_TUBE_FELL_BACK;
        for (int j = 0; j <= k; ++j) {
            const float* r0 = lb + j * 7 * 64 + lane;
            const float tmax = r0[384];
            const bool searching = ok && tmax > tmin;
            const int sa = j == 0 ? -1 : seq[j - 1];
            const int sb = j == k ? -1 : seq[j];
            if (any_hit_wave4(s, searching, r0[0], r0[64], r0[128], r0[192], r0[256], r0[320], tmin, tmax, sa, sb,
                              wstack))
                blocked |= 1u << j;
        }
        return blocked;
    }
    for (int i = 0; i < nc; ++i) {
        const unsigned v = (unsigned)__builtin_amdgcn_readfirstlane(cand[i]);
        const int slot = (int)(v & RT_TUBE_IDX_MASK), j = (int)(v >> RT_TUBE_TAG_SHIFT);
        const float4 a = s.tri4[3 * slot], b = s.tri4[3 * slot + 1], c = s.tri4[3 * slot + 2];
        const int sf = __float_as_int(b.w);
        const int sa = j == 0 ? -1 : seq[j - 1];
        const int sb = j == k ? -1 : seq[j];
        if (sf == sa || sf == sb) continue;
        const float* r0 = lb + j * 7 * 64 + lane;
        const float tmax = r0[384];
        if (ok && tmax > tmin && !(blocked & (1u << j))) {
            float t;
            if (mt_hit(r0[0], r0[64], r0[128], r0[192], r0[256], r0[320], a, b, c, tmin, tmax, t)) blocked |= 1u << j;
        }
    }
    return blocked;
}

// --------------------------------------------------------------------------
// FP64 image method
// --------------------------------------------------------------------------
__device__ __forceinline__ double edge_raw(double sx, double sy, double ex, double ey, double px,
                                           double py)
{
#pragma clang fp contract(off)
    return (ex - sx) * (py - sy) - (ey - sy) * (px - sx);
}

// Edge function from the lexicographically smaller end point (exactly
// antisymmetric in the edge direction).
__device__ __forceinline__ double edge2(double sx, double sy, double ex, double ey, double px,
                                        double py)
{
    bool s_first = (sx < ex) || (sx == ex && sy < ey);
    return s_first ? edge_raw(sx, sy, ex, ey, px, py) : -edge_raw(ex, ey, sx, sy, px, py);
}

__device__ __forceinline__ bool top_left(double sx, double sy, double ex, double ey)
{
    double dy = ey - sy, dx = ex - sx;
    return (dy < 0.0) || (dy == 0.0 && dx < 0.0);
}

// Projection used by the containment test, computed once per triangle (same
// FP64 operations as a test that derives it on the fly): drop the axis of
// largest |normal| (lowest axis on ties), keep the other two in cyclic order,
// make the projected triangle counter-clockwise.  Writes 6 coordinates and
// the axes (16 if the projected area is 0: such a triangle contains nothing).
__device__ inline void triangle_projection(const double* v, double* out, int32_t* axes)
{
#pragma clang fp contract(off)
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = v[3 + k] - v[k];
        e2[k] = v[6 + k] - v[k];
    }
    double n0 = e1[1] * e2[2] - e1[2] * e2[1];
    double n1 = e1[2] * e2[0] - e1[0] * e2[2];
    double n2 = e1[0] * e2[1] - e1[1] * e2[0];
    double ax = fabs(n0), ay = fabs(n1), az = fabs(n2);
    int drop = 0;
    if (ay > ax && ay >= az) drop = 1;
    else if (az > ax && az > ay) drop = 2;
    int i0 = (drop + 1) % 3, i1 = (drop + 2) % 3;
    double a0 = v[i0], a1 = v[i1];
    double b0 = v[3 + i0], b1 = v[3 + i1];
    double c0 = v[6 + i0], c1 = v[6 + i1];
    double area = edge2(a0, a1, b0, b1, c0, c1);
    if (area < 0.0) {
        double t0 = b0, t1 = b1;
        b0 = c0; b1 = c1;
        c0 = t0; c1 = t1;
    }
    out[0] = a0; out[1] = a1; out[2] = b0; out[3] = b1; out[4] = c0; out[5] = c1;
    *axes = (area == 0.0) ? 16 : (i0 | (i1 << 2));
}

// p on the triangle's plane inside triangle t?  Half-open top-left rule in
// the triangle's projection: a point on an edge belongs to the triangle only
// if that edge is top-left, so a point on an edge shared by two coplanar
// triangles belongs to exactly one of them.
__device__ inline bool contains_proj(const SceneView& s, int t, const double* p)
{
#pragma clang fp contract(off)
    const int ax = s.t_axes[t];
    if (ax & 16) return false;
    const double* q6 = s.t_proj + 6 * t;
    const double a0 = q6[0], a1 = q6[1], b0 = q6[2], b1 = q6[3], c0 = q6[4], c1 = q6[5];
    const double q0 = p[ax & 3], q1 = p[(ax >> 2) & 3];
    double w0 = edge2(b0, b1, c0, c1, q0, q1);
    double w1 = edge2(c0, c1, a0, a1, q0, q1);
    double w2 = edge2(a0, a1, b0, b1, q0, q1);
    bool in0 = (w0 > 0.0) || (w0 == 0.0 && top_left(b0, b1, c0, c1));
    bool in1 = (w1 > 0.0) || (w1 == 0.0 && top_left(c0, c1, a0, a1));
    bool in2 = (w2 > 0.0) || (w2 == 0.0 && top_left(a0, a1, b0, b1));
    return in0 && in1 && in2;
}

__device__ __forceinline__ double plane_side(const double* pl, const double* p)
{
#pragma clang fp contract(off)
    return (pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2]) - pl[3];
}

// Triangle of surface sf that contains p, or -1: the first in the
// surface's list.  With a grid, only the triangles listed for p's cell are
// tested, in list order: every triangle whose test could accept p overlaps
// that cell, so the answer is the same.  The counting build scans the whole
// list (the method's work).
template <bool CNT = false>
__device__ inline int surface_contains(const SceneView& s, int sf, const double* p, WorkCount* wc = nullptr)
{
    const double* bx = s.s_box + 6 * sf;
    if (p[0] < bx[0] || p[1] < bx[1] || p[2] < bx[2] || p[0] > bx[3] || p[1] > bx[4] || p[2] > bx[5])
        return -1;
    const int gax = CNT ? -1 : s.g_axes[sf];
    if (gax >= 0) {
        const double* fr = s.g_frame + 4 * sf;
        const int cell = sgrid_index(p[gax & 3], fr[0], fr[2]) * RT_SGRID + sgrid_index(p[(gax >> 2) & 3], fr[1], fr[3]);
        const int b = s.s_ptr[sf];
        const int64_t beg = (int64_t)b * RT_SGRID_CELLS + (int64_t)cell * (s.s_ptr[sf + 1] - b);
        const int cnt = s.g_cnt[sf * RT_SGRID_CELLS + cell];
        for (int j = 0; j < cnt; ++j) {
            const int t = s.g_tris[beg + j];
            if (contains_proj(s, t, p)) return t;
        }
        return -1;
    }
    for (int j = s.s_ptr[sf]; j < s.s_ptr[sf + 1]; ++j) {
        int t = s.s_tris[j];
        if (CNT) wc->contain++;
        if (contains_proj(s, t, p)) return t;
    }
    return -1;
}

// Mirror p in plane pl (n, c).
__device__ __forceinline__ void mirror(const double* pl, const double* p, double* out)
{
#pragma clang fp contract(off)
    double nn = pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2];
    double f = 2.0 * plane_side(pl, p) / nn;
    out[0] = p[0] - f * pl[0];
    out[1] = p[1] - f * pl[1];
    out[2] = p[2] - f * pl[2];
}

// Back-trace from X through images I[1..k] (I[0] = source S) over surfaces
// seq; on success fills P[0..k) and tri[0..k).  The loops run over the
// compile-time bound KM >= k with constant indices so the arrays stay in
// registers.
template <int KM>
__device__ inline bool image_backtrace(const SceneView& s, const int* seq, int k, const double (*I)[3],
                                       const double* X, double (*P)[3], int* tri)
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
        int t = surface_contains(s, seq[i - 1], p);
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

// --------------------------------------------------------------------------
// Patterns.  Whether a pattern factor is zero is decided on the FP64 cosine
// (cos^p: cos <= 0; monopole: sin(theta) = 0; isotropic: never), so that the
// decision does not depend on an underflow of the factor.  The amplitude
// factor sqrt(F) is evaluated directly in FP32: cos^(p/2), and the
// monopole's |cos(kh cos) - cos(kh)| / sin(theta) with sin^2 from FP64.
// --------------------------------------------------------------------------
__device__ __forceinline__ double cos_between(const double* v, const double* axis, double axis_norm)
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    return (v[0] * axis[0] + v[1] * axis[1] + v[2] * axis[2]) / (n * axis_norm);
}

__device__ __forceinline__ bool pattern_on(int kind, double c)
{
    c = fmin(1.0, fmax(-1.0, c));
    if (kind == 0) return true;
    if (kind == 1) return c > 0.0;
    return 1.0 - c * c > 0.0;
}

__device__ __forceinline__ float pattern_amp(int kind, double param, double c64)
{
    c64 = fmin(1.0, fmax(-1.0, c64));
    if (kind == 0) return 1.0f;
    if (kind == 1) {   // 2^((p/2) log2 c) with the hardware's base-2 logarithm and exponential (1 ulp each)
        const float c = (float)c64;
        return c > 0.0f ? __builtin_amdgcn_exp2f((float)(0.5 * param) * __builtin_amdgcn_logf(c)) : 0.0f;
    }
    const double s2 = 1.0 - c64 * c64;   // sin^2(theta) in FP64: no cancellation to 0 near the axis
    if (!(s2 > 0.0)) return 0.0f;
    const float c = (float)c64, kh = (float)(6.283185307179586 * param);
    return fabsf(cosf(kh * c) - cosf(kh)) / sqrtf((float)s2);
}

// Gate and amplitude factor sqrt(F) of a pattern for the direction v against
// its axis.  For cos^p the gate (cos > 0) is the sign of v . axis, the
// cosine's numerator (the same decision as the FP64 cosine's sign: its
// denominator is positive), and the amplitude needs the cosine only in FP32;
// the monopole's gate needs the FP64 cosine itself; the isotropic pattern
// needs neither.
__device__ __forceinline__ bool pattern_gate_amp(int kind, double param, const double* v, const double* axis,
                                                 double axis_norm, float& amp)
{
    if (kind == 0) {
        amp = 1.0f;
        return true;
    }
    if (kind == 1) {
        const double dn = v[0] * axis[0] + v[1] * axis[1] + v[2] * axis[2];
        const float vv = (float)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const float c = fminf(1.0f, (float)dn * __builtin_amdgcn_rsqf(vv) * __builtin_amdgcn_rcpf((float)axis_norm));
        amp = c > 0.0f ? __builtin_amdgcn_exp2f((float)(0.5 * param) * __builtin_amdgcn_logf(c)) : 0.0f;
        return dn > 0.0;
    }
    const double c = cos_between(v, axis, axis_norm);
    amp = pattern_amp(kind, param, c);
    return pattern_on(kind, c);
}

// e^{-j 2 pi d / lambda} = e^{-j 2 pi f}, f = frac(d / lambda) taken in FP64
// (d times 1 / lambda: a relative error of a few 1e-16 in turns); cosine and
// sine of the fraction of a turn by the hardware's v_cos/v_sin (their argument
// is in turns).
__device__ __forceinline__ void phase_cs(double d, double inv_lambda, float& cs, float& sn)
{
#pragma clang fp contract(off)
    const double x = d * inv_lambda;
    const float f = (float)(x - floor(x));
    cs = __builtin_amdgcn_cosf(f);
    sn = -__builtin_amdgcn_sinf(f);
}

// Fresnel reflection coefficient (Section II-B, specular reflection) of
// triangle t's material for a wave arriving along d (FP64): TE (pol 1)
//   (c - r) / (c + r), TM (pol 2) (eps c - r) / (eps c + r), r = sqrt(eps - 1 + c^2),
// c = |d . n| / |d| with n the unit normal of e1 x e2 from the FP64 vertices
// (precomputed per triangle) and len = |d| from the caller, eps = eps_r - j
// sigma sig_scale, principal square root (stable form for either sign of
// the real part).
__device__ inline float2 fresnel_coef(const SceneView& s, int t, const double* d, double len, int pol,
                                     double sig_scale)
{
#pragma clang fp contract(off)
    const double* nv = s.nrm + 3 * (int64_t)t;
    const double c = fmin(fabs(d[0] * nv[0] + d[1] * nv[1] + d[2] * nv[2]) / len, 1.0);   // len = |d|
    const float2 m = s.mat[t];
    const double er = (double)m.x, ei = -(double)m.y * sig_scale;
    const double a = er - (1.0 - c * c), b = ei;
    const double h = sqrt(a * a + b * b);
    double rr, ri;
    if (a >= 0.0) {
        rr = sqrt(0.5 * (h + a));
        ri = rr > 0.0 ? b / (2.0 * rr) : 0.0;
    } else {
        const double q = sqrt(0.5 * (h - a));
        rr = fabs(b) / (2.0 * q);
        ri = b < 0.0 ? -q : q;
    }
    double pr, pi, qr, qi;   // numerator p, denominator q
    if (pol == 1) {
        pr = c - rr; pi = -ri;
        qr = c + rr; qi = ri;
    } else {
        pr = er * c - rr; pi = ei * c - ri;
        qr = er * c + rr; qi = ei * c + ri;
    }
    const double iq = 1.0 / (qr * qr + qi * qi);
    return make_float2((float)((pr * qr + pi * qi) * iq), (float)((pi * qr - pr * qi) * iq));
}

// --------------------------------------------------------------------------
// launchers implemented in the .hip files
// --------------------------------------------------------------------------

}  // namespace rt
