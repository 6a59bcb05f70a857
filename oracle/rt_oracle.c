/*
 * Oracle for the RIS ray tracer: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, brute-force CPU implementation of the geometric part of the
 * method of "Ray Tracing Algorithm for Reconfigurable Intelligent Surfaces"
 * (arXiv 2402.13034).  It is used by the tests, by the smoke check and by the
 * CPU baseline leg of the benchmark, never by the product path.  It shares no
 * code with the GPU library.
 *
 * What it computes (field evaluation lives in oracle.py, in FP64 NumPy):
 *   - discovery rays from a source, closest hit over every triangle, specular
 *     bounces (stand-in for the analytic first stage of the hybrid tracer,
 *     Section II);
 *   - the image method between a source and a receiver for a given sequence
 *     of triangles (Section II-B; sources are the Tx, the RIS centre and each
 *     RIS element);
 *   - visibility of every leg of a path by ray launch (the second stage of the
 *     hybrid tracer, Section II, and the relaunch of Section IV-A).
 *
 * Precision readings (the paper names none):
 *   - decisions that pick triangle IDs by ray launch (closest hit, occlusion)
 *     are taken in FP32, the precision of the GPU kernels, with one fixed
 *     formula (Moller-Trumbore, left-to-right sums, no fused multiply-add,
 *     one correctly rounded division);
 *   - image method, containment and side tests, lengths: FP64, no fused
 *     multiply-add.
 * Compile with -ffp-contract=off and without -ffast-math.
 *
 * Built with -DOR_FP64_DECISIONS the same ray decisions are taken in FP64
 * instead (origin and direction not rounded to FP32): not the reading the
 * parity tests use, but the reference that measures how many decisions the
 * FP32 reading moves (hit lists, blocked legs, rays that escape a closed
 * room).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EPS 1e-4 /* metres: legs ignore hits within EPS of their ends */

#ifdef OR_FP64_DECISIONS
typedef double rfloat; /* precision of the ray decisions */
#else
typedef float rfloat;
#endif

static int64_t g_leg_count = 0; /* legs tested since the last or_leg_count() */

/* Number of visibility legs tested since the last call (for timing reports). */
/* threads an OpenMP loop of the oracle uses (reported with timings) */
int or_threads(void) { return omp_get_max_threads(); }

int64_t or_leg_count(void)
{
    int64_t n;
#pragma omp atomic capture
    { n = g_leg_count; g_leg_count = 0; }
    return n;
}

/* ----------------------------------------------------------------------- */
/* Ray / triangle test (FP32, or FP64 with OR_FP64_DECISIONS)              */
/* ----------------------------------------------------------------------- */
typedef struct {
    rfloat v0[3], e1[3], e2[3];
} tri32;

static void make_tri32(const float* V, const int32_t* T, int64_t i, tri32* t)
{
    const float* a = V + 3 * (int64_t)T[3 * i + 0];
    const float* b = V + 3 * (int64_t)T[3 * i + 1];
    const float* c = V + 3 * (int64_t)T[3 * i + 2];
    for (int k = 0; k < 3; ++k) {
        t->v0[k] = a[k];
        t->e1[k] = (rfloat)b[k] - (rfloat)a[k];
        t->e2[k] = (rfloat)c[k] - (rfloat)a[k];
    }
}

/* Moller-Trumbore, two-sided.  Returns 1 and the parameter t if the ray
 * o + t d meets the closed triangle with tmin < t < tmax. */
static int hit32(const rfloat o[3], const rfloat d[3], const tri32* tr, rfloat tmin, rfloat tmax,
                 rfloat* t_out)
{
    const rfloat* e1 = tr->e1;
    const rfloat* e2 = tr->e2;
    rfloat px = d[1] * e2[2] - d[2] * e2[1];
    rfloat py = d[2] * e2[0] - d[0] * e2[2];
    rfloat pz = d[0] * e2[1] - d[1] * e2[0];
    rfloat det = e1[0] * px + e1[1] * py + e1[2] * pz;
    if (det == (rfloat)0) return 0;
    rfloat inv = (rfloat)1 / det;
    rfloat sx = o[0] - tr->v0[0];
    rfloat sy = o[1] - tr->v0[1];
    rfloat sz = o[2] - tr->v0[2];
    rfloat u = (sx * px + sy * py + sz * pz) * inv;
    if (!(u >= (rfloat)0 && u <= (rfloat)1)) return 0;
    rfloat qx = sy * e1[2] - sz * e1[1];
    rfloat qy = sz * e1[0] - sx * e1[2];
    rfloat qz = sx * e1[1] - sy * e1[0];
    rfloat v = (d[0] * qx + d[1] * qy + d[2] * qz) * inv;
    if (!(v >= (rfloat)0 && u + v <= (rfloat)1)) return 0;
    rfloat t = (e2[0] * qx + e2[1] * qy + e2[2] * qz) * inv;
    if (!(t > tmin && t < tmax)) return 0;
    *t_out = t;
    return 1;
}

/* Closest hit over all triangles except `skip`; ties in t go to the lowest
 * triangle index. Returns -1 on a miss. */
static int64_t closest32(const tri32* tris, int64_t nt, const rfloat o[3], const rfloat d[3],
                         rfloat tmin, int64_t skip, rfloat* t_best)
{
    int64_t best = -1;
    rfloat bt = INFINITY;
    for (int64_t i = 0; i < nt; ++i) {
        if (i == skip) continue;
        rfloat t;
        if (hit32(o, d, &tris[i], tmin, INFINITY, &t)) {
            if (t < bt) {
                bt = t;
                best = i;
            }
        }
    }
    *t_best = bt;
    return best;
}

/* Specular reflection of d off the plane of triangle tr:
 * n = e1 x e2 (not normalised), d' = d - (2 (d.n) / (n.n)) n. */
static void reflect32(const tri32* tr, const rfloat d[3], rfloat out[3])
{
    const rfloat* e1 = tr->e1;
    const rfloat* e2 = tr->e2;
    rfloat nx = e1[1] * e2[2] - e1[2] * e2[1];
    rfloat ny = e1[2] * e2[0] - e1[0] * e2[2];
    rfloat nz = e1[0] * e2[1] - e1[1] * e2[0];
    rfloat dn = d[0] * nx + d[1] * ny + d[2] * nz;
    rfloat nn = nx * nx + ny * ny + nz * nz;
    rfloat k = ((rfloat)2 * dn) / nn;
    out[0] = d[0] - k * nx;
    out[1] = d[1] - k * ny;
    out[2] = d[2] - k * nz;
}

static tri32* build_tris(const float* V, const int32_t* T, int64_t nt)
{
    tri32* tris = (tri32*)malloc(sizeof(tri32) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t i = 0; i < nt; ++i) make_tri32(V, T, i, &tris[i]);
    return tris;
}

/* ----------------------------------------------------------------------- */
/* Optional acceleration for large scenes: a median-split BVH               */
/* ----------------------------------------------------------------------- */
/* A binary tree of its own (split at the median centroid along the longest
 * axis of the centroid bounds, up to 4 triangles per leaf; unlike the
 * library's Morton-ordered LBVH), with FP64 boxes grown by 1e-4 m + 1e-5 |x|
 * so that no triangle the FP32 test would hit is ever pruned.  Closest hit
 * keeps the lowest (t, index) and any-hit stops at a hit: the results are
 * those of the brute-force loops, in any traversal order.  Switched on with
 * or_set_accel(1); built once per scene (recognised by a hash of its
 * triangles) before the parallel loops that use it. */
typedef struct {
    double lo[3], hi[3];
    int64_t left, right; /* children (internal node) */
    int64_t first, count; /* triangle range in g_idx (leaf: count > 0) */
} bvh_node;

static int g_accel = 0;
static bvh_node* g_nodes = NULL;
static int64_t* g_idx = NULL;
static int64_t g_nt = -1;
static uint64_t g_hash = 0;

void or_set_accel(int on) { g_accel = on; }

static uint64_t tris_hash(const tri32* tris, int64_t nt)
{
    uint64_t h = 1469598103934665603ull; /* FNV-1a over the triangles' bytes */
    const unsigned char* p = (const unsigned char*)tris;
    size_t nb = sizeof(tri32) * (size_t)nt;
    for (size_t i = 0; i < nb; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

static double* g_cent = NULL; /* centroids while building */
static int g_axis = 0;
static int cmp_cent(const void* a, const void* b)
{
    double ca = g_cent[3 * *(const int64_t*)a + g_axis], cb = g_cent[3 * *(const int64_t*)b + g_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    int64_t ia = *(const int64_t*)a, ib = *(const int64_t*)b;
    return (ia > ib) - (ia < ib);
}

static void tri_bounds(const tri32* t, double lo[3], double hi[3])
{
    for (int k = 0; k < 3; ++k) {
        double a = (double)t->v0[k], b = a + (double)t->e1[k], c = a + (double)t->e2[k];
        lo[k] = fmin(a, fmin(b, c));
        hi[k] = fmax(a, fmax(b, c));
    }
}

static void bvh_build(const tri32* tris, int64_t nt)
{
    uint64_t h = tris_hash(tris, nt);
    if (g_nodes && g_nt == nt && g_hash == h) return;
    free(g_nodes);
    free(g_idx);
    g_nodes = (bvh_node*)malloc(sizeof(bvh_node) * (size_t)(2 * nt + 1));
    g_idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    g_cent = (double*)malloc(sizeof(double) * 3 * (size_t)(nt > 0 ? nt : 1));
    for (int64_t i = 0; i < nt; ++i) {
        double lo[3], hi[3];
        tri_bounds(&tris[i], lo, hi);
        for (int k = 0; k < 3; ++k) g_cent[3 * i + k] = 0.5 * (lo[k] + hi[k]);
        g_idx[i] = i;
    }
    int64_t n_nodes = 1;
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * 256);
    int sp = 0;
    g_nodes[0].first = 0;
    g_nodes[0].count = nt;
    stack[sp++] = 0;
    while (sp > 0) {
        int64_t ni = stack[--sp];
        bvh_node* nd = &g_nodes[ni];
        int64_t f = nd->first, c = nd->count;
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < 3; ++k) {
            nd->lo[k] = INFINITY;
            nd->hi[k] = -INFINITY;
        }
        for (int64_t j = f; j < f + c; ++j) {
            double lo[3], hi[3];
            tri_bounds(&tris[g_idx[j]], lo, hi);
            for (int k = 0; k < 3; ++k) {
                nd->lo[k] = fmin(nd->lo[k], lo[k]);
                nd->hi[k] = fmax(nd->hi[k], hi[k]);
                clo[k] = fmin(clo[k], g_cent[3 * g_idx[j] + k]);
                chi[k] = fmax(chi[k], g_cent[3 * g_idx[j] + k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            double m = 1e-4 + 1e-5 * fmax(fabs(nd->lo[k]), fabs(nd->hi[k]));
            nd->lo[k] -= m;
            nd->hi[k] += m;
        }
        if (c <= 4) {
            nd->left = nd->right = -1;
            continue;
        }
        int ax = 0;
        for (int k = 1; k < 3; ++k)
            if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
        g_axis = ax;
        qsort(g_idx + f, (size_t)c, sizeof(int64_t), cmp_cent);
        int64_t half = c / 2;
        int64_t l = n_nodes++, r = n_nodes++;
        nd = &g_nodes[ni];
        nd->left = l;
        nd->right = r;
        g_nodes[l].first = f;
        g_nodes[l].count = half;
        g_nodes[r].first = f + half;
        g_nodes[r].count = c - half;
        nd->count = 0;
        if (sp + 2 > 256) abort(); /* depth of a median split stays near log2(n) */
        stack[sp++] = l;
        stack[sp++] = r;
    }
    free(stack);
    free(g_cent);
    g_cent = NULL;
    g_nt = nt;
    g_hash = h;
}

/* entry distance of the ray into the node's box, or -1 if it misses it in [0, tmax] */
static double box_entry(const bvh_node* nd, const double o[3], const double inv[3], double tmax)
{
    double t0 = 0.0, t1 = tmax;
    for (int k = 0; k < 3; ++k) {
        double a = (nd->lo[k] - o[k]) * inv[k], b = (nd->hi[k] - o[k]) * inv[k];
        if (a > b) {
            double x = a;
            a = b;
            b = x;
        }
        if (a != a) a = -INFINITY; /* 0 * inf: the ray runs inside the slab's plane */
        if (b != b) b = INFINITY;
        t0 = fmax(t0, a);
        t1 = fmin(t1, b);
    }
    return t0 <= t1 ? t0 : -1.0;
}

/* Closest hit with the BVH; same result as closest32. */
static int64_t closest_bvh(const tri32* tris, const rfloat o[3], const rfloat d[3], rfloat tmin, int64_t skip,
                           rfloat* t_best)
{
    int64_t best = -1;
    rfloat bt = INFINITY;
    double od[3] = {(double)o[0], (double)o[1], (double)o[2]};
    double inv[3];
    double dn = sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]);
    for (int k = 0; k < 3; ++k) inv[k] = 1.0 / (double)d[k];
    int64_t stack[256];
    double entry[256];
    int sp = 0;
    stack[sp] = 0;
    entry[sp++] = box_entry(&g_nodes[0], od, inv, INFINITY);
    while (sp > 0) {
        --sp;
        const bvh_node* nd = &g_nodes[stack[sp]];
        /* boxes entered beyond the best hit so far (plus a slack far above the rounding) hold no closer one */
        double lim = bt < INFINITY ? (double)bt + 1e-3 / (dn > 0 ? dn : 1.0) : INFINITY;
        if (entry[sp] < 0.0 || entry[sp] > lim) continue;
        if (nd->count > 0) {
            for (int64_t j = nd->first; j < nd->first + nd->count; ++j) {
                int64_t i = g_idx[j];
                if (i == skip) continue;
                rfloat t;
                if (hit32(o, d, &tris[i], tmin, INFINITY, &t))
                    if (t < bt || (t == bt && i < best)) {
                        bt = t;
                        best = i;
                    }
            }
        } else {
            /* the nearer child is popped first */
            double el = box_entry(&g_nodes[nd->left], od, inv, lim), er = box_entry(&g_nodes[nd->right], od, inv, lim);
            int64_t nl = nd->left, nr = nd->right;
            if (el >= 0.0 && er >= 0.0 && er < el) {
                double x = el;
                el = er;
                er = x;
                int64_t y = nl;
                nl = nr;
                nr = y;
            }
            if (er >= 0.0) {
                stack[sp] = nr;
                entry[sp++] = er;
            }
            if (el >= 0.0) {
                stack[sp] = nl;
                entry[sp++] = el;
            }
        }
    }
    *t_best = bt;
    return best;
}

/* Any hit with the BVH, skipping two surfaces; same result as the brute loop. */
static int any_bvh(const tri32* tris, const int32_t* surf, const rfloat o[3], const rfloat d[3], rfloat tmin,
                   rfloat tmax, int64_t skip_a, int64_t skip_b)
{
    double od[3] = {(double)o[0], (double)o[1], (double)o[2]};
    double inv[3];
    double dn = sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]);
    for (int k = 0; k < 3; ++k) inv[k] = 1.0 / (double)d[k];
    double lim = (double)tmax + 1e-3 / (dn > 0 ? dn : 1.0);
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bvh_node* nd = &g_nodes[stack[--sp]];
        if (box_entry(nd, od, inv, lim) < 0.0) continue;
        if (nd->count > 0) {
            for (int64_t j = nd->first; j < nd->first + nd->count; ++j) {
                int64_t i = g_idx[j];
                if (surf[i] == skip_a || surf[i] == skip_b) continue;
                rfloat t;
                if (hit32(o, d, &tris[i], tmin, tmax, &t)) return 1;
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    return 0;
}

/* ----------------------------------------------------------------------- */
/* Discovery                                                                */
/* ----------------------------------------------------------------------- */
/* Spherical Fibonacci point i of n (FP64):
 *   z = 1 - (2 i + 1) / n,  phi = 2 pi frac(i (sqrt 5 - 1) / 2). */
void or_fib_dir(int64_t i, int64_t n, double out[3])
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

/*
 * Shoot discovery rays from `src` and record up to K closest-hit triangle IDs
 * per ray (-1 after the first miss).
 *   hemi == 0: n rays on the full sphere; rows = n.
 *   hemi != 0: a 2n-point sphere, of which only the directions with
 *              d . hemi_n > 0 (FP64) are launched; rows = 2n, rows of rays
 *              not launched are all -1 and `launched` is 0 for them.
 * Each bounce starts at the FP32 hit point, ignores the triangle just hit and
 * hits with t <= EPS.  Returns the number of segments traced.
 */
int64_t or_discover(const float* V, const int32_t* T, int64_t nt, const double src[3], int hemi,
                    const double hemi_n[3], int64_t n, int K, int32_t* hits, uint8_t* launched)
{
    tri32* tris = build_tris(V, T, nt);
    const int accel = g_accel && nt > 0;
    if (accel) bvh_build(tris, nt);
    int64_t rows = hemi ? 2 * n : n;
    int64_t segs = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : segs)
    for (int64_t i = 0; i < rows; ++i) {
        double d64[3];
        or_fib_dir(i, rows, d64);
        for (int b = 0; b < K; ++b) hits[i * K + b] = -1;
        int go = 1;
        if (hemi) go = (d64[0] * hemi_n[0] + d64[1] * hemi_n[1] + d64[2] * hemi_n[2]) > 0.0;
        launched[i] = (uint8_t)go;
        if (!go) continue;
        rfloat o[3] = {(rfloat)src[0], (rfloat)src[1], (rfloat)src[2]};
        rfloat d[3] = {(rfloat)d64[0], (rfloat)d64[1], (rfloat)d64[2]};
        int64_t skip = -1;
        for (int b = 0; b < K; ++b) {
            rfloat t;
            segs += 1;
            int64_t h = accel ? closest_bvh(tris, o, d, (rfloat)OR_EPS, skip, &t)
                              : closest32(tris, nt, o, d, (rfloat)OR_EPS, skip, &t);
            if (h < 0) break;
            hits[i * K + b] = (int32_t)h;
            rfloat p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            rfloat r[3];
            reflect32(&tris[h], d, r);
            o[0] = p[0]; o[1] = p[1]; o[2] = p[2];
            d[0] = r[0]; d[1] = r[1]; d[2] = r[2];
            skip = h;
        }
    }
    free(tris);
    return segs;
}

/* ----------------------------------------------------------------------- */
/* Visibility of a leg (FP32 decision, or FP64 with OR_FP64_DECISIONS)     */
/* ----------------------------------------------------------------------- */
/* The leg A -> B (FP64 end points) is blocked if some triangle that is not
 * part of surface skip_a or skip_b (the surfaces its end points lie on, -1 for
 * none) is met at EPS < t < L - EPS by the FP32 ray with origin fl(A) and
 * direction fl((B - A) x (1 / L)) (one correctly rounded division, three
 * products). */
static int leg_blocked(const tri32* tris, const int32_t* surf, int64_t nt, const double A[3],
                       const double B[3], int64_t skip_a, int64_t skip_b)
{
    double w0 = B[0] - A[0], w1 = B[1] - A[1], w2 = B[2] - A[2];
    double L = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    rfloat o[3] = {(rfloat)A[0], (rfloat)A[1], (rfloat)A[2]};
    double il = 1.0 / L;
    rfloat d[3] = {(rfloat)(w0 * il), (rfloat)(w1 * il), (rfloat)(w2 * il)};
    rfloat tmin = (rfloat)OR_EPS;
    rfloat tmax = (rfloat)(L - OR_EPS);
#pragma omp atomic
    g_leg_count += 1;
    if (!(tmax > tmin)) return 0;
    if (g_accel && nt > 0) return any_bvh(tris, surf, o, d, tmin, tmax, skip_a, skip_b);
    for (int64_t i = 0; i < nt; ++i) {
        if (surf[i] == skip_a || surf[i] == skip_b) continue;
        rfloat t;
        if (hit32(o, d, &tris[i], tmin, tmax, &t)) return 1;
    }
    return 0;
}

int or_leg_blocked(const float* V, const int32_t* T, const int32_t* surf, int64_t nt,
                   const double A[3], const double B[3], int64_t skip_a, int64_t skip_b)
{
    tri32* tris = build_tris(V, T, nt);
    if (g_accel && nt > 0) bvh_build(tris, nt);
    int r = leg_blocked(tris, surf, nt, A, B, skip_a, skip_b);
    free(tris);
    return r;
}

/* ----------------------------------------------------------------------- */
/* Image method (FP64)                                                      */
/* ----------------------------------------------------------------------- */
typedef struct {
    double v[3][3]; /* vertices */
    double n[3];    /* (v1 - v0) x (v2 - v0) */
    double c;       /* n . v0 */
} tri64;

static void make_tri64(const float* V, const int32_t* T, int64_t i, tri64* t)
{
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) t->v[j][k] = (double)V[3 * (int64_t)T[3 * i + j] + k];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = t->v[1][k] - t->v[0][k];
        e2[k] = t->v[2][k] - t->v[0][k];
    }
    t->n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    t->n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    t->n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    t->c = t->n[0] * t->v[0][0] + t->n[1] * t->v[0][1] + t->n[2] * t->v[0][2];
}

static double plane_side(const tri64* t, const double p[3])
{
    return (t->n[0] * p[0] + t->n[1] * p[1] + t->n[2] * p[2]) - t->c;
}

static double edge_raw(const double s[2], const double e[2], const double p[2])
{
    return (e[0] - s[0]) * (p[1] - s[1]) - (e[1] - s[1]) * (p[0] - s[0]);
}

/* Edge function of the directed edge s -> e at p, evaluated from the
 * lexicographically smaller end point so that the two directions of one edge
 * give exactly opposite values (an edge shared by two triangles then splits
 * the plane identically for both). */
static double edge2(const double s[2], const double e[2], const double p[2])
{
    int s_first = (s[0] < e[0]) || (s[0] == e[0] && s[1] < e[1]);
    return s_first ? edge_raw(s, e, p) : -edge_raw(e, s, p);
}

/* Top-left ownership of a directed edge of a counter-clockwise triangle. */
static int top_left(const double s[2], const double e[2])
{
    double dy = e[1] - s[1];
    double dx = e[0] - s[0];
    return (dy < 0.0) || (dy == 0.0 && dx < 0.0);
}

/* Is p (assumed on the plane) inside the triangle?  Projection drops the
 * axis of largest |n| (lowest axis on ties); the projected triangle is made
 * counter-clockwise; a point on an edge belongs to the triangle only if that
 * edge is top-left, so a point on an edge shared by two coplanar triangles
 * belongs to exactly one of them. */
static int contains64(const tri64* t, const double p[3])
{
    double ax = fabs(t->n[0]), ay = fabs(t->n[1]), az = fabs(t->n[2]);
    int drop = 0;
    if (ay > ax && ay >= az) drop = 1;
    else if (az > ax && az > ay) drop = 2;
    int i0 = (drop + 1) % 3, i1 = (drop + 2) % 3;
    double a[2] = {t->v[0][i0], t->v[0][i1]};
    double b[2] = {t->v[1][i0], t->v[1][i1]};
    double c[2] = {t->v[2][i0], t->v[2][i1]};
    double q[2] = {p[i0], p[i1]};
    double area = edge2(a, b, c);
    if (area == 0.0) return 0;
    if (area < 0.0) {
        double tmp0 = b[0], tmp1 = b[1];
        b[0] = c[0]; b[1] = c[1];
        c[0] = tmp0; c[1] = tmp1;
    }
    double w0 = edge2(b, c, q);
    double w1 = edge2(c, a, q);
    double w2 = edge2(a, b, q);
    int in0 = (w0 > 0.0) || (w0 == 0.0 && top_left(b, c));
    int in1 = (w1 > 0.0) || (w1 == 0.0 && top_left(c, a));
    int in2 = (w2 > 0.0) || (w2 == 0.0 && top_left(a, b));
    return in0 && in1 && in2;
}

int or_contains(const float* V, const int32_t* T, int64_t tri, const double p[3])
{
    tri64 t;
    make_tri64(V, T, tri, &t);
    return contains64(&t, p);
}

/* Surfaces: planar sets of coplanar triangles (a wall, a face of a box).
 * surf[i] is the surface of triangle i; a surface's plane is that of its
 * lowest-numbered triangle. */
typedef struct {
    int64_t n;       /* number of surfaces */
    int64_t* ptr;    /* n + 1 */
    int64_t* tris;   /* triangle indices, grouped by surface, ascending */
} surf_table;

static void build_surfaces(const int32_t* surf, int64_t nt, surf_table* st)
{
    int64_t n = 0;
    for (int64_t i = 0; i < nt; ++i)
        if (surf[i] + 1 > n) n = surf[i] + 1;
    st->n = n;
    st->ptr = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    st->tris = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t i = 0; i < nt; ++i) st->ptr[surf[i] + 1] += 1;
    for (int64_t s = 0; s < n; ++s) st->ptr[s + 1] += st->ptr[s];
    int64_t* fill = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int64_t i = 0; i < nt; ++i) {
        int64_t s = surf[i];
        st->tris[st->ptr[s] + fill[s]] = i;
        fill[s] += 1;
    }
    free(fill);
}

static void free_surfaces(surf_table* st)
{
    free(st->ptr);
    free(st->tris);
}

/* Which triangle of surface s contains p (-1 if none). */
static int64_t surface_contains(const tri64* t64, const surf_table* st, int64_t s, const double p[3])
{
    for (int64_t j = st->ptr[s]; j < st->ptr[s + 1]; ++j)
        if (contains64(&t64[st->tris[j]], p)) return st->tris[j];
    return -1;
}

/* Image method for source S, receiver X and surfaces seq[0..k-1].
 * Images: I_0 = S, I_i = mirror of I_{i-1} in plane i.  Back-trace from X:
 * P_i = (segment I_i -> P_{i+1}) meets plane i at parameter s in (0, 1) and
 * lies inside surface i.  Then each P_i must have its neighbours (P_{i-1}
 * or S, P_{i+1} or X) strictly on the same side of plane i.
 * Returns 1, the points and the triangles that contain them on success. */
static int image_path(const tri64* t64, const surf_table* st, const int32_t* seq, int k,
                      const double S[3], const double X[3], double P[][3], int64_t* tri_of)
{
    double I[8][3];
    I[0][0] = S[0]; I[0][1] = S[1]; I[0][2] = S[2];
    for (int i = 1; i <= k; ++i) {
        const tri64* t = &t64[st->tris[st->ptr[seq[i - 1]]]];
        double nn = t->n[0] * t->n[0] + t->n[1] * t->n[1] + t->n[2] * t->n[2];
        double f = 2.0 * plane_side(t, I[i - 1]) / nn;
        for (int c = 0; c < 3; ++c) I[i][c] = I[i - 1][c] - f * t->n[c];
    }
    double Q[3] = {X[0], X[1], X[2]};
    for (int i = k; i >= 1; --i) {
        const tri64* t = &t64[st->tris[st->ptr[seq[i - 1]]]];
        double w[3] = {Q[0] - I[i][0], Q[1] - I[i][1], Q[2] - I[i][2]};
        double den = t->n[0] * w[0] + t->n[1] * w[1] + t->n[2] * w[2];
        if (den == 0.0) return 0;
        double s = (t->c - (t->n[0] * I[i][0] + t->n[1] * I[i][1] + t->n[2] * I[i][2])) / den;
        if (!(s > 0.0 && s < 1.0)) return 0;
        double p[3] = {I[i][0] + s * w[0], I[i][1] + s * w[1], I[i][2] + s * w[2]};
        int64_t tri = surface_contains(t64, st, seq[i - 1], p);
        if (tri < 0) return 0;
        tri_of[i - 1] = tri;
        P[i - 1][0] = p[0]; P[i - 1][1] = p[1]; P[i - 1][2] = p[2];
        Q[0] = p[0]; Q[1] = p[1]; Q[2] = p[2];
    }
    for (int i = 0; i < k; ++i) {
        const tri64* t = &t64[st->tris[st->ptr[seq[i]]]];
        const double* prev = (i == 0) ? S : P[i - 1];
        const double* next = (i == k - 1) ? X : P[i + 1];
        double a = plane_side(t, prev);
        double b = plane_side(t, next);
        if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0;
    }
    return 1;
}

/* All legs of a path S -> P_0 .. P_{k-1} -> X unblocked?  A leg ignores the
 * surfaces its end points lie on. */
static int path_clear(const tri32* tris, const int32_t* surf, int64_t nt, const int32_t* seq, int k,
                      const double S[3], const double X[3], double P[][3])
{
    for (int j = 0; j <= k; ++j) {
        const double* A = (j == 0) ? S : P[j - 1];
        const double* B = (j == k) ? X : P[j];
        int64_t sa = (j == 0) ? -1 : seq[j - 1];
        int64_t sb = (j == k) ? -1 : seq[j];
        if (leg_blocked(tris, surf, nt, A, B, sa, sb)) return 0;
    }
    return 1;
}

static int seq_len(const int32_t* row, int K)
{
    int k = 0;
    while (k < K && row[k] >= 0) ++k;
    return k;
}

/*
 * Paths from one source S to every receiver for every candidate sequence.
 *   cands: nc x K surface IDs, -1 padded (an all -1 row is the direct path).
 * For every (rx, cand) pair whose image-method geometry holds and whose legs
 * are all unblocked, writes (rx, cand), the K reflection points and the K
 * triangles containing them into the outputs (rx-major, then candidate
 * order).  Returns the number of paths, or -(needed) if cap is too small.
 */
int64_t or_find_paths(const float* V, const int32_t* T, const int32_t* surf, int64_t nt,
                      const double S[3], const int32_t* cands, int64_t nc, int K, const double* rx,
                      int64_t R, int64_t cap, int32_t* out_rx, int32_t* out_cand, double* out_pts,
                      int32_t* out_tri)
{
    tri32* t32 = build_tris(V, T, nt);
    if (g_accel && nt > 0) bvh_build(t32, nt);
    tri64* t64 = (tri64*)malloc(sizeof(tri64) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t i = 0; i < nt; ++i) make_tri64(V, T, i, &t64[i]);
    surf_table st;
    build_surfaces(surf, nt, &st);
    int64_t cells = R * nc;
    uint8_t* ok = (uint8_t*)calloc((size_t)(cells > 0 ? cells : 1), 1);
    double* pts = (double*)calloc((size_t)(cells * K * 3 > 0 ? cells * K * 3 : 1), sizeof(double));
    int32_t* trs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cells * K > 0 ? cells * K : 1));
    /* every (rx, cand) cell on its own: the threads share all cells, not only receivers */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t cell = 0; cell < cells; ++cell) {
        const int64_t r = cell / nc, c = cell - r * nc;
        const int32_t* seq = cands + c * K;
        int k = seq_len(seq, K);
        double P[8][3];
        int64_t tri_of[8];
        for (int j = 0; j < K; ++j) trs[cell * K + j] = -1;
        if (!image_path(t64, &st, seq, k, S, rx + 3 * r, P, tri_of)) continue;
        if (!path_clear(t32, surf, nt, seq, k, S, rx + 3 * r, P)) continue;
        ok[cell] = 1;
        for (int j = 0; j < k; ++j) {
            trs[cell * K + j] = (int32_t)tri_of[j];
            for (int q = 0; q < 3; ++q) pts[(cell * K + j) * 3 + q] = P[j][q];
        }
    }
    int64_t n = 0;
    for (int64_t r = 0; r < R; ++r)
        for (int64_t c = 0; c < nc; ++c) {
            if (!ok[r * nc + c]) continue;
            if (n < cap) {
                out_rx[n] = (int32_t)r;
                out_cand[n] = (int32_t)c;
                for (int j = 0; j < K * 3; ++j) out_pts[n * K * 3 + j] = pts[(r * nc + c) * K * 3 + j];
                for (int j = 0; j < K; ++j) out_tri[n * K + j] = trs[(r * nc + c) * K + j];
            }
            ++n;
        }
    free(ok);
    free(pts);
    free(trs);
    free(t32);
    free(t64);
    free_surfaces(&st);
    return n <= cap ? n : -n;
}

/*
 * RIS element paths (Section II-B: sequences found between the RIS centre
 * and the Rx are re-run through the image method for every element; every
 * leg is re-checked as in the relaunch of Section IV-A).
 *   elems: M x 3 element centres.  tx: transmitter.  rx: R x 3.
 *   Sequences valid from the RIS centre to receiver r are the rows
 *   useq[uptr[r] .. uptr[r+1]) (each K wide, -1 padded, order >= 1).
 * Slot layout: receiver r owns slots uptr[r] + r .. uptr[r+1] + r; its first
 * slot is the direct element -> Rx path, the others follow its sequences.
 * For every slot and element:
 *   valid[slot * M + m] = 1 if Tx -> m is unblocked and the image method from
 *   m through the slot's sequence holds with all legs unblocked;
 *   pts[((slot * M + m) * K + j) * 3 + q] = reflection points;
 *   tri[(slot * M + m) * K + j] = triangles containing them.
 * txm_clear[m] reports the Tx -> element leg.
 */
/* lit: NULL, or per element whether any field reaches it (the incoming paths
 * of Section II-B's supporting reflections); NULL means the direct leg
 * Tx -> m alone decides. */
void or_ris_paths(const float* V, const int32_t* T, const int32_t* surf, int64_t nt,
                  const double tx[3], const double* elems, int64_t M, const double* rx, int64_t R,
                  const int64_t* uptr, const int32_t* useq, int K, uint8_t* valid, double* pts,
                  int32_t* tri, uint8_t* txm_clear, const uint8_t* lit)
{
    tri32* t32 = build_tris(V, T, nt);
    if (g_accel && nt > 0) bvh_build(t32, nt);
    tri64* t64 = (tri64*)malloc(sizeof(tri64) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t i = 0; i < nt; ++i) make_tri64(V, T, i, &t64[i]);
    surf_table st;
    build_surfaces(surf, nt, &st);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m)
        txm_clear[m] = (uint8_t)!leg_blocked(t32, surf, nt, tx, elems + 3 * m, -1, -1);
    /* receiver of every slot (receiver r owns slots uptr[r] + r .. uptr[r + 1] + r) */
    const int64_t n_slots = R > 0 ? uptr[R] + R : 0;
    int64_t* slot_rx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
    for (int64_t r = 0; r < R; ++r)
        for (int64_t slot = uptr[r] + r; slot <= uptr[r + 1] + r; ++slot) slot_rx[slot] = r;
    /* every (slot, element) cell on its own: the threads share all cells, not only receivers */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t cell = 0; cell < n_slots * M; ++cell) {
        const int64_t slot = cell / M, m = cell - slot * M;
        const int64_t r = slot_rx[slot], s = slot - (uptr[r] + r);
        int32_t empty[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
        const int32_t* seq = (s == 0) ? empty : useq + (uptr[r] + s - 1) * K;
        int k = (s == 0) ? 0 : seq_len(seq, K);
        double P[8][3];
        int64_t tri_of[8];
        for (int j = 0; j < K * 3; ++j) pts[cell * K * 3 + j] = 0.0;
        for (int j = 0; j < K; ++j) tri[cell * K + j] = -1;
        int ok = lit ? lit[m] : txm_clear[m];
        if (ok) ok = image_path(t64, &st, seq, k, elems + 3 * m, rx + 3 * r, P, tri_of);
        if (ok) ok = path_clear(t32, surf, nt, seq, k, elems + 3 * m, rx + 3 * r, P);
        valid[cell] = (uint8_t)ok;
        if (ok)
            for (int j = 0; j < k; ++j) {
                tri[cell * K + j] = (int32_t)tri_of[j];
                for (int q = 0; q < 3; ++q) pts[(cell * K + j) * 3 + q] = P[j][q];
            }
    }
    free(slot_rx);
    free(t32);
    free(t64);
    free_surfaces(&st);
}
