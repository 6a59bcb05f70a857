/* Drives every entry point of the oracle's C part on the 5 x 4 x 3 m box
 * room (12 triangles, 6 surfaces) so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can check its memory accesses and arithmetic:
 * discovery from the Tx and from the RIS centre (half-space), candidates of
 * order <= 2 (every sequence without an immediate repeat), paths from the Tx
 * and from the RIS centre, the per-element paths of a 7 x 7 RIS and the small
 * helpers.  Prints a few counts; exits 0 when they are consistent (25 Tx
 * paths per receiver up to order 2: the image lattice of a box). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t or_discover(const float* V, const int32_t* T, int64_t nt, const double src[3], int hemi,
                    const double hemi_n[3], int64_t n, int K, int32_t* hits, uint8_t* launched);
int64_t or_find_paths(const float* V, const int32_t* T, const int32_t* surf, int64_t nt, const double S[3],
                      const int32_t* cands, int64_t nc, int K, const double* rx, int64_t R, int64_t cap,
                      int32_t* out_rx, int32_t* out_cand, double* out_pts, int32_t* out_tri);
void or_ris_paths(const float* V, const int32_t* T, const int32_t* surf, int64_t nt, const double tx[3],
                  const double* elems, int64_t M, const double* rx, int64_t R, const int64_t* uptr,
                  const int32_t* useq, int K, uint8_t* valid, double* pts, int32_t* tri, uint8_t* txm_clear,
                  const uint8_t* lit);
int or_leg_blocked(const float* V, const int32_t* T, const int32_t* surf, int64_t nt, const double A[3],
                   const double B[3], int64_t skip_a, int64_t skip_b);
int or_contains(const float* V, const int32_t* T, int64_t tri, const double p[3]);
void or_fib_dir(int64_t i, int64_t n, double out[3]);
int64_t or_leg_count(void);

#define K 2
#define R 16
#define M 49

int main(void)
{
    /* box [0,5] x [0,4] x [0,3]: 8 corners, each face two triangles */
    const float V[8 * 3] = {0, 0, 0, 5, 0, 0, 5, 4, 0, 0, 4, 0, 0, 0, 3, 5, 0, 3, 5, 4, 3, 0, 4, 3};
    const int32_t T[12 * 3] = {0, 1, 2, 0, 2, 3,   /* z = 0 */
                               4, 6, 5, 4, 7, 6,   /* z = 3 */
                               0, 5, 1, 0, 4, 5,   /* y = 0 */
                               3, 2, 6, 3, 6, 7,   /* y = 4 */
                               0, 3, 7, 0, 7, 4,   /* x = 0 */
                               1, 5, 6, 1, 6, 2};  /* x = 5 */
    const int32_t S[12] = {0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5};
    const int64_t nt = 12;
    const double tx[3] = {1.0, 1.0, 1.5};
    const double u[3] = {4.999, 2.0, 1.5};
    const double nrm[3] = {-1.0, 0.0, 0.0};
    int fails = 0;

    /* discovery */
    const int64_t n = 2000;
    int32_t* hits = malloc(sizeof(int32_t) * 2 * n * K);
    uint8_t* launched = malloc(2 * n);
    int64_t segs = or_discover(V, T, nt, tx, 0, nrm, n, K, hits, launched);
    int64_t segs_u = or_discover(V, T, nt, u, 1, nrm, n, K, hits, launched);
    for (int64_t i = 0; i < n * K; ++i)
        if (hits[i] < -1 || hits[i] >= nt) ++fails;
    printf("discovery segments %lld + %lld\n", (long long)segs, (long long)segs_u);

    /* candidates: empty, 6 of order 1, 30 of order 2 */
    int32_t cands[37 * K];
    int nc = 0;
    cands[nc * K] = -1;
    cands[nc * K + 1] = -1;
    ++nc;
    for (int a = 0; a < 6; ++a) {
        cands[nc * K] = a;
        cands[nc * K + 1] = -1;
        ++nc;
    }
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b)
            if (a != b) {
                cands[nc * K] = a;
                cands[nc * K + 1] = b;
                ++nc;
            }
    double rx[R * 3];
    for (int r = 0; r < R; ++r) {
        rx[3 * r] = 0.5 + 4.0 * r / (R - 1) + 1e-4 * (r % 3);
        rx[3 * r + 1] = 3.3 - 0.6 * r / (R - 1);
        rx[3 * r + 2] = 1.5 + 2e-4 * (r % 5);
    }
    const int64_t cap = 64 * R;
    int32_t* o_rx = malloc(sizeof(int32_t) * cap);
    int32_t* o_c = malloc(sizeof(int32_t) * cap);
    double* o_p = malloc(sizeof(double) * cap * K * 3);
    int32_t* o_t = malloc(sizeof(int32_t) * cap * K);
    int64_t np_tx = or_find_paths(V, T, S, nt, tx, cands, nc, K, rx, R, cap, o_rx, o_c, o_p, o_t);
    if (np_tx != 25 * R) ++fails;
    int64_t tiny = or_find_paths(V, T, S, nt, tx, cands, nc, K, rx, R, 3, o_rx, o_c, o_p, o_t);
    if (tiny != -25 * R) ++fails;   /* capacity too small: minus the count */
    printf("paths from the Tx %lld (expected %d)\n", (long long)np_tx, 25 * R);

    /* sequences valid from the RIS centre, grouped by receiver */
    int64_t np_u = or_find_paths(V, T, S, nt, u, cands, nc, K, rx, R, cap, o_rx, o_c, o_p, o_t);
    int64_t uptr[R + 1] = {0};
    int32_t* useq = malloc(sizeof(int32_t) * (np_u > 0 ? np_u : 1) * K);
    int64_t nu = 0;
    for (int64_t i = 0; i < np_u; ++i) {
        if (o_c[i] == 0) continue;   /* the direct path is slot 0 of every receiver */
        useq[nu * K] = cands[o_c[i] * K];
        useq[nu * K + 1] = cands[o_c[i] * K + 1];
        uptr[o_rx[i] + 1] += 1;
        ++nu;
    }
    for (int r = 0; r < R; ++r) uptr[r + 1] += uptr[r];
    double elems[M * 3];
    const double lam = 299792458.0 / 28e9;
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j) {
            elems[3 * (7 * i + j)] = u[0];
            elems[3 * (7 * i + j) + 1] = u[1] + (i - 3) * lam / 2;
            elems[3 * (7 * i + j) + 2] = u[2] + (j - 3) * lam / 2;
        }
    const int64_t n_slots = nu + R;
    uint8_t* valid = malloc((size_t)(n_slots * M));
    double* pts = malloc(sizeof(double) * n_slots * M * K * 3);
    int32_t* tri = malloc(sizeof(int32_t) * n_slots * M * K);
    uint8_t txm[M];
    uint8_t lit[M];
    for (int m = 0; m < M; ++m) lit[m] = (uint8_t)(m % 2);
    or_ris_paths(V, T, S, nt, tx, elems, M, rx, R, uptr, useq, K, valid, pts, tri, txm, NULL);
    int64_t nv = 0;
    for (int64_t i = 0; i < n_slots * M; ++i) nv += valid[i];
    or_ris_paths(V, T, S, nt, tx, elems, M, rx, R, uptr, useq, K, valid, pts, tri, txm, lit);
    int64_t nv_lit = 0;
    for (int64_t i = 0; i < n_slots * M; ++i) nv_lit += valid[i];
    printf("centre sequences %lld, element paths %lld (%lld with half the elements lit)\n", (long long)nu,
           (long long)nv, (long long)nv_lit);
    /* every element of a convex room sees at least its direct path to every receiver,
       and at most the slots' sequences; lighting half the elements removes paths */
    if (nv < (int64_t)M * R || nv > n_slots * M || !(nv_lit < nv)) ++fails;

    /* helpers */
    const double a[3] = {1.0, 1.0, 1.0}, b[3] = {4.0, 3.0, 2.0}, out[3] = {6.0, 2.0, 1.0};
    if (or_leg_blocked(V, T, S, nt, a, b, -1, -1) != 0) ++fails;
    if (or_leg_blocked(V, T, S, nt, a, out, -1, -1) != 1) ++fails;
    const double on_floor[3] = {2.0, 1.0, 0.0};
    if (or_contains(V, T, 0, on_floor) + or_contains(V, T, 1, on_floor) != 1) ++fails;
    double d[3];
    or_fib_dir(7, 100, d);
    printf("legs %lld\n", (long long)or_leg_count());
    free(hits);
    free(launched);
    free(o_rx);
    free(o_c);
    free(o_p);
    free(o_t);
    free(useq);
    free(valid);
    free(pts);
    free(tri);
    printf(fails ? "FAIL %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
