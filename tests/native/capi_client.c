/* A client of the risrt C ABI in plain C99: no HIP, no Python.  It reads a
 * problem from a binary file, builds the scene and the RIS, traces, and
 * writes the channel (E_env, H) with two trace counts to another file.
 *
 * Input, little-endian: int64 n_vtx, n_tri, M, R, n_rays, max_order; float32
 * vertices [n_vtx][3]; int32 triangles [n_tri][3]; int32 surfaces [n_tri];
 * float32 reflection coefficients, real [n_tri] then imaginary [n_tri];
 * float64 element centres [M][3]; float64 RIS centre[3], normal[3], d_y, d_z,
 * element gain, pattern q; float64 Tx position[3], axis[3], power, gain,
 * pattern kind, parameter; float64 Rx axis[3], gain, pattern kind,
 * parameter; float64 frequency; float64 receivers [R][3].
 * Output: int64 R, M, segments, environment paths; float32 E_env [R][2];
 * float32 H [R][M][2].  Exit status 0, or 1 with the library's message. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "risrt.h"

static FILE* in;

static void* take(size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p || (bytes && fread(p, 1, bytes, in) != bytes)) {
        fprintf(stderr, "input too short\n");
        exit(2);
    }
    return p;
}

#define CHECK(call)                                                              \
    do {                                                                         \
        rt_status s_ = (call);                                                   \
        if (s_ != RT_OK) {                                                       \
            fprintf(stderr, "%s failed: %d %s\n", #call, (int)s_, rt_last_error()); \
            return 1;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s problem.bin channel.bin\n", argv[0]);
        return 2;
    }
    in = fopen(argv[1], "rb");
    if (!in) {
        perror(argv[1]);
        return 2;
    }
    const int64_t* hdr = (const int64_t*)take(6 * sizeof(int64_t));
    const int64_t n_vtx = hdr[0], n_tri = hdr[1], M = hdr[2], R = hdr[3];
    const float* vtx = (const float*)take(12 * (size_t)n_vtx);
    const int32_t* tri = (const int32_t*)take(12 * (size_t)n_tri);
    const int32_t* surf = (const int32_t*)take(4 * (size_t)n_tri);
    const float* refl_re = (const float*)take(4 * (size_t)n_tri);
    const float* refl_im = (const float*)take(4 * (size_t)n_tri);
    const double* elems = (const double*)take(24 * (size_t)M);
    const double* rg = (const double*)take(10 * sizeof(double));
    const double* td = (const double*)take(10 * sizeof(double));
    const double* rd = (const double*)take(6 * sizeof(double));
    const double* freq = (const double*)take(sizeof(double));
    const double* rx = (const double*)take(24 * (size_t)R);
    fclose(in);

    rt_tx tx = {{td[0], td[1], td[2]}, {td[3], td[4], td[5]}, td[6], td[7], (int32_t)td[8], td[9]};
    rt_rx rxa = {{rd[0], rd[1], rd[2]}, rd[3], (int32_t)rd[4], rd[5]};
    rt_params prm = {freq[0], (int32_t)hdr[5], hdr[4], 0u};

    rt_ctx ctx;
    uint64_t scene = 0, ris = 0, ch = 0;
    rt_stats st;
    int64_t R2 = 0, M2 = 0, n_env = 0, n_slots = 0;
    CHECK(rt_init(0, 0, &ctx));
    CHECK(rt_scene_create(ctx, vtx, n_vtx, tri, n_tri, surf, refl_re, refl_im, NULL, &scene));
    CHECK(rt_ris_create(ctx, elems, M, rg, rg + 3, rg[6], rg[7], rg[8], rg[9], &ris));
    CHECK(rt_trace(ctx, scene, ris, &tx, rx, R, &rxa, &prm, NULL, &ch, &st));
    CHECK(rt_channel_info(ctx, ch, &R2, &M2, &n_env, &n_slots));
    float* E = (float*)malloc(8 * (size_t)(R2 > 0 ? R2 : 1));
    float* H = (float*)malloc(8 * (size_t)(R2 * M2 > 0 ? R2 * M2 : 1));
    CHECK(rt_channel_read(ctx, ch, E, H, NULL));
    CHECK(rt_destroy(ctx, ch));
    CHECK(rt_destroy(ctx, ris));
    CHECK(rt_destroy(ctx, scene));
    CHECK(rt_shutdown(ctx));

    FILE* out = fopen(argv[2], "wb");
    if (!out) {
        perror(argv[2]);
        return 2;
    }
    const int64_t counts[4] = {R2, M2, st.segments, st.n_env_paths};
    fwrite(counts, sizeof(int64_t), 4, out);
    fwrite(E, 8, (size_t)R2, out);
    fwrite(H, 8, (size_t)(R2 * M2), out);
    fclose(out);
    printf("traced %lld receivers x %lld elements, %lld segments, %lld environment paths\n", (long long)R2,
           (long long)M2, (long long)st.segments, (long long)st.n_env_paths);
    return 0;
}
