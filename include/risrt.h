/*
 * risrt: RIS-aware ray tracer for AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path of "Ray Tracing Algorithm for Reconfigurable
 * Intelligent Surfaces" (arXiv 2402.13034): ray launch over a triangle mesh,
 * specular reflections up to order K found by discovery rays and the image
 * method (Section II, Section II-B), the per-element RIS path-loss model
 * (Section II-A, eqs. (4)-(8)), the coherent sum at a set of receivers
 * (eqs. (9)-(10)) and that sum over many RIS configurations.
 *
 * Conventions shared by every call
 *   - Units are SI: metres, hertz, watts; gains and patterns are linear power
 *     quantities.  Vertices are float32, other positions float64.
 *   - Complex arrays are interleaved (re, im) float32 pairs.
 *   - Every input pointer may be host or device memory unless stated; the
 *     library copies what it keeps and holds no caller pointer after a call
 *     returns.  Outputs marked "device" must be device memory owned by the
 *     caller and stay valid until `stream` has finished the call's work.
 *   - `stream` is a hipStream_t (NULL: the null stream).  Calls enqueue their
 *     work on it and return; a call that must know a size on the host (noted
 *     below) waits for the stream up to that point.
 *   - Errors are returned, never thrown; on error no output is written and
 *     rt_last_error() returns a message for the calling thread.
 *   - Handles (scene, RIS, channel) are nonzero 64-bit values owned by the
 *     context; rt_destroy() releases one once work already enqueued on the
 *     stream that last used it has finished.
 *   - Results are deterministic: identical inputs give bit-identical outputs,
 *     whether a call runs alone or concurrently with others.
 */
#ifndef RISRT_H
#define RISRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;

#define RT_MAX_ORDER 5   /* largest reflection order K (Section II-B's order of the image method) */
#define RT_OK 0
#define RT_EINVAL (-1)       /* invalid argument */
#define RT_ENOMEM (-2)       /* the context's memory budget would be exceeded */
#define RT_EDEVICE (-3)      /* a HIP call failed */
#define RT_EBUSY (-4)        /* handle in use */
#define RT_ENOTFOUND (-5)    /* unknown or destroyed handle */
#define RT_EUNSUPPORTED (-6) /* size or option outside what the library supports */

/* antenna / element pattern kinds (power patterns, 1 at the maximum) */
#define RT_PAT_ISO 0      /* F = 1 */
#define RT_PAT_COSPOW 1   /* F = cos^p(theta) for theta < 90 deg, else 0: eq. (11) with
                             p = G_t/2 - 1, eq. (13) with p = 1 */
#define RT_PAT_MONOPOLE 2 /* eq. (12), monopole height h = p * lambda; 0 at theta = 0, pi */

/* rt_params.flags */
#define RT_FLAG_KEEP_HITS 1u   /* keep discovery hit lists (rt_hits_read) */
#define RT_FLAG_KEEP_PATHS 2u  /* keep path lists (rt_paths_read) and the element paths' fields
                                  (rt_ris_paths_read: 16 B per slot and element) */
#define RT_FLAG_BRUTE_FORCE 4u /* test every triangle instead of walking the BVH */
#define RT_FLAG_EXHAUSTIVE 8u  /* candidates = every surface sequence of order <= K
                                  (no discovery rays; small scenes only) */
#define RT_FLAG_COUNT_WORK 16u /* run the counting builds of discovery and of the per-element
                                  kernel and report their work in rt_stats.discovery_work and
                                  rt_stats.ris_work (same results) */
#define RT_FLAG_FRESNEL_TE 64u /* per bounce, the Fresnel coefficient (Section II-B) of the triangle's
                                  material (rt_scene_set_materials) at the incidence angle, for the
                                  field perpendicular to the plane of incidence, instead of the
                                  fixed coefficient; eps = eps_r - j sigma / (2 pi f eps0) */
#define RT_FLAG_FRESNEL_TM 128u /* the same for the field in the plane of incidence; at most one of the
                                  two; not with RT_FLAG_COUNT_WORK */
#define RT_FLAG_KEEP_CIR 256u  /* keep per-path delays and amplitudes for rt_cir (the RIS paths'
                                  amplitude and unfolded length per slot and element: 16 B each);
                                  not with RT_FLAG_RIS_INCOMING */
#define RT_FLAG_STAGE_TIMES 512u /* fill every rt_stats.ms_stage entry (events between the stages);
                                   without it only ms_stage[5], the per-element kernel, is timed */
#define RT_FLAG_RIS_INCOMING 32u /* the field reaching each element also by reflections
                                  Tx -> surfaces -> element (Section II-B, supporting
                                  reflections): image method per element for the Tx
                                  candidate sequences (order 1..K) valid and unblocked from
                                  the Tx to the RIS centre; without it, the direct leg alone */

/* rt_ris_sum precision */
#define RT_PREC_VALU_F32 0   /* FP32 complex multiply-add on the vector ALUs */
#define RT_PREC_MFMA_BF16X2 1 /* H = H_hi + H_lo (bf16 each), Gamma rounded once to bf16,
                                 two bf16 matrix-core products, FP32 accumulation */
#define RT_PREC_MFMA_BF16X3 2 /* also Gamma = G_hi + G_lo: three products */
#define RT_PREC_MFMA_F16X2 3  /* each receiver's H rows scaled by a power of two that puts their largest
                                 magnitude in [2^14, 2^15), split into fp16 hi + lo; Gamma rounded once
                                 to fp16 (|Gamma| below 6.1e-5 falls into fp16's subnormal range); two fp16
                                 matrix-core products, FP32 accumulation, the scale undone exactly */

typedef struct rt_ctx_s* rt_ctx;

/* Transmitter (Section III-B): position, pattern axis (boresight), transmit
 * power P_t [W], gain G_t (linear), pattern kind and parameter. */
typedef struct {
    double pos[3];
    double axis[3];
    double power_w;
    double gain;
    int32_t pattern;
    double param;
} rt_tx;

/* Receiver antenna shared by all receiver points (Section III-B): pattern
 * axis (monopole wire axis), gain G_r (linear), pattern kind and parameter. */
typedef struct {
    double axis[3];
    double gain;
    int32_t pattern;
    double param;
} rt_rx;

/* freq_hz: carrier (Table I).  max_order: K, reflections between the source
 * (Tx or RIS element) and the receiver, 0..RT_MAX_ORDER.  n_rays: discovery rays per
 * source (the RIS-centre source launches into the half-space in front of the
 * RIS, about n_rays).  flags: RT_FLAG_*. */
typedef struct {
    double freq_hz;
    int32_t max_order;
    int64_t n_rays;
    uint32_t flags;
} rt_params;

/* Work counts and stage times of one rt_trace call (times only if requested,
 * which waits for the stream at the end of the call; the stages other than
 * the per-element kernel only with RT_FLAG_STAGE_TIMES). */
typedef struct {
    int64_t segments;            /* all ray segments traced */
    int64_t discovery_segments;  /* discovery closest-hit segments */
    int64_t leg_segments;        /* visibility legs (any-hit segments) */
    int64_t n_cand_tx;           /* candidate sequences from the Tx (incl. order 0) */
    int64_t n_cand_u;            /* candidate sequences from the RIS centre */
    int64_t n_env_paths;         /* valid Tx -> Rx paths */
    int64_t n_u_paths;           /* valid RIS-centre -> Rx sequences of order >= 1 */
    int64_t n_ris_slots;         /* (rx, sequence) slots expanded per element */
    float ms_stage[8];           /* setup, candidates (discovery, dedupe, images), -, Tx paths,
                                    RIS-centre paths, per-element kernel, Tx->element legs, total */
    int64_t ris_work[5];         /* with RT_FLAG_COUNT_WORK: BVH node visits, triangle tests,
                                    FP64 containment tests, (slot, element) pairs, legs of
                                    the per-element kernel */
    int64_t leg_walk_fallbacks;  /* slots whose grouped leg walk outgrew its on-chip lists and
                                    were walked leg by leg (same results, diagnostic only) */
    int64_t n_in_seq;            /* RT_FLAG_RIS_INCOMING: Tx candidate sequences valid and unblocked
                                    from the Tx to the RIS centre (order >= 1) */
    int64_t n_in_paths;          /* RT_FLAG_RIS_INCOMING: emitted paths Tx -> surfaces -> element */
    int64_t discovery_work[6];   /* with RT_FLAG_COUNT_WORK: binary BVH node visits, triangle tests and
                                    segments of discovery from the Tx, then the same from the RIS
                                    centre (each ray walks the tree on its own) */
    float ms_discovery[3];       /* with RT_FLAG_STAGE_TIMES: the discovery kernel of the Tx, of the RIS
                                    centre (events on their streams), and the span of both (they
                                    overlap on two streams) */
} rt_stats;

/* Environment path record (RT_FLAG_KEEP_PATHS): Tx -> surfaces seq[0..k) ->
 * receiver rx, reflecting on triangles tri[0..k) (-1 from k on). */
typedef struct {
    int32_t rx;
    int32_t order;
    int32_t seq[RT_MAX_ORDER];
    int32_t tri[RT_MAX_ORDER];
    double length;   /* unfolded path length [m] */
    float amp[2];    /* complex amplitude at the receiver (E field, V/m) */
} rt_env_path;

/* Thread-local message for the last failing call ("" if none). */
const char* rt_last_error(void);

/* Open a context on HIP device `device`.  mem_budget_bytes bounds the device
 * memory the context holds at once (objects plus the scratch of calls in
 * flight); 0 means 90% of the device's free memory. */
rt_status rt_init(int device, uint64_t mem_budget_bytes, rt_ctx* out);
rt_status rt_shutdown(rt_ctx ctx);

/* Bytes currently held and the budget. */
rt_status rt_mem_info(rt_ctx ctx, uint64_t* in_use, uint64_t* budget);

/* Scene: n_vtx float32 vertices (x, y, z), n_tri triangles (3 vertex
 * indices each), surf[n_tri] the planar surface each triangle belongs to (a
 * wall or a face: the "surfaces" whose permutations Section II-B searches;
 * triangles of one surface must be coplanar; ids 0..n_surf-1, each used), and
 * a complex reflection coefficient per triangle applied at every specular
 * bounce.  n_tri may be 0 (free space); at most 2^29 - 1 triangles and
 * 2^21 - 1 surfaces (RT_EINVAL beyond).  Builds the BVH on `stream`
 * (waits for it once, to check the tree depth; device arrays are read in
 * place, host arrays staged, all before the call returns). */
rt_status rt_scene_create(rt_ctx ctx, const float* vtx_xyz, int64_t n_vtx, const int32_t* tri,
                          int64_t n_tri, const int32_t* surf, const float* refl_re,
                          const float* refl_im, void* stream, uint64_t* scene);

/* Sizes of a scene: triangles, surfaces, the depth of its BVH (the longest
 * root-to-leaf path of the binary tree; the traversal kernels keep 32 stack
 * entries per lane below depth 31, else 64) and the device bytes it holds.
 * Any pointer may be NULL. */
rt_status rt_scene_info(rt_ctx ctx, uint64_t scene, int64_t* n_tri, int64_t* n_surf, int32_t* bvh_depth,
                        uint64_t* bytes);

/* RIS (Section II-A, Section III-C): M element centres (x, y, z), the RIS
 * centre u (the point the reflection search starts from, Section II-B), the
 * unit normal n pointing into the room (z axis of every element's frame),
 * effective element size d_y, d_z, element gain G (<= 0: 4 pi d_y d_z /
 * lambda^2 at the trace frequency) and element pattern cos^q. */
rt_status rt_ris_create(rt_ctx ctx, const double* elem_xyz, int64_t M, const double centre[3],
                        const double normal[3], double dy, double dz, double elem_gain,
                        double pattern_q, uint64_t* ris);

/* Trace one problem and build its channel:
 *   H[r, m]   = field at receiver r through element m for Gamma_m = 1: direct
 *               Tx -> m -> r plus m -> surfaces -> r for every sequence valid
 *               from the RIS centre to r (eqs. (4)-(8), Section II-B);
 *   E_env[r]  = field of Tx -> surfaces -> r paths, orders 0..K (eq. (3)).
 * ris may be 0 (no RIS: only E_env).  rx_xyz: R float64 receiver points,
 * R <= 65535 x 64 (RT_EUNSUPPORTED beyond, before any work is queued).
 * Waits for `stream` several times (candidate and path counts). */
rt_status rt_trace(rt_ctx ctx, uint64_t scene, uint64_t ris, const rt_tx* tx, const double* rx_xyz,
                   int64_t R, const rt_rx* rx, const rt_params* params, void* stream,
                   uint64_t* channel, rt_stats* stats);

/* Channel built from given arrays (for RIS sums of channels made elsewhere):
 * E_env[2R], H[2 R M] (interleaved complex, host or device). */
rt_status rt_channel_create(rt_ctx ctx, int64_t R, int64_t M, const float* E_env, const float* H,
                            void* stream, uint64_t* channel);

/* R, M and path counts of a channel. */
rt_status rt_channel_info(rt_ctx ctx, uint64_t channel, int64_t* R, int64_t* M, int64_t* n_env_paths,
                          int64_t* n_ris_slots);

/* Copy E_env (2R floats) and/or H (2RM floats, receiver-major) to host or
 * device memory (either may be NULL).  Waits for the stream. */
rt_status rt_channel_read(rt_ctx ctx, uint64_t channel, float* E_env, float* H, void* stream);

/* Discovery hit lists (RT_FLAG_KEEP_HITS): source 0 = Tx (n_rays rows),
 * 1 = RIS centre (2 n_rays rows of a 2n-point sphere; rows not launched are
 * -1).  Row i, bounce b at hits[i * K + b]: triangle index, -1 after a miss.
 * cap = capacity in int32; *rows receives the row count.  Waits. */
rt_status rt_hits_read(rt_ctx ctx, uint64_t channel, int32_t source, int32_t* hits, int64_t cap,
                       int64_t* rows);

/* Path lists (RT_FLAG_KEEP_PATHS), all in canonical (receiver, sequence key)
 * order, host memory.  Each pointer may be NULL; *_n receive the counts.
 *   env[cap_env]          environment paths;
 *   useq[cap_u * (1 + RT_MAX_ORDER)]  (rx, s_0 .. s_4, -1 padded) sequences
 *                         valid from the RIS centre;
 *   ris_valid[cap_slots * M] 1 if the element path of slot s, element m is
 *                         emitted; slots are receiver-major, the first slot
 *                         of a receiver is the direct path and the others
 *                         follow its useq rows in order.  Waits. */
rt_status rt_paths_read(rt_ctx ctx, uint64_t channel, rt_env_path* env, int64_t cap_env,
                        int64_t* n_env, int32_t* useq, int64_t cap_u, int64_t* n_u,
                        uint8_t* ris_valid, int64_t cap_slots, int64_t* n_slots);

/* Per-path RIS fields (RT_FLAG_KEEP_PATHS or RT_FLAG_KEEP_CIR), one cell
 * per (slot, element) in the slot order of rt_paths_read's ris_valid
 * (cell = slot * M + m): amp[2 cell .. 2 cell + 1] = complex amplitude of the
 * element path at the receiver for Gamma_m = 1 (eq. (7) times eq. (8), with
 * the reflection coefficients of its bounces; 0 where no path is emitted);
 * length[cell] = its unfolded length, d_t + D_r for the direct incoming leg
 * (eqs. (7)-(8)), D_r alone with RT_FLAG_RIS_INCOMING (the element's field
 * then sums several incoming paths).  Either pointer may be NULL; host or
 * device memory of cap_cells entries; *n_cells receives n_slots * M.
 * RT_EINVAL if the channel kept no paths or cap_cells is too small.  Waits. */
rt_status rt_ris_paths_read(rt_ctx ctx, uint64_t channel, float* amp, double* length, int64_t cap_cells,
                           int64_t* n_cells);

/* Candidate sequences (surface ids, -1 padded, RT_MAX_ORDER per row) found
 * for source 0 (Tx) or 1 (RIS centre), in key order (the order of
 * sum_j (s_j + 1) 2^(21 j) as an integer); cap in int32.  Kept with
 * RT_FLAG_KEEP_PATHS or RT_FLAG_KEEP_HITS.  Waits. */
rt_status rt_candidates_read(rt_ctx ctx, uint64_t channel, int32_t source, int32_t* seq, int64_t cap,
                             int64_t* n);

/* Coherent RIS sum (eqs. (9)-(10)) for C configurations:
 *   E[r, c] = E_env[r] + gamma_scale * sum_m H[r, m] Gamma[m, c],
 *   P[r, c] = |E[r, c]|^2 / (2 eta0),  eta0 = 120 pi.
 * gamma: complex [M x C] (configuration fastest), device memory.
 * gamma_is_real != 0 declares every imaginary part zero (half the work).
 * E_out: device [R x C] complex or NULL; P_out: device [R x C] float or NULL.
 * precision: RT_PREC_*. */
rt_status rt_ris_sum(rt_ctx ctx, uint64_t channel, const float* gamma, int64_t C, float gamma_scale,
                     int32_t gamma_is_real, int32_t precision, float* E_out, float* P_out,
                     void* stream);

/* The coherent sum of rt_ris_sum (same arguments, same kernels, same
 * results) for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * allocates nothing: the split of H and Gamma goes to a static 64 MiB array
 * that every device the library runs on holds until the process ends, and is
 * rebuilt on every call (no cached split).  gamma, E_out and P_out are the
 * caller's device memory as for rt_ris_sum.  Scratch needed: 2 (2R rounded up
 * to 256) Kp + (1, or 2 for RT_PREC_MFMA_BF16X3) (C rounded up to 256) Kp
 * bytes, times 2 for 16-bit values, plus 4R for RT_PREC_MFMA_F16X2, with
 * Kp = M (real Gamma) or 2M (complex) rounded up to 32; a larger sum returns
 * RT_EUNSUPPORTED (e.g. 4096 receivers x 1024 elements x 4096 real
 * configurations fit; 16384 x 1024 do not).  RT_PREC_VALU_F32 uses no
 * scratch.  Every call on one device shares that array: calls that overlap
 * on the device (on different streams without an order between them) race
 * and must be serialised by the caller. */
rt_status rt_ris_sum_noalloc(rt_ctx ctx, uint64_t channel, const float* gamma, int64_t C, float gamma_scale,
                            int32_t gamma_is_real, int32_t precision, float* E_out, float* P_out, void* stream);

/* Channel impulse response of one RIS configuration (the paths' delays,
 * Section II-B / Fig. 3 context): cir[r, b] = sum of the complex amplitudes
 * of the paths reaching receiver r with unfolded length d in
 * [b L, (b + 1) L), L = c * bin_s (c = 299 792 458 m/s; bin = floor(d / L)):
 * the environment paths as traced, and every RIS path of element m
 * multiplied by gamma[m]; paths past the last bin are left out, so the bins
 * sum to the narrowband field E = E_env + H gamma when none is.  gamma:
 * complex [M], device; cir: device complex [R x n_bins]; 0 < n_bins <= 2^24.
 * The channel must have been traced with RT_FLAG_KEEP_CIR (RT_EINVAL
 * otherwise).  Enqueued on `stream`. */
rt_status rt_cir(rt_ctx ctx, uint64_t channel, const float* gamma, double bin_s, int64_t n_bins, float* cir,
                 void* stream);

/* Materials of a scene's triangles (original order) for the Fresnel
 * coefficients (RT_FLAG_FRESNEL_TE/TM; Section III's table gives metal as
 * eps_r = 1, sigma = 1e7 S/m): relative permittivity eps_r >= 1 and
 * conductivity sigma >= 0 [S/m], host or device arrays of n_tri floats,
 * copied (the call waits for the copy); the first call also computes the
 * triangles' unit normals the coefficients use (on `stream`).  Calling again
 * replaces the materials for later traces.  RT_EINVAL on a null array or an
 * out-of-range value. */
rt_status rt_scene_set_materials(rt_ctx ctx, uint64_t scene, const float* eps_r, const float* sigma,
                                 void* stream);

/* Sort n keys of `words` 64-bit words each (1 or 2; word 0 the least
 * significant) in device memory, in place, by their bits [begin_bit,
 * end_bit) (0 <= begin_bit <= end_bit <= 64 words), stably: keys equal on
 * those bits keep their order.  With unique != 0, keys equal in every word
 * are then kept once.  This is the primitive behind the de-duplication of
 * the candidate surface sequences (packed 21 bits per surface; Section II-B
 * searches the permutations of surfaces) and the Morton order of the BVH
 * build.  *n_out (may be NULL) receives the number of keys left; the call
 * waits for the stream.  RT_EINVAL on bad arguments or host memory,
 * RT_EUNSUPPORTED for 2^32 keys or more. */
rt_status rt_keys_sort(rt_ctx ctx, uint64_t* keys, int64_t n, int32_t words, int32_t begin_bit, int32_t end_bit,
                       int32_t unique, int64_t* n_out, void* stream);

/* Release a scene, RIS or channel. */
rt_status rt_destroy(rt_ctx ctx, uint64_t handle);

#ifdef __cplusplus
}
#endif

#endif /* RISRT_H */
