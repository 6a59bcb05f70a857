"""Benchmark of the RIS ray tracer's hot path on one MI355X.

One step = the whole path on the lab-room workload (6 x 5 x 3 m room with 20
furniture boxes, 1908 triangles; 127-element hexagonal RIS; horn Tx; 64 x 64
receivers; reflections up to order 3; 1e6 discovery rays per source):
BVH build from the device-resident mesh, discovery, dedupe, image-method
paths and their visibility legs from the Tx and from the RIS centre, the
per-element expansion into H, and the coherent sum for the configured
2-bit RIS phases.

Prints one JSON line: value = ray segments traced per second (millions),
plus the dominant kernel's roofline, the many-configuration RIS sum on the
matrix cores (TFLOP/s, 16384 receivers x 1024 elements x 4096
configurations; bf16 and fp16 split products, the VALU sum, and the plain
per-configuration tracer that traces again for every configuration) and the
oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
VECTOR_PEAK_TFLOPS = 78.6   # FP32 (non-packed FMA) = FP64 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz

# Algorithmic flops of the per-element kernel's units of work, the unit costs
# the hot-path scope fixes for the traversal and the per-candidate FP64 work:
#   BVH node visit (two slab tests)                                 -> 40
#   ray/triangle test                                               -> 40
#   (slot, element) pair: images, back-trace, containment, side
#     tests, patterns, lengths, phase, amplitude, leg set-up (FP64)  -> 150 (the low end of 150-300)
# Containment tests and leg set-ups are inside the pair's 150; the counting
# build reports them separately.  The counts come from a counting instance
# that walks the binary tree per leg (the method's LBVH walk); the timed
# instance walks the tube of each slot's legs once, so `achieved` is the
# method's algorithmic work per second, not the instructions executed: those
# are in `valu_issue_share` (SQ counters of the timed instance).
FLOPS_PER = {"node": 40, "tri": 40, "contain": 0, "pair": 150, "leg": 0}
FLOPS_PER_PAIR_HIGH = 300
SQ_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_ris_lab_room_sq_counters.json")
KERNEL_SOURCES = ["paper_2402_13034_amd/csrc/rt_trace.hip", "paper_2402_13034_amd/csrc/rt_internal.hpp"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_ris_lab_room_hbm_counters.json")
DISC_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_discover_office_floor_hbm_counters.json")


def kernel_source_hash(kernel="k_ris"):
    """Hash of what a trace kernel is compiled from: the device header and the
    kernel's own text in the trace source (its template line to the closing
    brace), so host-side changes elsewhere in the file keep it."""
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, KERNEL_SOURCES[1]), "rb") as f:
        h.update(f.read())
    with open(os.path.join(ROOT, KERNEL_SOURCES[0])) as f:
        lines = f.read().split("\n")
    start = next(i for i, l in enumerate(lines) if (" void %s(" % kernel) in l) - 1
    end = next(i for i in range(start, len(lines)) if lines[i] == "}")
    h.update("\n".join(lines[start:end + 1]).encode())
    return h.hexdigest()[:16]


def measured_traffic(path=COUNTERS_FILE, kernel="k_ris"):
    """HBM bytes per launch of a kernel from a committed counter summary, if
    it was taken on the current kernel sources."""
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


def measured_valu_share():
    """VALU issue share of the timed k_ris instance (VALU wave instructions x 4
    cycles over 1024 SIMDs x launch time x clock) from the committed SQ
    counters, if they were taken on the current kernel sources."""
    try:
        with open(SQ_COUNTERS_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return {"valu_issue_share": d.get("valu_issue_share"), "clock_ghz": d.get("clock_ghz"),
            "valu_wave_insts": d.get("valu_wave_insts"), "launch_us": d.get("launch_us")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def device_mesh(prob):
    import torch
    sc = prob.scene
    return (torch.from_numpy(np.ascontiguousarray(sc.V, np.float32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(sc.T, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(sc.surf, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(sc.refl_re, np.float32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(sc.refl_im, np.float32)).cuda())


def run_trace_bench(ctx, prob, steps, warmup, variants=True):
    import torch
    from paper_2402_13034_amd import risrt, synth
    mesh = device_mesh(prob)
    rx = torch.from_numpy(prob.rx_pos).cuda()
    gamma = torch.from_numpy(prob.gamma.astype(np.complex64)).cuda()
    r = prob.ris
    ris = ctx.ris_create(r.elems, r.centre, r.normal, r.dy, r.dz, r.gain, r.q)
    P_out = torch.empty((prob.rx_pos.shape[0], gamma.shape[1]), dtype=torch.float32, device="cuda")

    host_ms = []

    def step():
        t0 = time.perf_counter()
        scene = ctx.scene_create(*mesh)
        t1 = time.perf_counter()
        ch, st = risrt.trace_problem(ctx, prob, scene, ris, rx=rx)
        t2 = time.perf_counter()
        ctx.ris_sum(ch, gamma, precision=risrt.PREC_VALU_F32, want_P=False, P_out=P_out)
        t3 = time.perf_counter()
        ctx.destroy(ch)
        ctx.destroy(scene)
        t4 = time.perf_counter()
        host_ms.append([(t1 - t0) * 1e3, (t2 - t1) * 1e3, (t3 - t2) * 1e3, (t4 - t3) * 1e3])
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    host_ms.clear()
    # as timeit does: no interpreter garbage collection inside the timed steps
    # (a full collection over torch's objects stalls the host for tens of ms)
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        stats = [step() for _ in range(steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        gc.enable()
    for s, h in zip(stats, host_ms):
        s["host_ms"] = h
    # counting build of the per-element kernel (untimed; same inputs and results)
    scene = ctx.scene_create(*mesh)
    ch, cst = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_COUNT_WORK)
    ctx.destroy(ch)
    # the time of every stage (untimed: its events sit between the stages); the timed
    # steps time only the per-element kernel
    ch, sst = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_STAGE_TIMES)
    ctx.destroy(ch)
    stats[-1]["stage_ms_all"] = sst["ms_stage"]
    if not variants:
        ctx.destroy(scene)
        ctx.destroy(ris)
        return stats, t1 - t0, cst["ris_work"], None
    # the same step with the reflections Tx -> surfaces -> element as well (its own line,
    # not the headline: the workload's channel has the direct incoming leg only)
    n_in = max(2, steps // 2)
    ch, _ = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_RIS_INCOMING)   # warm-up
    ctx.destroy(ch)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        t2 = time.perf_counter()
        in_stats = []
        for _ in range(n_in):
            ch, sti = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_RIS_INCOMING)
            ctx.ris_sum(ch, gamma, precision=risrt.PREC_VALU_F32, want_P=False, P_out=P_out)
            ctx.destroy(ch)
            in_stats.append(sti)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
    finally:
        gc.enable()
    incoming = {"ms_per_step_without_scene_build": (t3 - t2) / n_in * 1e3, "steps": n_in,
                "segments_per_step": in_stats[-1]["segments"], "n_in_seq": in_stats[-1]["n_in_seq"],
                "n_in_paths": in_stats[-1]["n_in_paths"],
                "Mray_segments_per_s": sum(x["segments"] for x in in_stats) / (t3 - t2) / 1e6}
    # and with TM Fresnel coefficients of seeded materials (one per surface) instead of the fixed ones
    pf = synth.with_materials(prob, 2)
    ctx.scene_set_materials(scene, pf.mat_eps_r, pf.mat_sigma)
    ch, _ = risrt.trace_problem(ctx, pf, scene, ris, rx=rx)   # warm-up
    ctx.destroy(ch)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        t4 = time.perf_counter()
        f_stats = []
        for _ in range(n_in):
            ch, stf = risrt.trace_problem(ctx, pf, scene, ris, rx=rx)
            ctx.ris_sum(ch, gamma, precision=risrt.PREC_VALU_F32, want_P=False, P_out=P_out)
            ctx.destroy(ch)
            f_stats.append(stf)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
    finally:
        gc.enable()
    fresnel = {"ms_per_step_without_scene_build": (t5 - t4) / n_in * 1e3, "steps": n_in,
               "polarisation": "TM", "Mray_segments_per_s": sum(x["segments"] for x in f_stats) / (t5 - t4) / 1e6,
               "k_ris_ms": sum(x["ms_stage"][5] for x in f_stats) / n_in}
    # impulse response of the configuration: 0.25 ns bins, 400 of them (every path of the room)
    ch, stc = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_KEEP_CIR)
    g0 = gamma[:, 0].contiguous()
    ctx.cir(ch, g0, 2.5e-10, 400)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        h = ctx.cir(ch, g0, 2.5e-10, 400)
    e1.record()
    torch.cuda.synchronize()
    cir = {"bins": 400, "bin_ns": 0.25, "ms": e0.elapsed_time(e1) / 3, "receivers": int(h.shape[0]),
           "ris_paths_kept": int(stc["n_ris_slots"]) * prob.ris.elems.shape[0]}
    ctx.destroy(ch)
    ctx.destroy(scene)
    ctx.destroy(ris)
    return stats, t1 - t0, cst["ris_work"], {"ris_incoming_reflections": incoming, "fresnel_tm": fresnel,
                                             "impulse_response": cir}


# bytes of the discovery walk per unit (this library's layouts): a binary node
# visit reads both child boxes and links (four float4, 64 B), a triangle test
# reads (v0, id), (e1, surface), (e2, -) (48 B); per segment the ray (32 B) and
# the hit (8 B) as the traversal roofline counts them
DISC_BYTES = {"segment": 40, "node": 64, "tri": 48}


def run_large_bench(ctx, reps=2):
    """The large configuration: the office floor (about 1.08e6 triangles,
    5064 surfaces), order 5, 1e7 discovery rays per source (1e8 discovery
    segments), 256 x 256 receivers, 64 x 64 RIS; scene build, whole traces
    (discovery to H), the stage and discovery-kernel times, the discovery
    walk priced in algorithmic bytes (counting build) against HBM, and the
    1024-configuration sum of its channel on the matrix cores."""
    import torch
    from paper_2402_13034_amd import risrt, synth
    prob = synth.office_floor()
    mesh = device_mesh(prob)
    rx = torch.from_numpy(prob.rx_pos).cuda()
    r = prob.ris
    ris = ctx.ris_create(r.elems, r.centre, r.normal, r.dy, r.dz, r.gain, r.q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scene = ctx.scene_create(*mesh)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    info = ctx.scene_info(scene)
    ch, _ = risrt.trace_problem(ctx, prob, scene, ris, rx=rx)   # warm-up
    ctx.destroy(ch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = []
    for _ in range(reps):
        ch, st = risrt.trace_problem(ctx, prob, scene, ris, rx=rx)
        ctx.destroy(ch)
        sts.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    stage = []
    for _ in range(2):
        ch, sst = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_STAGE_TIMES)
        ctx.destroy(ch)
        stage.append(sst)
    ch, cst = risrt.trace_problem(ctx, prob, scene, ris, rx=rx, flags=risrt.FLAG_COUNT_WORK)
    ctx.destroy(ch)
    ms_tx = float(np.mean([s_["ms_discovery"][0] for s_ in stage]))
    ms_span = float(np.mean([s_["ms_discovery"][2] for s_ in stage]))
    # the per-element kernel priced as on the lab room (same unit costs)
    ris_units = dict(zip(["node", "tri", "contain", "pair", "leg"], cst["ris_work"]))
    ris_ms = float(np.mean([s_["ms_stage"][5] for s_ in stage]))
    ris_flops = sum(FLOPS_PER[k] * ris_units[k] for k in ris_units)
    ris_ach = ris_flops / (ris_ms * 1e-3) / 1e12
    w = cst["discovery_work"]
    units_tx = {"node": w[0], "tri": w[1], "segment": w[2]}
    units_all = {"node": w[0] + w[3], "tri": w[1] + w[4], "segment": w[2] + w[5]}
    bytes_tx = sum(DISC_BYTES[k] * v for k, v in units_tx.items())
    bytes_all = sum(DISC_BYTES[k] * v for k, v in units_all.items())
    ach_tx = bytes_tx / (ms_tx * 1e-3) / 1e9
    ach_all = bytes_all / (ms_span * 1e-3) / 1e9
    # the 1024-configuration sum of the channel (65536 receivers x 4096 elements)
    ch, _ = risrt.trace_problem(ctx, prob, scene, ris, rx=rx)
    R, M = prob.rx_pos.shape[0], prob.ris.elems.shape[0]
    C = 1024
    rng = np.random.default_rng(prob.seed + 9)
    g = torch.from_numpy((rng.integers(0, 2, size=(M, C)) * 2 - 1).astype(np.complex64)).cuda()
    P = torch.empty((R, C), dtype=torch.float32, device="cuda")
    ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=risrt.PREC_MFMA_BF16X2, P_out=P)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=risrt.PREC_MFMA_BF16X2, P_out=P)
    e1.record()
    torch.cuda.synchronize()
    ms_sum = e0.elapsed_time(e1) / 3
    for h in (ch, scene, ris):
        ctx.destroy(h)
    segs = sts[-1]["segments"]
    return {"workload": "office floor 40x20x3 m, 200 rooms, %d triangles / %d surfaces, order<=5, "
                        "1e7 rays per source, 256x256 receivers at 1.2 m, 64x64 RIS" % (info["n_tri"], info["n_surf"]),
            "scene_build_ms": build_ms, "bvh_depth": info["bvh_depth"], "scene_bytes": info["bytes"],
            "ms_per_trace": dt * 1e3, "segments_per_trace": segs,
            "discovery_segments": sts[-1]["discovery_segments"], "leg_segments": sts[-1]["leg_segments"],
            "Mray_segments_per_s": segs / dt / 1e6,
            "n_cand_tx": sts[-1]["n_cand_tx"], "n_cand_u": sts[-1]["n_cand_u"],
            "n_env_paths": sts[-1]["n_env_paths"], "n_ris_slots": sts[-1]["n_ris_slots"],
            "leg_walk_fallbacks": sts[-1]["leg_walk_fallbacks"],
            "stage_ms": stage[-1]["ms_stage"], "discovery_kernel_ms": {"tx": ms_tx, "both_span": ms_span},
            "roofline_discovery": {"kernel": "k_discover (Tx, 1e7 rays, order 5)", "bound": "hbm",
                                   "achieved": ach_tx, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": ach_tx / HBM_PEAK_GBS,
                                   "traffic": measured_traffic(DISC_COUNTERS_FILE, "k_discover"),
                                   "work_per_launch": units_tx, "bytes_per_unit": DISC_BYTES,
                                   "both_sources": {"achieved": ach_all, "frac": ach_all / HBM_PEAK_GBS,
                                                    "work": units_all}},
            "roofline_ris": {"kernel": "k_ris (order 5)", "bound": "alu", "achieved": ris_ach,
                             "peak": VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ris_ach / VECTOR_PEAK_TFLOPS,
                             "traffic": None, "launch_ms": ris_ms, "work_per_launch": ris_units,
                             "flops_per_unit": FLOPS_PER,
                             "binary_node_visits_per_leg": ris_units["node"] / max(ris_units["leg"], 1)},
            "ris_sum_1024": {"ms": ms_sum, "shape": {"R": R, "M": M, "C": C},
                             "tflops_complex_equiv": 8.0 * R * M * C / (ms_sum * 1e-3) / 1e12,
                             "tflops_executed": 8.0 * R * M * C / (ms_sum * 1e-3) / 1e12}}


def run_paper_bench(ctx, reps=3):
    """Section III's reflective scenario (metal walls, TE Fresnel, order 2):
    the 2 mm map (101 x 101 receivers) and the 1 cm map (61 x 91), each a
    whole trace (BVH build to H) plus the field of one configuration."""
    import torch
    from paper_2402_13034_amd import risrt, synth
    out = {}
    for grid in ("fine", "coarse"):
        prob = synth.paper_room(reflective=True, grid=grid)
        M = prob.ris.elems.shape[0]
        g = torch.full((M, 1), 1.25 + 0j, dtype=torch.complex64, device="cuda")
        rx = torch.from_numpy(prob.rx_pos).cuda()
        sc = prob.scene
        V, T, S = (torch.from_numpy(a).cuda() for a in (sc.V, sc.T, sc.surf))
        rr, ri = (torch.from_numpy(a).cuda() for a in (sc.refl_re, sc.refl_im))
        ris = ctx.ris_create(prob.ris.elems, prob.ris.centre, prob.ris.normal, prob.ris.dy, prob.ris.dz,
                             prob.ris.gain, prob.ris.q)

        def one():
            scene = ctx.scene_create(V, T, S, rr, ri)
            ctx.scene_set_materials(scene, prob.mat_eps_r, prob.mat_sigma)
            ch, st = risrt.trace_problem(ctx, prob, scene, ris, rx=rx)
            _, P = ctx.ris_sum(ch, g, precision=risrt.PREC_VALU_F32)
            ctx.destroy(ch)
            ctx.destroy(scene)
            return st

        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [one() for _ in range(reps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ctx.destroy(ris)
        out[grid] = {"receivers": int(prob.rx_pos.shape[0]), "ms_per_map": dt * 1e3,
                     "segments_per_map": sts[-1]["segments"], "Mray_segments_per_s": sts[-1]["segments"] / dt / 1e6}
    return out


def run_gemm_bench(ctx, reps=20, warm=20):
    """Many-configuration RIS sum on the matrix cores: channel from the box
    room with a 32 x 32 RIS and 128 x 128 receivers, 4096 random +-1
    configurations (Gamma = 0.9 s)."""
    import torch
    from paper_2402_13034_amd import risrt, synth
    prob = synth.precision_problem()
    scene, ris = risrt.upload_problem(ctx, prob)
    ch, st = risrt.trace_problem(ctx, prob, scene, ris)
    R, M = prob.rx_pos.shape[0], prob.ris.elems.shape[0]
    rng = np.random.default_rng(prob.seed + 7)
    C = 4096
    s = (rng.integers(0, 2, size=(M, C)) * 2 - 1).astype(np.complex64)
    g = torch.from_numpy(s).cuda()
    P = torch.empty((R, C), dtype=torch.float32, device="cuda")
    out = {}
    # error of the matrix-core sum against FP64 on the same FP32 channel (256 sampled receivers)
    E_env, H = ctx.channel_read(ch)
    rows = np.random.default_rng(6).choice(R, 256, replace=False)
    E_ref = E_env[rows].astype(np.complex128)[:, None] + 0.9 * (H[rows].astype(np.complex128) @ s.astype(np.complex128))
    P_ref = np.abs(E_ref) ** 2 / (2 * 120 * math.pi)
    inc = (np.abs(E_env[rows]).astype(float)[:, None] + 0.9 * np.abs(H[rows]).astype(float).sum(1)[:, None]) ** 2 \
        / (2 * 120 * math.pi)
    sel = P_ref >= 1e-3 * inc
    rows_t = torch.from_numpy(rows).cuda()
    for name, prec in (("bf16x2", risrt.PREC_MFMA_BF16X2), ("f16x2", risrt.PREC_MFMA_F16X2),
                       ("valu_f32", risrt.PREC_VALU_F32)):
        # warm-up long enough for the clocks to settle under matrix-core load (~10 ms)
        for _ in range(warm if prec != risrt.PREC_VALU_F32 else 1):
            ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=prec, P_out=P)
        torch.cuda.synchronize()
        n = reps if prec != risrt.PREC_VALU_F32 else 2
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=prec, P_out=P)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        Eo, Po = ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=prec, want_E=True, want_P=True)
        torch.cuda.synchronize()
        Es = Eo[rows_t].cpu().numpy().astype(np.complex128)
        Ps = Po[rows_t].cpu().numpy().astype(np.float64)
        del Eo, Po
        out[name] = {"ms": ms, "tflops_complex_equiv": 8.0 * R * M * C / (ms * 1e-3) / 1e12,
                     "tflops_executed": (4.0 * R * M * C * (1 if prec == risrt.PREC_VALU_F32 else 2)) / (ms * 1e-3) / 1e12,
                     "err_vs_fp64": {"max_db": float(np.max(np.abs(10 * np.log10(Ps[sel] / P_ref[sel])))),
                                     "max_phase_rad": float(np.max(np.abs(np.angle(Es[sel] / E_ref[sel])))),
                                     "nrmse": float(np.sqrt(np.mean(np.abs(Es - E_ref) ** 2) /
                                                            np.mean(np.abs(E_ref) ** 2))),
                                     "rows_sampled": 256, "frac_above_null_threshold": float(sel.mean())}}
    # the plain per-configuration tracer: the whole trace again for every
    # configuration, then that configuration's field (timed for a few, scaled to C)
    n_rt = 4
    g1 = [g[:, j:j + 1].contiguous() for j in range(n_rt)]
    P1 = torch.empty((R, 1), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for j in range(n_rt):
        ch_j, _ = risrt.trace_problem(ctx, prob, scene, ris)
        ctx.ris_sum(ch_j, g1[j], scale=0.9, gamma_is_real=True, precision=risrt.PREC_VALU_F32, P_out=P1)
        ctx.destroy(ch_j)
    e1.record()
    torch.cuda.synchronize()
    ms_cfg = e0.elapsed_time(e1) / n_rt
    out["per_config_retrace"] = {"ms_per_config": ms_cfg, "configs_timed": n_rt,
                                 "ms_for_all_configs": ms_cfg * C,
                                 "speedup_bf16x2": ms_cfg * C / out["bf16x2"]["ms"],
                                 "speedup_f16x2": ms_cfg * C / out["f16x2"]["ms"],
                                 "speedup_valu_f32": ms_cfg * C / out["valu_f32"]["ms"]}
    for h in (ch, scene, ris):
        ctx.destroy(h)
    out["shape"] = {"R": R, "M": M, "C": C}
    return out


def run_serving_bench(ctx, n_queries=2000, n_slots=4, probe=(0.2, 0.3, 0.4, 0.5, 0.6, 0.7), loads=(0.5, 0.7, 0.9),
                      cache_share=0.8):
    """The serving configuration: 16 random box rooms of 1k-200k triangles,
    32 deployments (RIS of 37-4096 elements, 16^2-256^2 receivers, order
    1-3), queries of 1-512 2-bit configurations drawn Zipf-like over the
    deployments, 2000 queries per seeded stream.  The channel cache holds
    `cache_share` of the deployments' channel bytes, so the streams evict
    channels and trace them again.  Every deployment is traced once first.
    A closed-loop burst of one stream gives the burst saturation; seeded
    Poisson streams at `probe` x that rate find the sustained rate (the
    highest offered rate achieved to within 5 %); streams at `loads` x the
    sustained rate follow (the headline is the one at 70 %), then a light
    stream at 20 % of it.  Latencies are reported for all queries, for cache
    hits and for misses (queries whose batch traced its channel or waited
    for it)."""
    from paper_2402_13034_amd import serve, workloads
    scenes, riss, deps = workloads.serving_mix_c4()
    mix_bytes = sum(workloads.channel_bytes(d, riss) for d in deps)
    srv = serve.Server(ctx, n_slots=n_slots, cache_bytes=int(cache_share * mix_bytes))
    for k, v in scenes.items():
        srv.add_scene(k, v)
    for k, v in riss.items():
        srv.add_ris(k, v)
    for d in deps:
        srv.add_deployment(d)
    t0 = time.perf_counter()
    for d in deps:   # trace every deployment once (the cache evicts as it fills)
        M = riss[d.ris_key].elems.shape[0]
        srv.submit(d.key, np.ones((M, 1), np.complex64)).result()
    t_warm = time.perf_counter() - t0
    log("bench: serving warm-up, %d deployments traced in %.1f s" % (len(deps), t_warm))
    # long-lived objects out of the collector's way, as a serving process would
    gc.collect()
    gc.freeze()

    def summary(st, n, dt, cols, offered=None):
        tr = st["traces"] - summary.traces
        summary.traces = st["traces"]
        out = {"achieved_qps": n / dt, "configs_per_s": cols / dt, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
               "hits": st["hits"], "hit_p50_ms": st["hit_p50_ms"], "hit_p99_ms": st["hit_p99_ms"],
               "misses": st["misses"], "miss_p50_ms": st["miss_p50_ms"], "miss_p99_ms": st["miss_p99_ms"],
               "traces": tr}
        if offered is not None:
            out["offered_qps"] = offered
        return {k: round(v, 3) if isinstance(v, float) else v for k, v in out.items()}
    summary.traces = srv.stats()["traces"]

    qs = workloads.query_stream(deps, riss, n_queries, seed=12)
    srv.clear_latencies()
    t0 = time.perf_counter()
    futs = [srv.submit(k, g) for k, g in qs]
    for f in futs:
        f.result()
    dt = time.perf_counter() - t0
    burst = summary(srv.stats(), n_queries, dt, sum(g.shape[1] for _, g in qs))
    burst_qps = burst["achieved_qps"]
    log("bench: serving burst", json.dumps(burst))

    def poisson(rate, seed, n=n_queries):
        stream = workloads.query_stream(deps, riss, n, seed=seed)
        srv.clear_latencies()
        t = time.perf_counter()
        serve.run_poisson(srv, stream, rate_hz=rate, seed=seed + 1)
        dt = time.perf_counter() - t
        r = summary(srv.stats(), n, dt, sum(g.shape[1] for _, g in stream), rate)
        log("bench: serving poisson", json.dumps(r))
        return r

    probes = []
    for i, f in enumerate(probe):
        probes.append(poisson(f * burst_qps, 100 + 2 * i))
        if probes[-1]["achieved_qps"] < 0.95 * probes[-1]["offered_qps"]:
            break
    ok = [r for r in probes if r["achieved_qps"] >= 0.95 * r["offered_qps"]]
    sustained = max(r["offered_qps"] for r in ok) if ok else probes[0]["offered_qps"]
    sweep = [dict(poisson(f * sustained, 200 + 2 * i), load_of_sustained=f) for i, f in enumerate(loads)]
    head = sweep[list(loads).index(0.7)] if 0.7 in loads else sweep[len(sweep) // 2]
    low = poisson(0.2 * sustained, 15, n_queries // 4)
    st = srv.stats()
    srv.close()
    return {"p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "load_of_sustained": 0.7,
            "offered_queries_per_s": head["offered_qps"], "achieved_queries_per_s": head["achieved_qps"],
            "configs_per_s": head["configs_per_s"],
            "hit_p50_ms": head["hit_p50_ms"], "hit_p99_ms": head["hit_p99_ms"],
            "miss_p50_ms": head["miss_p50_ms"], "miss_p99_ms": head["miss_p99_ms"],
            "misses": head["misses"], "hits": head["hits"], "traces_in_stream": head["traces"],
            "light_load": low, "sustained_queries_per_s": sustained, "burst": burst, "probes": probes,
            "sweep": sweep,
            "queries_per_stream": n_queries, "slots": n_slots, "warmup_trace_s": t_warm,
            "cache_bytes": int(cache_share * mix_bytes), "mix_channel_bytes": mix_bytes,
            "evictions": st["evictions"], "traces": st["traces"],
            "admission_waits": st["admission_waits"], "errors": st["errors"], "deployments": len(deps),
            "channel_cache_hits": st["channel_cache_hits"],
            "channel_cache_hit_rate": st["channel_cache_hits"] / max(1, st["channel_cache_hits"] + st["traces"]),
            "scene_triangles": sorted(int(s.n_tri) for s in scenes.values()),
            "receivers": sorted({int(d.rx_pos.shape[0]) for d in deps}),
            "ris_elements": sorted({int(riss[d.ris_key].elems.shape[0]) for d in deps})}


def cpu_baseline(n_rx_side=40, n_rays=1_000_000):
    """The oracle on a bounded sample of the lab-room workload: full discovery
    (1e6 rays per source, order 3) and image-method paths, legs and fields
    for a 40 x 40 receiver subsample of the same grid (about 15 s on 16
    host threads)."""
    from oracle import oracle as O
    from paper_2402_13034_amd import synth
    prob = synth.lab_room()
    sel = np.linspace(0, 63, n_rx_side).round().astype(int)
    idx = (sel[:, None] * 64 + sel[None, :]).ravel()
    prob.rx_pos = prob.rx_pos[idx]
    O.lib()
    O.leg_count()
    t0 = time.perf_counter()
    r = O.trace(prob, n_rays=n_rays)
    dt = time.perf_counter() - t0
    segs = r["segments"] + O.leg_count()
    return {"value": segs / dt / 1e6, "unit": "Mray-segments/s", "cores": O.threads(), "kind": "oracle",
            "sample": "lab room, full discovery (%d rays per source, order 3) + paths for %d receivers "
                      "(a %dx%d subsample of the 64x64 grid); %d segments in %.1f s"
                      % (n_rays, idx.size, n_rx_side, n_rx_side, segs, dt)}


def environment() -> dict:
    """Where the numbers were taken: device, software versions and host CPU."""
    import platform
    import torch
    p = torch.cuda.get_device_properties(0)
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"gpu": p.name, "gpu_arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "hbm_gib": round(p.total_memory / 2 ** 30, 1), "hip": torch.version.hip, "torch": torch.__version__,
            "host_cpu": cpu, "host_logical_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gemm", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the optional-feature lines (incoming reflections, Fresnel, impulse response, the "
                         "paper's scenario)")
    ap.add_argument("--no-large", action="store_true", help="skip the office-floor (order 5, 1e6 triangles) line")
    ap.add_argument("--large-only", action="store_true", help="only the office-floor line (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path runs on a single device (receivers would shard "
              "across GPUs without communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2402_13034_amd import risrt, synth
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration %d MiB read + %d MiB written" % (args.copy_calibration, args.copy_calibration))
        del src, dst
    prob = synth.lab_room()
    ctx = risrt.Context(0)
    if args.large_only:
        large = run_large_bench(ctx)
        log("bench: large", json.dumps(large))
        ctx.close()
        print(json.dumps({"large_scene": large}))
        return
    log("bench: lab room, %d triangles, M=%d, R=%d, K=%d, rays=%d" % (
        prob.scene.n_tri, prob.ris.elems.shape[0], prob.rx_pos.shape[0], prob.order, prob.n_rays))
    stats, dt, work, variants = run_trace_bench(ctx, prob, args.steps, args.warmup, not args.no_variants)
    paper = None
    if not args.no_variants:
        log("bench: variants %s" % json.dumps(variants))
        paper = run_paper_bench(ctx)
        log("bench: paper scenario %s" % json.dumps(paper))
    segs = sum(s["segments"] for s in stats)
    value = segs / dt / 1e6
    ms_step = dt / args.steps * 1e3
    log("bench: %.1f Mseg/s, %.2f ms/step" % (value, ms_step))
    st0 = stats[-1]
    ris_ms = sum(s["ms_stage"][5] for s in stats) / len(stats)
    units = dict(zip(["node", "tri", "contain", "pair", "leg"], work))
    flops = sum(FLOPS_PER[k] * units[k] for k in units)
    achieved = flops / (ris_ms * 1e-3) / 1e12
    flops_high = flops + (FLOPS_PER_PAIR_HIGH - FLOPS_PER["pair"]) * units["pair"]
    roofline = {"kernel": "k_ris (per-element image method + visibility legs + field)", "bound": "alu",
                "achieved": achieved, "peak": VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(),
                "launch_ms": ris_ms, "work_per_launch": units, "flops_per_unit": FLOPS_PER,
                "flops_per_launch": flops,
                "frac_at_300_per_pair": flops_high / (ris_ms * 1e-3) / 1e12 / VECTOR_PEAK_TFLOPS,
                "executed": measured_valu_share()}
    log("bench: k_ris %.3f ms, work %s -> %.2f TFLOP/s" % (ris_ms, units, achieved))
    large = None
    if not args.no_large:
        large = run_large_bench(ctx)
        log("bench: large", json.dumps(large))
    gemm = None
    if not args.no_gemm:
        gemm = run_gemm_bench(ctx)
        log("bench: RIS sum", json.dumps(gemm))
    serving = None
    if not args.no_serve:
        serving = run_serving_bench(ctx)
        log("bench: serving", json.dumps(serving))
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()
        log("bench: cpu", json.dumps(cpu))
    ctx.close()
    out = {
        "metric": "Mray-segments/s traced (order<=3) + RIS field TFLOP/s; p50/p99 query latency",
        "value": value,
        "unit": "Mray-segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 geometry, f64 image method / lengths / phase",
        "data": "synthetic",
        "config": {"workload": "lab room: 6x5x3 m, 20 furniture boxes (%d triangles), 127-element hex RIS, "
                               "horn Tx cos^8, 64x64 Rx grid at 1.2 m, order<=3, 1e6 rays per source"
                               % prob.scene.n_tri,
                   "segments_per_step": segs // args.steps,
                   "stage_ms": st0["stage_ms_all"],
                   "host_ms_scene_trace_sum_destroy": [round(float(np.mean([s["host_ms"][k] for s in stats])), 3)
                                                       for k in range(4)]},
        "roofline": roofline,
        "variants": variants,
        "paper_scenario": paper,
        "large_scene": large,
        "ris_sum": gemm,
        "serving": serving,
        "latency_p50_ms": serving["p50_ms"] if serving else None,
        "latency_p99_ms": serving["p99_ms"] if serving else None,
        "ris_field_tflops": gemm["bf16x2"]["tflops_complex_equiv"] if gemm else None,
        "cpu_baseline": cpu,
        "env": environment(),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
