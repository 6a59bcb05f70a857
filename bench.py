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
configurations) and the oracle timed on a bounded sample of the same
workload on the host cores.
"""
import argparse
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
FP64_VECTOR_PEAK_TFLOPS = 78.6


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


def run_trace_bench(ctx, prob, steps, warmup):
    import torch
    from paper_2402_13034_amd import risrt
    mesh = device_mesh(prob)
    rx = torch.from_numpy(prob.rx_pos).cuda()
    gamma = torch.from_numpy(prob.gamma.astype(np.complex64)).cuda()
    r = prob.ris
    ris = ctx.ris_create(r.elems, r.centre, r.normal, r.dy, r.dz, r.gain, r.q)
    P_out = torch.empty((prob.rx_pos.shape[0], gamma.shape[1]), dtype=torch.float32, device="cuda")

    def step():
        scene = ctx.scene_create(*mesh)
        ch, st = risrt.trace_problem(ctx, prob, scene, ris, rx=rx)
        ctx.ris_sum(ch, gamma, precision=risrt.PREC_VALU_F32, want_P=False, P_out=P_out)
        ctx.destroy(ch)
        ctx.destroy(scene)
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.destroy(ris)
    return stats, t1 - t0


def run_gemm_bench(ctx, reps=5):
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
    for name, prec in (("bf16x2", risrt.PREC_MFMA_BF16X2), ("valu_f32", risrt.PREC_VALU_F32)):
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
        out[name] = {"ms": ms, "tflops_complex_equiv": 8.0 * R * M * C / (ms * 1e-3) / 1e12,
                     "tflops_executed": (4.0 * R * M * C * (2 if prec == 1 else 1)) / (ms * 1e-3) / 1e12}
    for h in (ch, scene, ris):
        ctx.destroy(h)
    out["shape"] = {"R": R, "M": M, "C": C}
    return out


def cpu_baseline(n_rx_side=4, n_rays=1_000_000):
    """The oracle on a bounded sample of the lab-room workload: full discovery
    (1e6 rays per source, order 3) and image-method paths, legs and fields
    for a 4 x 4 receiver subsample of the same grid."""
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
    return {"value": segs / dt / 1e6, "unit": "Mray-segments/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": "lab room, full discovery (%d rays per source, order 3) + paths for %d receivers "
                      "(a %dx%d subsample of the 64x64 grid); %d segments in %.1f s"
                      % (n_rays, idx.size, n_rx_side, n_rx_side, segs, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gemm", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path runs on a single device (see DESIGN.md for how it "
              "would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2402_13034_amd import risrt, synth
    torch.cuda.set_device(0)
    prob = synth.lab_room()
    ctx = risrt.Context(0)
    log("bench: lab room, %d triangles, M=%d, R=%d, K=%d, rays=%d" % (
        prob.scene.n_tri, prob.ris.elems.shape[0], prob.rx_pos.shape[0], prob.order, prob.n_rays))
    stats, dt = run_trace_bench(ctx, prob, args.steps, args.warmup)
    segs = sum(s["segments"] for s in stats)
    value = segs / dt / 1e6
    ms_step = dt / args.steps * 1e3
    log("bench: %.1f Mseg/s, %.2f ms/step" % (value, ms_step))
    st0 = stats[-1]
    gemm = None
    if not args.no_gemm:
        gemm = run_gemm_bench(ctx)
        log("bench: RIS sum", json.dumps(gemm))
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
                   "stage_ms": st0["ms_stage"]},
        "ris_sum": gemm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
