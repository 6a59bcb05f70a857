"""Serving loop: results are the same alone and in a concurrent mix; the
loop admits by memory and reports latencies."""
import numpy as np
import pytest

from paper_2402_13034_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_13034_amd import workloads
    scenes, riss, deps = workloads.serving_mix(tri_targets=(1_000, 5_000), ris_rings=(3, 6), ris_square=(),
                                               grids=(8, 16), orders=(1, 2), n_deployments=4, n_rays=20_000)
    return scenes, riss, deps


def _server(ctx, mix, n_slots, cache_bytes=None):
    from paper_2402_13034_amd import serve
    scenes, riss, deps = mix
    s = serve.Server(ctx, n_slots=n_slots, cache_bytes=cache_bytes)
    for k, v in scenes.items():
        s.add_scene(k, v)
    for k, v in riss.items():
        s.add_ris(k, v)
    for d in deps:
        s.add_deployment(d)
    return s


def test_alone_equals_mix(mix):
    from paper_2402_13034_amd import risrt, serve, workloads
    scenes, riss, deps = mix
    qs = workloads.query_stream(deps, riss, 40, seed=3, max_cols=64)
    with risrt.Context(0) as ctx:
        alone = []
        s1 = _server(ctx, mix, 1)
        for dk, g in qs:
            alone.append(s1.submit(dk, g).result(timeout=120))
        s1.close()
        s4 = _server(ctx, mix, 4)
        futs = serve.run_poisson(s4, qs, rate_hz=2000.0, seed=1)
        mixed = [f.result(timeout=120) for f in futs]
        st = s4.stats()
        s4.close()
    for a, b in zip(alone, mixed):
        assert a.shape == b.shape
        assert a.tobytes() == b.tobytes()
    assert st["queries"] == len(qs) and st["errors"] == 0
    assert st["batches"] <= len(qs)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_evictions_retrace_bit_identical(mix):
    """A channel cache that holds one deployment's channel: a stream over four
    deployments evicts and traces again, and every answer is bit-identical to
    the one of a server whose cache holds them all; the misses (queries whose
    batch traced or waited for a trace) are counted and timed apart from the
    hits."""
    from paper_2402_13034_amd import risrt, serve, workloads
    scenes, riss, deps = mix
    qs = workloads.query_stream(deps, riss, 48, seed=21, max_cols=16, zipf_a=0.5)
    one = max(workloads.channel_bytes(d, riss) for d in deps)
    with risrt.Context(0) as ctx:
        big = _server(ctx, mix, 2)
        ref = [f.result(timeout=120) for f in serve.run_poisson(big, qs, rate_hz=3000.0, seed=4)]
        st_big = big.stats()
        big.close()
        small = _server(ctx, mix, 2, cache_bytes=one)
        got = [f.result(timeout=120) for f in serve.run_poisson(small, qs, rate_hz=3000.0, seed=4)]
        st = small.stats()
        small.close()
    for a, b in zip(ref, got):
        assert a.tobytes() == b.tobytes()
    assert st["errors"] == 0 and st["queries"] == len(qs)
    assert st_big["traces"] <= len(deps) and st_big["evictions"] == 0
    assert st["evictions"] > 0 and st["traces"] > st_big["traces"]
    assert st["misses"] >= st["traces"] - 1 and st["hits"] + st["misses"] == len(qs)
    assert st["miss_p50_ms"] is not None and st["miss_p99_ms"] >= st["miss_p50_ms"] > 0
    assert st["hits"] == 0 or st["hit_p99_ms"] >= st["hit_p50_ms"] > 0


def test_mix_matches_oracle_channel(mix):
    """One deployment's answers against the oracle's channel and FP64 sum."""
    from oracle import oracle as O
    from paper_2402_13034_amd import risrt, workloads
    scenes, riss, deps = mix
    d = deps[0]
    sc = scenes[d.scene_key]
    prob = synth.Problem("dep", sc, d.freq_hz, d.tx_pos, d.tx_power_w,
                         synth.Antenna(d.tx_axis, d.tx_gain, d.tx_pattern, d.tx_param), riss[d.ris_key],
                         d.rx_pos, synth.Antenna(d.rx_axis, d.rx_gain, d.rx_pattern, d.rx_param), d.order,
                         d.n_rays, 0)
    ref = O.trace(prob)
    rng = np.random.default_rng(5)
    g = synth.gamma_2bit(riss[d.ris_key].elems.shape[0], 33, 0.9, rng).astype(np.complex64)
    with risrt.Context(0) as ctx:
        s = _server(ctx, mix, 2)
        P = s.submit(d.key, g).result(timeout=120)
        s.close()
    E_ref, P_ref = O.ris_sum(ref["E_env"], ref["H"], g.astype(np.complex128))
    inc = (np.abs(ref["E_env"])[:, None] + np.abs(ref["H"]) @ np.abs(g).astype(float)) ** 2 / (2 * O.ETA0)
    sel = P_ref >= 1e-3 * inc
    assert np.max(np.abs(10 * np.log10(P[sel] / P_ref[sel]))) < 0.1


def test_small_budget_admission(mix):
    """A tight memory budget serialises work but every query completes; a
    query that cannot fit at all fails with RT_ENOMEM."""
    from paper_2402_13034_amd import risrt, serve, workloads
    scenes, riss, deps = mix
    qs = workloads.query_stream(deps, riss, 12, seed=9, max_cols=32)
    with risrt.Context(0, mem_budget_bytes=96 << 20) as ctx:
        s = _server(ctx, mix, 4)
        futs = serve.run_poisson(s, qs, rate_hz=5000.0, seed=2)
        res = [f.result(timeout=120) for f in futs]
        st = s.stats()
        s.close()
        assert len(res) == len(qs) and st["errors"] == 0
    with risrt.Context(0, mem_budget_bytes=1 << 20) as ctx:
        s = _server(ctx, mix, 2)
        f = s.submit(deps[0].key, qs[0][1] if qs[0][0] == deps[0].key else
                     synth.gamma_2bit(riss[deps[0].ris_key].elems.shape[0], 4, 0.9,
                                      np.random.default_rng(0)).astype(np.complex64))
        with pytest.raises(risrt.RtError) as ei:
            f.result(timeout=120)
        assert ei.value.status == risrt.RT_ENOMEM
        s.close()


def test_context_before_torch_in_a_fresh_process():
    """A context opened before the caller touches torch: torch still finds the
    device and a server (torch streams) runs a query."""
    import os
    import subprocess
    import sys
    code = (
        "from paper_2402_13034_amd import risrt, serve\n"
        "ctx = risrt.Context(0)\n"
        "import torch\n"
        "x = torch.zeros(4, device='cuda')\n"
        "srv = serve.Server(ctx, n_slots=1)\n"
        "torch.cuda.synchronize()\n"
        "print('ok', float(x.sum()))\n"
        "srv.close()\n"
        "ctx.close()\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0 and "ok 0.0" in r.stdout, r.stderr[-2000:]


def test_channel_file_round_trip(mix, tmp_path):
    """A traced channel written to a file and read back is bit-identical, and
    its sums are too."""
    import torch
    from paper_2402_13034_amd import risrt, synth
    scenes, riss, deps = mix
    d = deps[1]
    with risrt.Context(0) as ctx:
        s = _server(ctx, mix, 1)
        path = s.export_channel(d.key, str(tmp_path / "dep1"))
        s.close()
        ch, meta = risrt.channel_load(ctx, path)
        E, H = ctx.channel_read(ch)
        # trace the same deployment again: the library is deterministic
        sc, r = scenes[d.scene_key], riss[d.ris_key]
        scene = ctx.scene_create(sc.V, sc.T, sc.surf, sc.refl_re, sc.refl_im)
        ris = ctx.ris_create(r.elems, r.centre, r.normal, r.dy, r.dz, r.gain, r.q)
        ch2, _ = ctx.trace(scene, ris, d.tx_pos, d.tx_axis, d.tx_power_w, d.tx_gain, d.tx_pattern, d.tx_param,
                           d.rx_pos, d.rx_axis, d.rx_gain, d.rx_pattern, d.rx_param, d.freq_hz, d.order, d.n_rays)
        E2, H2 = ctx.channel_read(ch2)
        g = torch.from_numpy(synth.gamma_2bit(r.elems.shape[0], 20, 0.9, np.random.default_rng(2))
                             .astype(np.complex64)).cuda()
        _, P1 = ctx.ris_sum(ch, g, want_P=True)
        _, P2 = ctx.ris_sum(ch2, g, want_P=True)
        same = P1.cpu().numpy().tobytes() == P2.cpu().numpy().tobytes()
        for h in (ch, ch2, scene, ris):
            ctx.destroy(h)
    assert E.tobytes() == E2.tobytes() and H.tobytes() == H2.tobytes() and same
    assert meta["order"] == d.order and meta["scene_key"] == d.scene_key and (meta["R"], meta["M"]) == H.shape


def test_warm_start_from_files_and_query_log(mix, tmp_path):
    """Channels exported by one server and imported into a fresh one answer
    every query bit-identically with no trace; each server's JSON log has one
    line per query, consistent with its statistics."""
    import json
    from paper_2402_13034_amd import risrt, serve, workloads
    scenes, riss, deps = mix
    qs = workloads.query_stream(deps, riss, 32, seed=11, max_cols=16)
    log_a, log_b = tmp_path / "a.jsonl", tmp_path / "b.jsonl"
    with risrt.Context(0) as ctx:
        a = serve.Server(ctx, n_slots=2, log=str(log_a))
        for k, v in scenes.items():
            a.add_scene(k, v)
        for k, v in riss.items():
            a.add_ris(k, v)
        for d in deps:
            a.add_deployment(d)
        ref = [f.result(timeout=120) for f in serve.run_poisson(a, qs, rate_hz=2000.0, seed=3)]
        st_a = a.stats()
        paths = {d.key: a.export_channel(d.key, str(tmp_path / d.key)) for d in deps}
        a.close()
        b = serve.Server(ctx, n_slots=2, log=str(log_b))
        for k, v in riss.items():
            b.add_ris(k, v)    # no scenes: a trace would fail
        for d in deps:
            b.add_deployment(d)
            b.import_channel(d.key, paths[d.key])
        got = [f.result(timeout=120) for f in serve.run_poisson(b, qs, rate_hz=2000.0, seed=3)]
        st_b = b.stats()
        # a channel of another deployment's shape is refused
        other = next(d for d in deps if d.rx_pos.shape[0] != deps[0].rx_pos.shape[0]
                     or riss[d.ris_key].elems.shape[0] != riss[deps[0].ris_key].elems.shape[0])
        with pytest.raises(ValueError):
            b.import_channel(deps[0].key, paths[other.key])
        b.close()
    for x, y in zip(ref, got):
        assert x.tobytes() == y.tobytes()
    assert st_b["traces"] == 0 and st_b["misses"] == 0 and st_b["errors"] == 0
    la = [json.loads(line) for line in log_a.read_text().splitlines()]
    lb = [json.loads(line) for line in log_b.read_text().splitlines()]
    assert len(la) == len(qs) == len(lb)
    assert sorted(r["qid"] for r in la) == list(range(len(qs)))
    assert sum(r["cache"] == "miss" for r in la) == st_a["misses"] and all(r["cache"] == "hit" for r in lb)
    assert sum(r["segments_traced"] > 0 for r in la) >= st_a["traces"] > 0
    assert all(r["segments_traced"] == 0 for r in lb)
    for r, (dk, g) in zip(sorted(la, key=lambda r: r["qid"]), qs):
        assert r["deployment"] == dk and r["columns"] == g.shape[1]
        assert r["latency_ms"] >= r["queue_ms"] >= 0 and r["batch_columns"] >= r["columns"]
        assert r["bytes_out"] == 4 * g.shape[1] * next(d.rx_pos.shape[0] for d in deps if d.key == dk)
