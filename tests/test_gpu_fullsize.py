"""Full-size checks in the launch configuration the benchmark times.

* Lab room (1908 triangles, 1e6 discovery rays per source, order 3, 64 x 64
  receivers, 127 elements): every discovery hit list and the candidate sets
  bit-exact against the oracle; path lists, RIS validity and H for a sample
  of receivers (the oracle evaluates them one receiver at a time).
* Many-configuration sum (16384 receivers x 1024 elements x 4096 +-1
  configurations, channel from the box-room tracer): sampled rows against an
  FP64 product on the same FP32 channel; the error in dB (where
  P >= 1e-3 P_incoherent), in phase and as a normalised RMS is printed and
  bounded (0.1 dB).
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_13034_amd import synth
from tests.test_gpu_parity import check_ris_paths

pytestmark = pytest.mark.gpu
ETA0 = 120.0 * math.pi


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_13034_amd import risrt
    c = risrt.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_lab_room_full_size(ctx):
    from paper_2402_13034_amd import risrt
    prob = synth.lab_room()
    K, R, M = prob.order, prob.rx_pos.shape[0], prob.ris.elems.shape[0]
    _say("case lab_room full: rays", prob.n_rays, "R", R, "M", M)
    scene, ris = risrt.upload_problem(ctx, prob)
    ch, st = risrt.trace_problem(ctx, prob, scene, ris, flags=risrt.FLAG_KEEP_HITS | risrt.FLAG_KEEP_PATHS)
    hits_tx = ctx.hits_read(ch, 0, K)
    hits_u = ctx.hits_read(ch, 1, K)
    paths = ctx.paths_read(ch)
    E_env, H = ctx.channel_read(ch)
    c_tx = ctx.candidates_read(ch, 0)[:, :K]
    c_u = ctx.candidates_read(ch, 1)[:, :K]
    amp, length = ctx.ris_paths_read(ch)
    for h in (ch, scene, ris):
        ctx.destroy(h)
    # discovery: every ray, every bounce
    ref_tx, _, _ = O.discover(prob.scene, prob.tx_pos, prob.n_rays, K)
    assert np.array_equal(hits_tx, ref_tx)
    ref_u, _, _ = O.discover(prob.scene, prob.ris.centre, prob.n_rays, K, hemi_normal=prob.ris.normal)
    assert np.array_equal(hits_u, ref_u)
    assert np.array_equal(c_tx, O.candidates_from_hits_np(O.surface_hits(prob.scene, ref_tx), K))
    assert np.array_equal(c_u, O.candidates_from_hits_np(O.surface_hits(prob.scene, ref_u), K))
    # receivers sampled across the grid, first and last included
    sample = np.unique(np.concatenate([[0, R - 1], np.random.default_rng(4).choice(R, 510, replace=False)]))
    sub = synth.lab_room()
    sub.rx_pos = prob.rx_pos[sample]
    ref = O.trace(sub, n_rays=prob.n_rays)
    env = paths["env"]
    sel = np.isin(env["rx"], sample)
    remap = {int(r): i for i, r in enumerate(sample)}
    assert np.array_equal(np.array([remap[int(r)] for r in env["rx"][sel]]), ref["env_rx"])
    assert np.array_equal(env["seq"][sel][:, :K], ref["env_seq"])
    assert np.array_equal(env["tri"][sel][:, :K], ref["env_tri"])
    a_gpu = env["amp"][sel][:, 0] + 1j * env["amp"][sel][:, 1]
    assert np.max(np.abs(np.abs(a_gpu) ** 2 / np.abs(ref["env_amp"]) ** 2 - 1)) < 1e-4
    assert np.max(np.abs(np.angle(a_gpu / ref["env_amp"]))) < 1e-3
    useq = paths["useq"]
    sel_u = np.isin(useq[:, 0], sample)
    assert np.array_equal(useq[sel_u, 1:1 + K], ref["u_seq"])
    # RIS validity per (slot, element) for the sampled receivers
    counts = np.bincount(useq[:, 0], minlength=R)
    base = np.concatenate([[0], np.cumsum(counts)[:-1]]) + np.arange(R)
    gpu_rows = np.concatenate([np.arange(base[r], base[r] + counts[r] + 1) for r in sample])
    assert np.array_equal(paths["ris_valid"][gpu_rows], ref["ris_valid"])
    # every element path of those receivers one by one (power 1e-4, phase 1e-3 rad, length)
    check_ris_paths(amp[gpu_rows], length[gpu_rows], ref, paths["ris_valid"][gpu_rows])
    del amp, length
    # fields
    inc_e = np.zeros(len(sample))
    np.add.at(inc_e, ref["env_rx"], np.abs(ref["env_amp"]))
    scale_e = np.maximum(np.abs(ref["E_env"]) ** 2, 1e-3 * inc_e ** 2)
    assert np.max(np.abs(np.abs(E_env[sample]) ** 2 - np.abs(ref["E_env"]) ** 2) / scale_e) < 1e-4
    ee = np.abs(E_env[sample] - ref["E_env"]) ** 2 / scale_e
    assert ee.max() < 1e-6   # complex error: 1e-3 rad where |E|^2 >= 1e-3 of the incoherent sum
    sl, mm = ref["ris_amp_idx"][:, 0], ref["ris_amp_idx"][:, 1]
    inc = np.zeros((len(sample), M))
    np.add.at(inc, (ref["ris_slot_rx"][sl], mm), np.abs(ref["ris_amp"]))
    scale_h = np.maximum(np.abs(ref["H"]) ** 2, 1e-3 * inc ** 2)
    assert np.max(np.abs(np.abs(H[sample]) ** 2 - np.abs(ref["H"]) ** 2) / scale_h) < 1e-4
    he = np.abs(H[sample] - ref["H"]) ** 2 / scale_h
    assert he.max() < 1e-6
    _say("lab room full: %d segments, hits bit-exact (%d + %d rows), %d sampled receivers, max |dH|^2 rel %.2e"
         % (st["segments"], hits_tx.shape[0], hits_u.shape[0], len(sample), he.max()))


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_many_configuration_sum_full_size(ctx, prec):
    import torch
    from paper_2402_13034_amd import risrt
    prob = synth.precision_problem()
    R, M, C = prob.rx_pos.shape[0], prob.ris.elems.shape[0], prob.gamma.shape[1]
    _say("case precision full: R", R, "M", M, "C", C, "precision", prec)
    scene, ris = risrt.upload_problem(ctx, prob)
    ch, st = risrt.trace_problem(ctx, prob, scene, ris)
    E_env, H = ctx.channel_read(ch)
    s = np.sign(prob.gamma.real).astype(np.complex64)   # Gamma = 0.9 s
    g = torch.from_numpy(s).cuda()
    E, P = ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=prec, want_E=True, want_P=True)
    torch.cuda.synchronize()
    rows = np.random.default_rng(6).choice(R, 256, replace=False)
    rows_t = torch.from_numpy(rows).cuda()
    E_s = E[rows_t].cpu().numpy()
    P_s = P[rows_t].cpu().numpy()
    for h in (ch, scene, ris):
        ctx.destroy(h)
    E_ref, P_ref = O.ris_sum(E_env[rows].astype(np.complex128), H[rows].astype(np.complex128),
                             s.astype(np.complex128), 0.9)
    inc = (np.abs(E_env[rows]).astype(float)[:, None] + 0.9 * np.abs(H[rows]).astype(float) @ np.ones((M, C))) ** 2 \
        / (2 * ETA0)
    sel = P_ref >= 1e-3 * inc
    db = np.abs(10 * np.log10(P_s[sel] / P_ref[sel]))
    ph = np.abs(np.angle(E_s[sel] / E_ref[sel]))
    nrmse = math.sqrt(np.mean(np.abs(E_s - E_ref) ** 2) / np.mean(np.abs(E_ref) ** 2))
    _say("precision %d: max dB %.2e, p99 dB %.2e, max phase %.2e rad, NRMSE %.2e, %.1f%% of outputs above the "
         "null threshold" % (prec, db.max(), np.percentile(db, 99), ph.max(), nrmse, 100 * sel.mean()))
    assert db.max() < 0.1
    assert ph.max() < 1e-2
    assert nrmse < 1e-3
    # the channel itself against the oracle for a few receivers (end to end)
    sub = synth.precision_problem()
    pick = rows[:6]
    sub.rx_pos = prob.rx_pos[pick]
    ref = O.trace(sub)
    sl, mm = ref["ris_amp_idx"][:, 0], ref["ris_amp_idx"][:, 1]
    incH = np.zeros((len(pick), M))
    np.add.at(incH, (ref["ris_slot_rx"][sl], mm), np.abs(ref["ris_amp"]))
    he = np.abs(H[pick] - ref["H"]) ** 2 / np.maximum(np.abs(ref["H"]) ** 2, 1e-3 * incH ** 2)
    assert he.max() < 1e-6
