"""The large configuration at full size: the office floor (about 1.08e6
triangles, 5064 surfaces, 40 x 20 x 3 m, 200 rooms), reflections up to
order 5 (two-word candidate keys), 1e7 discovery rays per source, 256 x 256
receivers, a 64 x 64 RIS, and the 1024-configuration sum of its channel.

* every discovery hit list (2 x 1e7 rays, 5 bounces) bit-exact against the
  oracle's discovery, which walks its own median-split BVH;
* both candidate sets bit-exact against the oracle's prefixes of its hits;
* for receivers sampled in the RIS's room, its neighbours and far away:
  environment paths, RIS-centre sequences, element-path validity, every
  element path's amplitude and length, H and E_env against the oracle (its
  trace reuses its own hit lists), and H of the sampled trace equal bit for
  bit to those rows of the full trace;
* the 1024-configuration sum of the full channel on the matrix cores within
  0.1 dB of FP64 on sampled receivers.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_13034_amd import synth
from tests.test_gpu_parity import _close_complex, _incoherent, check_ris_paths

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


def test_office_floor_full_size(ctx):
    import copy
    import time
    import torch
    from paper_2402_13034_amd import risrt
    prob = synth.office_floor()
    K, R, M = prob.order, prob.rx_pos.shape[0], prob.ris.elems.shape[0]
    sc = prob.scene
    _say("case office floor full: triangles", sc.n_tri, "rays", prob.n_rays, "R", R, "M", M, "K", K)
    scene, ris = risrt.upload_problem(ctx, prob)
    info = ctx.scene_info(scene)
    _say("scene", info)
    t0 = time.time()
    ch, st = risrt.trace_problem(ctx, prob, scene, ris, flags=risrt.FLAG_KEEP_HITS)
    torch.cuda.synchronize()
    _say("gpu trace %.2f s: %d segments, %d + %d candidates, %d slots" % (
        time.time() - t0, st["segments"], st["n_cand_tx"], st["n_cand_u"], st["n_ris_slots"]))
    hits_tx = ctx.hits_read(ch, 0, K)
    hits_u = ctx.hits_read(ch, 1, K)
    c_tx = ctx.candidates_read(ch, 0)[:, :K]
    c_u = ctx.candidates_read(ch, 1)[:, :K]
    E_env, H = ctx.channel_read(ch)
    # the 1024-configuration sum of the full channel (65536 x 4096 x 1024) on the matrix cores
    C = 1024
    rng = np.random.default_rng(prob.seed + 9)
    s = (rng.integers(0, 2, size=(M, C)) * 2 - 1).astype(np.complex64)
    g = torch.from_numpy(s).cuda()
    Eo, Po = ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=True, precision=risrt.PREC_MFMA_BF16X2, want_E=True)
    torch.cuda.synchronize()
    rows = np.random.default_rng(3).choice(R, 128, replace=False)
    rows_t = torch.from_numpy(rows).cuda()
    Es = Eo[rows_t].cpu().numpy().astype(np.complex128)
    Ps = Po[rows_t].cpu().numpy().astype(np.float64)
    del Eo, Po
    ctx.destroy(ch)
    E_ref, P_ref = O.ris_sum(E_env[rows].astype(np.complex128), H[rows].astype(np.complex128),
                             s.astype(np.complex128), 0.9)
    inc = (np.abs(E_env[rows]).astype(float)[:, None] + 0.9 * np.abs(H[rows]).astype(float).sum(1)[:, None]) ** 2 \
        / (2 * ETA0)
    sel = (P_ref >= 1e-3 * inc) & (inc > 0)
    if sel.any():
        db = np.abs(10 * np.log10(Ps[sel] / P_ref[sel]))
        _say("sum: max dB %.2e on %d outputs above the null threshold" % (db.max(), sel.sum()))
        assert db.max() < 0.1
    # discovery: the oracle walks its own BVH; every ray, every bounce
    t0 = time.time()
    with O.accelerated():
        ref_tx, _, _ = O.discover(sc, prob.tx_pos, prob.n_rays, K)
        ref_u, _, _ = O.discover(sc, prob.ris.centre, prob.n_rays, K, hemi_normal=prob.ris.normal)
    _say("oracle discovery %.1f s on %d threads" % (time.time() - t0, O.threads()))
    assert np.array_equal(hits_tx, ref_tx)
    assert np.array_equal(hits_u, ref_u)
    del hits_tx, hits_u
    assert np.array_equal(c_tx, O.candidates_from_hits_np(O.surface_hits(sc, ref_tx), K))
    assert np.array_equal(c_u, O.candidates_from_hits_np(O.surface_hits(sc, ref_u), K))
    # receivers sampled in the RIS's room (x 8-10, y 8-10), its neighbours and far away
    xy = prob.rx_pos[:, :2]
    near = np.flatnonzero((xy[:, 0] > 8.1) & (xy[:, 0] < 9.9) & (xy[:, 1] > 8.1) & (xy[:, 1] < 9.9))
    mid = np.flatnonzero((xy[:, 0] > 6.1) & (xy[:, 0] < 12.0) & (xy[:, 1] > 6.1) & (xy[:, 1] < 12.0))
    pick = np.random.default_rng(8)
    sample = np.unique(np.concatenate([pick.choice(near, 4, replace=False), pick.choice(mid, 3, replace=False),
                                       pick.choice(R, 3, replace=False)]))
    sub = copy.copy(prob)
    sub.rx_pos = prob.rx_pos[sample]
    ch2, st2 = risrt.trace_problem(ctx, sub, scene, ris, flags=risrt.FLAG_KEEP_PATHS)
    p = ctx.paths_read(ch2)
    amp, length = ctx.ris_paths_read(ch2)
    E2, H2 = ctx.channel_read(ch2)
    for h in (ch2, scene, ris):
        ctx.destroy(h)
    assert np.array_equal(H2, H[sample]) and np.array_equal(E2, E_env[sample])
    t0 = time.time()
    with O.accelerated():
        ref = O.trace(sub, hits=(ref_tx, ref_u))
    _say("oracle paths for %d receivers %.1f s: %d env paths, %d centre sequences, %d element paths" % (
        len(sample), time.time() - t0, ref["env_rx"].shape[0], ref["u_seq"].shape[0], int(ref["ris_valid"].sum())))
    env = p["env"]
    assert np.array_equal(env["rx"], ref["env_rx"])
    assert np.array_equal(env["seq"][:, :K], ref["env_seq"])
    assert np.array_equal(env["tri"][:, :K], ref["env_tri"])
    a_gpu = env["amp"][:, 0] + 1j * env["amp"][:, 1]
    if a_gpu.size:
        assert np.max(np.abs(np.abs(a_gpu) ** 2 / np.abs(ref["env_amp"]) ** 2 - 1)) < 1e-4
        assert np.max(np.abs(np.angle(a_gpu / ref["env_amp"]))) < 1e-3
    assert np.array_equal(p["useq"][:, 0], ref["u_rx"])
    assert np.array_equal(p["useq"][:, 1:1 + K], ref["u_seq"])
    assert np.array_equal(p["ris_valid"], ref["ris_valid"])
    check_ris_paths(amp, length, ref, p["ris_valid"])
    n = len(sample)
    _close_complex(E2, ref["E_env"], _incoherent(ref["env_rx"], ref["env_amp"], n))
    sl, mm = ref["ris_amp_idx"][:, 0], ref["ris_amp_idx"][:, 1]
    _close_complex(H2, ref["H"], _incoherent((ref["ris_slot_rx"][sl], mm), ref["ris_amp"], (n, M)))
