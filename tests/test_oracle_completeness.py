"""Discovery completeness (ray-launched candidates against every surface
sequence, the plain definition) and the precision of the ray decisions
(FP32 against FP64) on the lab room and the tiny box, on the CPU."""
import numpy as np

from oracle import oracle as O
from oracle import reports
from paper_2402_13034_amd import synth


def test_sbr_finds_every_lab_room_path_order2():
    """Full discovery (10^6 rays per source) on the lab room: every
    environment path of order <= 2 of 16 receivers spread over the grid, and
    every RIS-centre sequence that leaves into the front half-space, is found;
    discovery never adds a path the exhaustive search does not have.  (The
    sequences it does not find start behind the RIS, where the element
    pattern is zero.)"""
    prob = synth.lab_room()
    rep = reports.completeness(prob, 2, reports.grid_sample(64, 4), prob.n_rays)
    assert rep["env"]["extra"] == 0 and rep["centre"]["extra"] == 0
    assert rep["env"]["missed"] == 0, rep["env"]["missed_examples"]
    assert rep["centre"]["front"]["missed"] == 0, rep["centre"]["front"]["missed_examples"]
    assert rep["env"]["paths"] > 300 and rep["centre"]["front"]["paths"] > 200


def test_fp64_decisions_change_nothing_on_the_tiny_box():
    """No marginal decision on the tiny box: hit lists, candidates and paths
    are the same with every ray decision in FP64."""
    prob = synth.tiny_box()
    a = O.trace(prob)
    with O.decisions_fp64():
        b = O.trace(prob)
    for k in ("hits_tx", "hits_u", "cand_tx", "cand_u", "env_rx", "env_seq", "env_tri", "u_seq", "ris_valid"):
        assert np.array_equal(a[k], b[k]), k


def test_fp64_decisions_lab_room_marginal_fraction():
    """Lab room, 10^5 rays per source: fewer than 1e-4 of the rays take a
    different hit at some bounce in FP64; the sampled receivers' paths are
    the same; rays that end early (a corner) do so in both precisions."""
    prob = synth.lab_room()
    rep = reports.decision_precision(prob, 100_000, reports.grid_sample(64, 3))
    for src in ("hits_tx", "hits_centre"):
        assert rep[src]["fraction"] < 1e-4, rep[src]
        assert rep[src]["escapes_fp32"] == rep[src]["escapes_fp64"]
    assert rep["paths"]["env"][2] == 0 and rep["paths"]["centre"][2] == 0
    assert rep["paths"].get("element", [0, 0, 0])[2] == 0


def test_escape_count_helper():
    hits = np.array([[1, 2, 3], [1, -1, -1], [-1, -1, -1], [4, 5, -1]], np.int32)
    assert reports.escapes(hits, 3) == 3
    assert reports.escapes(hits, 3, np.array([True, True, False, False])) == 1


def test_oracle_bvh_equals_brute_force():
    """The oracle's median-split BVH (for scenes too large for brute force)
    takes exactly the brute-force decisions: hit lists of both sources,
    candidates, paths, element-path validity and fields on the lab room."""
    prob = synth.lab_room(nx=6, ny=5)
    a = O.trace(prob, n_rays=60_000)
    with O.accelerated():
        b = O.trace(prob, n_rays=60_000)
    for k in ("hits_tx", "hits_u", "cand_tx", "cand_u", "env_rx", "env_seq", "env_tri", "u_seq", "ris_valid"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["H"], b["H"]) and np.array_equal(a["E_env"], b["E_env"])
    # a trace that reuses the oracle's own hit lists gives the same channel
    with O.accelerated():
        c = O.trace(prob, n_rays=60_000, hits=(a["hits_tx"], a["hits_u"]))
    assert np.array_equal(a["H"], c["H"]) and np.array_equal(a["cand_u"], c["cand_u"])
