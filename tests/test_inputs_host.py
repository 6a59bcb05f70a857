"""Host checks of the synthetic inputs: every generated scene meets the
library's input contract (surface ids 0..n_surf-1, each used; the triangles
of a surface coplanar to within 0.1 mm of its first triangle's plane; finite
vertices and in-range indices), so a GPU run rejects none of them."""
import numpy as np
import pytest

from paper_2402_13034_amd import synth, workloads


def _check_scene(sc):
    V = sc.V.astype(np.float64)
    T = sc.T
    assert np.all(np.isfinite(V))
    assert T.size == 0 or (T.min() >= 0 and T.max() < V.shape[0])
    if sc.n_tri == 0:
        return
    ids = np.unique(sc.surf)
    assert ids[0] == 0 and ids[-1] == ids.size - 1
    for s in ids:
        tris = np.flatnonzero(sc.surf == s)
        a, b, c = V[T[tris[0]]]
        n = np.cross(b - a, c - a)
        nl = np.linalg.norm(n)
        assert nl > 0
        d = np.abs((V[T[tris]].reshape(-1, 3) - a) @ n) / nl
        assert d.max() <= 1e-4, (s, d.max())


@pytest.mark.parametrize("make", [
    lambda: synth.tiny_box().scene,
    lambda: synth.lab_room().scene,
    lambda: synth.lab_room(sub=5).scene,
    lambda: synth.wide_ris_room().scene,
    lambda: synth.precision_problem(n_cfg=1).scene,
    lambda: synth.paper_room(reflective=True).scene,
    lambda: synth.paper_room(reflective=False).scene,
    lambda: synth.deep_tree_room().scene,
    lambda: synth.office_floor(n_rx=2).scene,
])
def test_generated_scenes_meet_the_input_contract(make):
    _check_scene(make())


def test_serving_scenes_meet_the_input_contract():
    scenes, _, _ = workloads.serving_mix()
    for sc in scenes.values():
        _check_scene(sc)


def test_full_serving_mix_spans_the_configuration():
    """The full serving mix: 16 rooms of 1k-200k triangles meeting the input
    contract; RIS sizes from 37 to 4096 elements, grids from 16^2 to 256^2,
    orders 1-3; no deployment above 2^24 receivers x elements."""
    scenes, riss, deps = workloads.serving_mix_c4()
    assert len(scenes) == 16 and len(deps) == 32
    tris = [sc.n_tri for sc in scenes.values()]
    assert 1_000 <= min(tris) and max(tris) <= 200_000
    for sc in scenes.values():
        _check_scene(sc)
    R = [d.rx_pos.shape[0] for d in deps]
    M = [riss[d.ris_key].elems.shape[0] for d in deps]
    assert max(R) == 256 * 256 and min(R) >= 16 * 16
    assert max(M) == 4096 and min(M) >= 37
    assert {d.order for d in deps} <= {1, 2, 3}
    assert all(r * m <= 1 << 24 for r, m in zip(R, M))
