"""Channel files (export / import of H and E_env): the reader accepts what the
writer's format states and rejects everything else, on the CPU."""
import json

import numpy as np
import pytest

from paper_2402_13034_amd import risrt


def _write(path, E, H, **meta):
    doc = dict(version=risrt.CHANNEL_FILE_VERSION, R=H.shape[0], M=H.shape[1] if H.ndim == 2 else -1)
    doc.update(meta)
    np.savez(path, E_env=E, H=H, meta=np.array(json.dumps(doc)))
    return str(path)


def _good(R=5, M=3, seed=0):
    rng = np.random.default_rng(seed)
    E = (rng.normal(size=R) + 1j * rng.normal(size=R)).astype(np.complex64)
    H = (rng.normal(size=(R, M)) + 1j * rng.normal(size=(R, M))).astype(np.complex64)
    return E, H


def test_reads_back_exactly(tmp_path):
    E, H = _good()
    p = _write(tmp_path / "ch.npz", E, H, scene_key="room0", order=2)
    E2, H2, meta = risrt.read_channel_file(p)
    assert E2.tobytes() == E.tobytes() and H2.tobytes() == H.tobytes()
    assert meta["scene_key"] == "room0" and meta["order"] == 2 and (meta["R"], meta["M"]) == (5, 3)


def test_empty_channel(tmp_path):
    E = np.zeros(0, np.complex64)
    H = np.zeros((0, 4), np.complex64)
    E2, H2, _ = risrt.read_channel_file(_write(tmp_path / "e.npz", E, H))
    assert E2.shape == (0,) and H2.shape == (0, 4)


@pytest.mark.parametrize("mistake", ["dtype", "rows", "meta_shape", "nan", "version", "missing", "pickled",
                                     "meta_not_json", "meta_not_object"])
def test_rejects(tmp_path, mistake):
    E, H = _good()
    p = tmp_path / "bad.npz"
    if mistake == "dtype":
        _write(p, E.astype(np.complex128), H)
    elif mistake == "rows":
        _write(p, E[:4], H)
    elif mistake == "meta_shape":
        _write(p, E, H, M=4)
    elif mistake == "nan":
        H[1, 2] = np.nan
        _write(p, E, H)
    elif mistake == "version":
        _write(p, E, H, version=99)
    elif mistake == "missing":
        np.savez(p, E_env=E, H=H)
    elif mistake == "pickled":
        np.savez(p, E_env=E, H=H, meta=np.array([{"version": 1}], dtype=object))
    elif mistake == "meta_not_json":
        np.savez(p, E_env=E, H=H, meta=np.array("{version: 1"))
    elif mistake == "meta_not_object":
        np.savez(p, E_env=E, H=H, meta=np.array(json.dumps([1, 5, 3])))
    with pytest.raises(ValueError):
        risrt.read_channel_file(str(p))


def test_deployment_metadata_is_json():
    from paper_2402_13034_amd import serve, synth
    rng = np.random.default_rng(1)
    d = serve.Deployment("d", "room0", "ris0", np.array([0.3, 0.3, 2.5]), np.array([1.0, 0.0, 0.0]), 0.01,
                         18.0, synth.PAT_COSPOW, 8.0, rng.uniform(size=(16, 3)), np.array([0.0, 0.0, 1.0]), 1.0,
                         synth.PAT_ISO, 0.0, 28e9, np.int64(2), 10_000)
    m = serve._dep_meta(d)
    back = json.loads(json.dumps(m))
    assert back == m and back["order"] == 2 and len(back["rx_pos_sha1"]) == 40 and "rx_pos" not in back
