"""The C ABI from plain C: `tests/native/capi_client.c` includes only
include/risrt.h and links only librisrt.so.  On the CPU it must compile as
C99 with every warning an error and link (every call it makes resolves); on
the GPU its channel must be the binding's, bit for bit, for the same problem."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from paper_2402_13034_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "capi_client.c")
LIB_DIR = os.path.join(ROOT, "paper_2402_13034_amd")


def _build(out_dir):
    if not os.path.exists(os.path.join(LIB_DIR, "librisrt.so")):
        pytest.skip("library not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = os.path.join(str(out_dir), "capi_client")
    cmd = [cc, "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           SRC, "-o", exe, "-L", LIB_DIR, "-lrisrt", "-Wl,-rpath," + LIB_DIR]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_client_compiles_and_links(tmp_path):
    assert os.path.exists(_build(tmp_path))


def _write_problem(path, prob):
    sc, ris = prob.scene, prob.ris
    with open(path, "wb") as f:
        np.array([sc.V.shape[0], sc.T.shape[0], ris.elems.shape[0], prob.rx_pos.shape[0], prob.n_rays, prob.order],
                 np.int64).tofile(f)
        np.ascontiguousarray(sc.V, np.float32).tofile(f)
        np.ascontiguousarray(sc.T, np.int32).tofile(f)
        np.ascontiguousarray(sc.surf, np.int32).tofile(f)
        np.ascontiguousarray(sc.refl_re, np.float32).tofile(f)
        np.ascontiguousarray(sc.refl_im, np.float32).tofile(f)
        np.ascontiguousarray(ris.elems, np.float64).tofile(f)
        np.array(list(ris.centre) + list(ris.normal) + [ris.dy, ris.dz, ris.gain, ris.q], np.float64).tofile(f)
        a = prob.tx_ant
        np.array(list(prob.tx_pos) + list(a.axis) + [prob.tx_power_w, a.gain, a.pattern, a.param],
                 np.float64).tofile(f)
        b = prob.rx_ant
        np.array(list(b.axis) + [b.gain, b.pattern, b.param], np.float64).tofile(f)
        np.array([prob.freq], np.float64).tofile(f)
        np.ascontiguousarray(prob.rx_pos, np.float64).tofile(f)


@pytest.mark.gpu
def test_c_client_channel_equals_binding(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_13034_amd import risrt
    exe = _build(tmp_path)
    prob = synth.tiny_box(order=2, n_rx=16, n_rays=20_000)
    _write_problem(tmp_path / "problem.bin", prob)
    print("case C client: tiny box, order 2, 16 receivers", file=sys.stderr, flush=True)
    r = subprocess.run([exe, str(tmp_path / "problem.bin"), str(tmp_path / "channel.bin")], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(tmp_path / "channel.bin", "rb").read()
    R, M, segments, n_env = np.frombuffer(raw[:32], np.int64)
    E_c = np.frombuffer(raw[32:32 + 8 * R], np.complex64)
    H_c = np.frombuffer(raw[32 + 8 * R:], np.complex64).reshape(R, M)
    with risrt.Context(0) as ctx:
        scene, ris = risrt.upload_problem(ctx, prob)
        ch, st = risrt.trace_problem(ctx, prob, scene, ris)
        E, H = ctx.channel_read(ch)
        for h in (ch, scene, ris):
            ctx.destroy(h)
    assert (R, M) == H.shape and segments == st["segments"] and n_env == st["n_env_paths"]
    assert E_c.tobytes() == E.tobytes() and H_c.tobytes() == H.tobytes()
