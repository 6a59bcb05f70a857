"""Error paths of the C ABI on the GPU: every invalid input returns its
status code (through the binding: RtError with that status) and leaves the
context usable; none may fault.  Also: a channel destroyed while a sum that
reads it is still queued keeps its memory until that sum is done."""
import math
import sys

import numpy as np
import pytest

from paper_2402_13034_amd import synth

pytestmark = pytest.mark.gpu


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


def _status(fn):
    from paper_2402_13034_amd import risrt
    with pytest.raises(risrt.RtError) as e:
        fn()
    return e.value.status


def _box():
    return synth.tiny_box(n_rx=4).scene


def _create(ctx, V, T, S, rr=None, ri=None):
    n = T.shape[0]
    rr = np.full(n, 0.5, np.float32) if rr is None else rr
    ri = np.zeros(n, np.float32) if ri is None else ri
    return ctx.scene_create(V, T, S, rr, ri)


def _still_works(ctx):
    """A valid scene and trace after the error: the context is intact."""
    from paper_2402_13034_amd import risrt
    prob = synth.tiny_box(n_rx=4)
    scene, ris = risrt.upload_problem(ctx, prob)
    ch, st = risrt.trace_problem(ctx, prob, scene, ris)
    assert st["n_env_paths"] == 4 * 7
    for h in (ch, scene, ris):
        ctx.destroy(h)


def test_scene_input_errors(ctx):
    from paper_2402_13034_amd import risrt
    sc = _box()
    V, T, S = sc.V.astype(np.float32), sc.T.astype(np.int32), sc.surf.astype(np.int32)
    cases = []
    v = V.copy()
    v[3, 1] = np.nan
    cases.append(("NaN vertex", v, T, S))
    v = V.copy()
    v[0, 0] = np.inf
    cases.append(("infinite vertex", v, T, S))
    t = T.copy()
    t[5, 2] = V.shape[0]
    cases.append(("vertex index past the end", V, t, S))
    t = T.copy()
    t[0, 0] = -1
    cases.append(("negative vertex index", V, t, S))
    s = S.copy()
    s[s == 2] = 7   # ids 0..6 with 2 unused
    cases.append(("gap in surface ids", V, T, s))
    s = S.copy()
    s[0] = T.shape[0] + 4
    cases.append(("surface id past n_tri", V, T, s))
    s = S.copy()
    s[1] = S[4]   # a triangle of one wall joins the surface of another wall
    cases.append(("non-coplanar surface", V, T, s))
    v = V.copy()
    t = T.copy()
    v = np.concatenate([v, v[:1]], axis=0)   # a duplicate of vertex 0
    first = int(np.flatnonzero(S == 3)[0])
    t[first] = [t[first][0], t[first][0], v.shape[0] - 1]   # zero area: no plane
    cases.append(("degenerate first triangle of a surface", v, t, S))
    for name, v, t, s in cases:
        _say("case", name)
        assert _status(lambda: _create(ctx, v, t, s)) == risrt.RT_EINVAL, name
    _still_works(ctx)


def test_trace_argument_errors(ctx):
    from paper_2402_13034_amd import risrt
    prob = synth.tiny_box(n_rx=4)
    scene, ris = risrt.upload_problem(ctx, prob)
    import dataclasses
    for K in (-1, risrt.MAX_ORDER + 1):
        _say("case order", K)
        p = dataclasses.replace(prob, order=K)
        assert _status(lambda: risrt.trace_problem(ctx, p, scene, ris)) == risrt.RT_EUNSUPPORTED
    _say("case unknown flag")
    assert _status(lambda: risrt.trace_problem(ctx, prob, scene, ris, flags=1 << 20)) == risrt.RT_EINVAL
    _say("case negative ray count")
    assert _status(lambda: risrt.trace_problem(ctx, prob, scene, ris, n_rays=-5)) == risrt.RT_EINVAL
    _say("case too many receivers (rejected before any work)")
    many = np.zeros((65535 * 64 + 1, 3))
    assert _status(lambda: risrt.trace_problem(ctx, prob, scene, ris, rx=many)) == risrt.RT_EUNSUPPORTED
    del many
    _say("case stale handles")
    assert _status(lambda: risrt.trace_problem(ctx, prob, scene + 1000, ris)) == risrt.RT_ENOTFOUND
    assert _status(lambda: risrt.trace_problem(ctx, prob, scene, ris + 1000)) == risrt.RT_ENOTFOUND
    assert _status(lambda: risrt.trace_problem(ctx, prob, ris, ris)) == risrt.RT_ENOTFOUND   # wrong kind
    _say("case impulse response of a channel without kept paths")
    ch, _ = risrt.trace_problem(ctx, prob, scene, ris)
    import torch
    g = torch.ones(prob.ris.elems.shape[0], dtype=torch.complex64, device="cuda")
    assert _status(lambda: ctx.cir(ch, g, 1e-9, 10)) == risrt.RT_EINVAL
    assert _status(lambda: ctx.ris_paths_read(ch)) == risrt.RT_EINVAL
    _say("case bad precision, host gamma")
    G = torch.ones((prob.ris.elems.shape[0], 3), dtype=torch.complex64, device="cuda")
    assert _status(lambda: ctx.ris_sum(ch, G, precision=7)) == risrt.RT_EINVAL
    assert _status(lambda: ctx.ris_sum(ch, G.cpu())) == risrt.RT_EINVAL
    ctx.destroy(ch)
    assert _status(lambda: ctx.destroy(ch)) == risrt.RT_ENOTFOUND
    for h in (scene, ris):
        ctx.destroy(h)
    _still_works(ctx)


def test_destroy_while_sum_queued(ctx):
    """The sum is enqueued on a side stream behind a long kernel, the channel
    is destroyed at once, and a new channel is created (it may take the
    released blocks if they were freed too early): the queued sum still
    reads the old channel and gives the result of an undisturbed run."""
    import torch
    from paper_2402_13034_amd import risrt
    rng = np.random.default_rng(3)
    R, M, C = 1024, 512, 256
    H = ((rng.normal(size=(R, M)) + 1j * rng.normal(size=(R, M))) * 1e-6).astype(np.complex64)
    E_env = (H[:, 0] * 0.3).astype(np.complex64)
    G = synth.gamma_2bit(M, C, 1.0, rng).astype(np.complex64)
    g = torch.from_numpy(G).cuda()
    ref_ch = ctx.channel_create(E_env, H)
    _, P_ref = ctx.ris_sum(ref_ch, g, precision=risrt.PREC_MFMA_BF16X2)
    torch.cuda.synchronize()
    P_ref = P_ref.cpu().numpy()
    ctx.destroy(ref_ch)
    s = torch.cuda.Stream()
    ch = ctx.channel_create(E_env, H, stream=s)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        big = torch.randn(4096, 4096, device="cuda")
        for _ in range(8):
            big = big @ big * 1e-2   # keeps the stream busy for a while
        _, P = ctx.ris_sum(ch, g, precision=risrt.PREC_MFMA_BF16X2, stream=s)
    ctx.destroy(ch)
    H2 = np.zeros_like(H)
    ch2 = ctx.channel_create(np.zeros_like(E_env), H2)
    s.synchronize()
    assert np.array_equal(P.cpu().numpy(), P_ref)
    ctx.destroy(ch2)


def test_split_rebuilt_while_other_stream_reads(ctx):
    """Two streams alternate number formats on one channel (each switch
    rebuilds the cached split of H); every result equals the single-stream
    result of its format."""
    import torch
    from paper_2402_13034_amd import risrt
    rng = np.random.default_rng(5)
    R, M, C = 700, 300, 500
    H = ((rng.normal(size=(R, M)) + 1j * rng.normal(size=(R, M))) * 1e-6).astype(np.complex64)
    E_env = (H[:, 0] * 0.3).astype(np.complex64)
    g = torch.from_numpy(synth.gamma_2bit(M, C, 1.0, rng).astype(np.complex64)).cuda()
    ch = ctx.channel_create(E_env, H)
    ref = {}
    for prec in (risrt.PREC_MFMA_BF16X2, risrt.PREC_MFMA_F16X2):
        _, P = ctx.ris_sum(ch, g, precision=prec)
        torch.cuda.synchronize()
        ref[prec] = P.cpu().numpy()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for i in range(8):
        prec = (risrt.PREC_MFMA_BF16X2, risrt.PREC_MFMA_F16X2)[i % 2]
        s = streams[i % 2]
        with torch.cuda.stream(s):
            _, P = ctx.ris_sum(ch, g, precision=prec, stream=s)
        outs.append((prec, P))
    torch.cuda.synchronize()
    for prec, P in outs:
        assert np.array_equal(P.cpu().numpy(), ref[prec])
    ctx.destroy(ch)



def test_out_of_budget_part_way_leaves_context_sound():
    """In one context, a channel held as ballast leaves 0.5 to 10 MiB of the
    budget free, so that traces run out of memory at different points (both
    branches' work already queued); each fails with RT_ENOMEM, and after the
    ballast is released the same context traces the problem bit-identically
    to its first trace."""
    from paper_2402_13034_amd import risrt
    prob = synth.lab_room(nx=16, ny=16)
    n_rays = 100_000
    failed = succeeded = 0
    with risrt.Context(0, mem_budget_bytes=96 << 20) as ctx:
        scene, ris = risrt.upload_problem(ctx, prob)
        ch, _ = risrt.trace_problem(ctx, prob, scene, ris, n_rays=n_rays)
        E_ref, H_ref = ctx.channel_read(ch)
        ctx.destroy(ch)
        for left_kib in (512, 1024, 2048, 3072, 4096, 5120, 6144, 8192):
            in_use, budget = ctx.mem_info()[:2]
            # allocations above 4 MiB are whole 2 MiB blocks: H is one such size, E_env (at most
            # 128 KiB here) takes a power-of-two block; about left_kib to left_kib + 2 MiB stay free
            h_bytes = (budget - in_use - (left_kib << 10) - (128 << 10)) // (2 << 20) * (2 << 20)
            rows = h_bytes // (8 * 1024)
            _say("case ballast leaving about %d KiB of the budget: %d x 1024 complex" % (left_kib, rows))
            ballast = ctx.channel_create(np.zeros(rows, np.complex64), np.zeros((rows, 1024), np.complex64))
            try:
                ch, _ = risrt.trace_problem(ctx, prob, scene, ris, n_rays=n_rays)
                ctx.destroy(ch)
                succeeded += 1
            except risrt.RtError as e:
                assert e.status == risrt.RT_ENOMEM, e
                failed += 1
            ctx.destroy(ballast)
            ch, _ = risrt.trace_problem(ctx, prob, scene, ris, n_rays=n_rays)
            E, H = ctx.channel_read(ch)
            ctx.destroy(ch)
            assert E.tobytes() == E_ref.tobytes() and H.tobytes() == H_ref.tobytes()
        for h in (scene, ris):
            ctx.destroy(h)
    _say("traces that ran out of budget: %d, that fit: %d" % (failed, succeeded))
    assert failed > 0
