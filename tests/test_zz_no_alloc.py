"""rt_ris_sum_noalloc (the allocation-free sum, its split buffers in the
library's static per-device scratch) against rt_ris_sum on the same channel
and configurations: two calls in a row, the second with a smaller channel,
every precision; the context's pool and torch's allocator hold no more
memory after the calls; a sum larger than the scratch is refused."""
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


def _channel(ctx, prob, n_rays):
    from paper_2402_13034_amd import risrt
    scene, ris = risrt.upload_problem(ctx, prob)
    ch, _ = risrt.trace_problem(ctx, prob, scene, ris, n_rays=n_rays)
    ctx.destroy(scene)
    ctx.destroy(ris)
    return ch


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_noalloc_sum_equals_sum(ctx, precision):
    import torch
    from paper_2402_13034_amd import risrt
    big = _channel(ctx, synth.lab_room(nx=24, ny=20), 20_000)        # 480 receivers x 127 elements
    small = _channel(ctx, synth.tiny_box(n_rx=37), None)              # 37 receivers x 49 elements
    rng = np.random.default_rng(precision)
    for real in (True, False):
        cases = []
        for ch, C in ((big, 300), (small, 70)):
            R, M, _, _ = ctx.channel_info(ch)
            G = synth.gamma_binary(M, C, 1.0, rng) if real else synth.gamma_2bit(M, C, 1.0, rng)
            g = torch.from_numpy(G.astype(np.complex64)).cuda()
            E_ref, P_ref = ctx.ris_sum(ch, g, scale=0.9, gamma_is_real=real, precision=precision, want_E=True)
            E = torch.empty((R, C), dtype=torch.complex64, device="cuda")
            P = torch.empty((R, C), dtype=torch.float32, device="cuda")
            cases.append((ch, g, E, P, E_ref, P_ref))
        torch.cuda.synchronize()
        held = ctx.mem_info()[0]
        torch_held = torch.cuda.memory_allocated()
        # two calls in a row through the C ABI, the second on the smaller channel
        for ch, g, E, P, _, _ in cases:
            _say("case noalloc precision", precision, "real", real, "shape", tuple(E.shape))
            risrt.ris_sum_noalloc(ctx, ch, g, E_out=E, P_out=P, scale=0.9, gamma_is_real=real, precision=precision)
        torch.cuda.synchronize()
        assert ctx.mem_info()[0] == held
        assert torch.cuda.memory_allocated() == torch_held
        for ch, g, E, P, E_ref, P_ref in cases:
            assert torch.equal(E, E_ref) and torch.equal(P, P_ref)
    for h in (big, small):
        ctx.destroy(h)


def test_noalloc_refuses_a_sum_beyond_the_scratch(ctx):
    import torch
    from paper_2402_13034_amd import risrt
    R, M, C = 16384, 1024, 64   # H split alone: 2 x 32768 x 1024 x 2 B = 128 MiB > 64 MiB
    H = np.zeros((R, M), np.complex64)
    H[:, 0] = 1e-6
    ch = ctx.channel_create(np.zeros(R, np.complex64), H)
    g = torch.ones((M, C), dtype=torch.complex64, device="cuda")
    P = torch.empty((R, C), dtype=torch.float32, device="cuda")
    with pytest.raises(risrt.RtError) as e:
        risrt.ris_sum_noalloc(ctx, ch, g, P_out=P, gamma_is_real=True, precision=risrt.PREC_MFMA_BF16X2)
    assert e.value.status == risrt.RT_EUNSUPPORTED
    # the VALU sum needs no scratch at any size
    risrt.ris_sum_noalloc(ctx, ch, g, P_out=P, gamma_is_real=True, precision=risrt.PREC_VALU_F32)
    _, P_ref = ctx.ris_sum(ch, g, gamma_is_real=True, precision=risrt.PREC_VALU_F32)
    torch.cuda.synchronize()
    assert torch.equal(P, P_ref)
    ctx.destroy(ch)
