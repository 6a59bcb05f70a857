"""Serving workload: a mix of deployments over random box rooms and a
seeded query stream (configurations of uneven batch sizes).

Only builds inputs (geometry, receiver grids, random RIS configurations)."""
from __future__ import annotations

import math

import numpy as np

from . import synth
from .serve import Deployment


def serving_mix(seed: int = synth.BASE_SEED + 3, tri_targets=(1_000, 10_000, 50_000, 200_000),
                ris_rings=(3, 6, 10), ris_square=(32,), grids=(16, 32, 64, 128), orders=(1, 2, 3),
                n_deployments: int = 12, n_rays: int = 100_000):
    """Returns (scenes {key: Scene}, riss {key: Ris}, deployments [Deployment]).

    Scenes: random box rooms with furniture, triangle counts from
    `tri_targets`.  RIS: hexagonal (37 / 127 / 331 elements) or square (1024)
    at lambda/2 on the far wall.  Receiver grids n x n at 1.2 m.  Tx: horn
    cos^8 (G_t = 18) in a corner aimed at the RIS."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = synth.C0 / freq
    scenes, dims = {}, {}
    for i, t in enumerate(tri_targets):
        sc, d = synth.random_box_room(rng, t)
        scenes["room%d" % i] = sc
        dims["room%d" % i] = d
    riss = {}
    deps = []
    ris_kinds = [("hex", r) for r in ris_rings] + [("sq", s) for s in ris_square]
    for j in range(n_deployments):
        sk = "room%d" % (j % len(tri_targets))
        L, W, H = dims[sk]
        kind, size = ris_kinds[rng.integers(len(ris_kinds))]
        normal = np.array([-1.0, 0.0, 0.0])
        centre = np.array([L - 0.001, W / 2, 1.5])
        elems = synth.hex_ris(size, lam / 2, centre, normal) if kind == "hex" else \
            synth.square_ris(size, size, lam / 2, centre, normal)
        rk = "ris%d" % j
        riss[rk] = synth.Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
        n = int(grids[rng.integers(len(grids))])
        rx = synth.rx_grid(0.4, L - 0.4, n, 0.4, W - 0.4, n, 1.2, 3e-4, rng)
        tx = np.array([0.3, 0.3, 2.5])
        order = int(orders[rng.integers(len(orders))])
        deps.append(Deployment("dep%d" % j, sk, rk, tx, synth.unit(centre - tx), 0.01, 18.0, synth.PAT_COSPOW, 8.0,
                               rx, np.array([0.0, 0.0, 1.0]), 1.0, synth.PAT_ISO, 0.0, freq, order, n_rays))
    return scenes, riss, deps


# RIS sizes of the serving configuration: centred hexagonal arrays of 3..18
# rings (37, 61, ..., 1027 elements) and square 32 x 32 and 64 x 64 arrays
C4_HEX_RINGS = tuple(range(3, 19))
C4_SQUARES = (32, 64)
C4_GRIDS = (16, 32, 64, 128, 256)


def serving_mix_c4(seed: int = synth.BASE_SEED + 5, n_scenes: int = 16, n_deployments: int = 32,
                   tri_range=(1_000, 200_000), orders=(1, 2, 3), n_rays: int = 100_000,
                   max_rx_x_elems: int = 1 << 24):
    """The full serving configuration: `n_scenes` random box rooms with
    triangle counts log-uniform in `tri_range`; `n_deployments` deployments,
    each a scene, an RIS drawn from the hexagonal sizes 37..1027 and the
    32 x 32 and 64 x 64 squares, an n x n receiver grid (n in 16..256), a
    reflection order 1..3.  A grid is redrawn while receivers x elements
    exceed `max_rx_x_elems` (the channel of such a pair would be 128 MiB or
    more).  The last two deployments (the least frequent in a Zipf-like
    stream) are the extremes of the ranges: a 256 x 256 grid with the
    127-element array, and the 64 x 64 array with a 64 x 64 grid.  Returns
    (scenes, riss, deployments) as `serving_mix`."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = synth.C0 / freq
    scenes, dims = {}, {}
    lo, hi = math.log(tri_range[0]), math.log(tri_range[1])
    for i in range(n_scenes):
        t = int(math.exp(rng.uniform(lo, hi)))
        sc, d = synth.random_box_room(rng, t)
        scenes["room%d" % i] = sc
        dims["room%d" % i] = d
    kinds = [("hex", r) for r in C4_HEX_RINGS] + [("sq", s) for s in C4_SQUARES]
    riss, deps = {}, []
    for j in range(n_deployments):
        sk = "room%d" % rng.integers(n_scenes)
        L, W, H = dims[sk]
        kind, size = kinds[rng.integers(len(kinds))]
        last = n_deployments - 1 - j   # 1: the 256 x 256 grid, 0: the 64 x 64 array
        if last == 1:
            kind, size = "hex", 6
        elif last == 0:
            kind, size = "sq", 64
        normal = np.array([-1.0, 0.0, 0.0])
        centre = np.array([L - 0.001, W / 2, 1.5])
        elems = synth.hex_ris(size, lam / 2, centre, normal) if kind == "hex" else \
            synth.square_ris(size, size, lam / 2, centre, normal)
        rk = "ris%d" % j
        riss[rk] = synth.Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
        while True:
            n = int(C4_GRIDS[rng.integers(len(C4_GRIDS))])
            if last < 2:
                n = 256 if last == 1 else 64
            if n * n * elems.shape[0] <= max_rx_x_elems:
                break
        rx = synth.rx_grid(0.4, L - 0.4, n, 0.4, W - 0.4, n, 1.2, 3e-4, rng)
        tx = np.array([0.3, 0.3, 2.5])
        order = int(orders[rng.integers(len(orders))])
        deps.append(Deployment("dep%d" % j, sk, rk, tx, synth.unit(centre - tx), 0.01, 18.0, synth.PAT_COSPOW, 8.0,
                               rx, np.array([0.0, 0.0, 1.0]), 1.0, synth.PAT_ISO, 0.0, freq, order, n_rays))
    return scenes, riss, deps


def channel_bytes(dep, riss) -> int:
    """Device bytes of a deployment's cached channel: H (complex FP32) and its
    matrix-core split for real configurations (hi and lo, 16-bit, two rows per
    receiver), E_env."""
    R, M = dep.rx_pos.shape[0], riss[dep.ris_key].elems.shape[0]
    return R * M * 8 + 2 * 2 * (2 * R) * M + R * 8


def query_stream(deps, riss, n_queries: int, seed: int = 7, max_cols: int = 512, zipf_a: float = 1.3):
    """(deployment key, Gamma [M x C]) pairs: deployments drawn Zipf-like,
    C log-uniform in 1..max_cols, 2-bit phases of magnitude 0.9."""
    rng = np.random.default_rng(seed)
    w = 1.0 / np.arange(1, len(deps) + 1) ** zipf_a
    w /= w.sum()
    out = []
    for _ in range(n_queries):
        d = deps[rng.choice(len(deps), p=w)]
        M = riss[d.ris_key].elems.shape[0]
        C = int(np.exp(rng.uniform(0.0, math.log(max_cols))))
        out.append((d.key, synth.gamma_2bit(M, C, 0.9, rng).astype(np.complex64)))
    return out
