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
