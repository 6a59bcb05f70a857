"""Oracle for the RIS ray tracer: TEST INFRASTRUCTURE ONLY.

Plain FP64 reference of the method of "Ray Tracing Algorithm for
Reconfigurable Intelligent Surfaces" (arXiv 2402.13034).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it; the product path
never imports it.  It shares no code with the GPU library: geometry and
visibility are in ``rt_oracle.c`` (brute force, FP64 image method, FP32 ray
decisions), the field model is written out here in NumPy FP64.

Field model (Section II-A):
  eq. (1)/(2)/(3): power density and the Tx field at distance d;
  eq. (4): launch field  |E_t| = sqrt(2 eta0 P_t G_t F_t(theta_t));
  eq. (5)-(7): per element  sqrt(G F_in F_out d_y d_z / (4 pi)) Gamma_m
               e^{-j 2 pi d_t / lambda} / d_t;
  eq. (8): to the Rx  sqrt(G_r F_r(theta_r)) lambda / (4 pi d_r)
           e^{-j 2 pi d_r / lambda};
  eq. (9): coherent sum over elements and multipath components;
  eq. (10): P_r = |E_r|^2 / (2 eta0).
Readings where the paper is silent: eta0 = 120 pi exactly (as printed);
c = 299 792 458 m/s; a reflected component spreads as 1 / (total unfolded
length) (image source); a pattern value for theta >= 90 deg of a cos^q
pattern is 0 and a path with any zero pattern factor is not emitted; the
scalar per-triangle reflection coefficient multiplies once per bounce.
"""
from __future__ import annotations

import contextlib
import ctypes
import itertools
import math
import os
import subprocess
from typing import Dict, Optional

import numpy as np

C0 = 299_792_458.0
ETA0 = 120.0 * math.pi
EPS = 1e-4
KEY_BITS = 21

PAT_ISO = 0
PAT_COSPOW = 1
PAT_MONOPOLE = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB64_PATH = os.path.join(_HERE, "liboracle_fp64dec.so")
_libs = {}
_fp64 = False   # ray decisions in FP64 (the reference of the precision report), not the parity reading


def build(force: bool = False, fp64_decisions: bool = False) -> str:
    """Compile the C part of the oracle (gcc, FP64/FP32 IEEE, no contraction);
    fp64_decisions: the variant that takes the ray decisions in FP64."""
    path = _LIB64_PATH if fp64_decisions else _LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        if fp64_decisions:
            cmd.insert(1, "-DOR_FP64_DECISIONS")
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


_accel = False   # median-split BVH instead of testing every triangle (same results)


@contextlib.contextmanager
def accelerated():
    """Within the block the oracle's ray tests walk its own median-split BVH
    (built once per scene) instead of testing every triangle: the same
    decisions, for scenes too large for brute force."""
    global _accel
    old = _accel
    _accel = True
    try:
        yield
    finally:
        _accel = old
        for L in _libs.values():
            L.or_set_accel(1 if _accel else 0)


@contextlib.contextmanager
def decisions_fp64():
    """Within the block every oracle call takes its ray decisions (closest hit,
    reflection, blocked leg) in FP64 instead of FP32."""
    global _fp64
    old = _fp64
    _fp64 = True
    try:
        yield
    finally:
        _fp64 = old


def lib():
    L = _libs.get(_fp64)
    if L is None:
        path = build(fp64_decisions=_fp64)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.or_discover.restype = i64
        L.or_discover.argtypes = [P, P, i64, P, ctypes.c_int, P, i64, ctypes.c_int, P, P]
        L.or_find_paths.restype = i64
        L.or_find_paths.argtypes = [P, P, P, i64, P, P, i64, ctypes.c_int, P, i64, i64, P, P, P, P]
        L.or_ris_paths.restype = None
        L.or_ris_paths.argtypes = [P, P, P, i64, P, P, i64, P, i64, P, P, ctypes.c_int, P, P, P, P, P]
        L.or_leg_blocked.restype = ctypes.c_int
        L.or_leg_blocked.argtypes = [P, P, P, i64, P, P, i64, i64]
        L.or_contains.restype = ctypes.c_int
        L.or_contains.argtypes = [P, P, i64, P]
        L.or_fib_dir.restype = None
        L.or_fib_dir.argtypes = [i64, i64, P]
        L.or_leg_count.restype = i64
        L.or_leg_count.argtypes = []
        L.or_threads.restype = ctypes.c_int
        L.or_threads.argtypes = []
        L.or_set_accel.restype = None
        L.or_set_accel.argtypes = [ctypes.c_int]
        _libs[_fp64] = L
    L.or_set_accel(1 if _accel else 0)
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# geometry wrappers
# --------------------------------------------------------------------------
def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().or_threads())


def leg_count() -> int:
    """Visibility legs tested since the previous call."""
    return int(lib().or_leg_count())


def fib_dir(i: int, n: int) -> np.ndarray:
    out = np.zeros(3)
    lib().or_fib_dir(i, n, _p(out))
    return out


def leg_blocked(scene, A, B, skip_a: int = -1, skip_b: int = -1) -> bool:
    """Is the leg A -> B blocked?  skip_a / skip_b: surfaces of its end
    points (-1 for none)."""
    V = _c(scene.V, np.float32)
    T = _c(scene.T, np.int32)
    S = _c(scene.surf, np.int32)
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    return bool(lib().or_leg_blocked(_p(V), _p(T), _p(S), T.shape[0], _p(A), _p(B), skip_a, skip_b))


def contains(scene, tri: int, p) -> bool:
    V = _c(scene.V, np.float32)
    T = _c(scene.T, np.int32)
    p = _c(p, np.float64)
    return bool(lib().or_contains(_p(V), _p(T), tri, _p(p)))


def discover(scene, src, n_rays: int, K: int, hemi_normal=None):
    """Discovery rays from ``src``: returns (hits [rows, K], launched [rows],
    segments traced)."""
    V = _c(scene.V, np.float32)
    T = _c(scene.T, np.int32)
    src = _c(src, np.float64)
    hemi = hemi_normal is not None
    hn = _c(hemi_normal if hemi else np.zeros(3), np.float64)
    rows = 2 * n_rays if hemi else n_rays
    hits = np.empty((rows, K), np.int32)
    launched = np.empty(rows, np.uint8)
    segs = lib().or_discover(_p(V), _p(T), T.shape[0], _p(src), int(hemi), _p(hn),
                             n_rays, K, _p(hits), _p(launched))
    return hits, launched.astype(bool), int(segs)


def seq_key(seq) -> int:
    """Packed key of a triangle sequence: sum (t_i + 1) << (21 i); the empty
    sequence is 0.  Sorting by this key is the canonical candidate order."""
    k = 0
    for i, t in enumerate(seq):
        if t < 0:
            break
        k |= (int(t) + 1) << (KEY_BITS * i)
    return k


def key_seq(key: int, K: int):
    out = [-1] * K
    for i in range(K):
        v = (key >> (KEY_BITS * i)) & ((1 << KEY_BITS) - 1)
        if v == 0:
            break
        out[i] = v - 1
    return out


def surface_hits(scene, hits: np.ndarray) -> np.ndarray:
    """Triangle hit lists -> surface hit lists (-1 stays -1)."""
    out = np.full(hits.shape, -1, np.int32)
    ok = hits >= 0
    out[ok] = scene.surf[hits[ok]]
    return out


def candidates_from_hits(hits: np.ndarray, K: int) -> np.ndarray:
    """All distinct prefixes (length 1..K) of every (surface) hit list, plus
    the empty sequence, sorted by key.  Returns int32 [nc, K], -1 padded."""
    keys = {0}
    for row in hits:
        k = 0
        for i in range(K):
            t = int(row[i])
            if t < 0:
                break
            k |= (t + 1) << (KEY_BITS * i)
            keys.add(k)
    ks = sorted(keys)
    return np.asarray([key_seq(k, K) for k in ks], np.int32).reshape(len(ks), K)


def candidates_from_hits_np(hits: np.ndarray, K: int) -> np.ndarray:
    """Same set as candidates_from_hits, via numpy (large inputs).  The key
    sum (t_i + 1) 2^(21 i) is held as two 64-bit words (positions 0-2 and
    3-4) and sorted by the high word, then the low one: the order of the
    integer key."""
    h = hits.astype(np.int64)
    lo = [np.zeros(1, np.uint64)]
    hi = [np.zeros(1, np.uint64)]
    acc = np.zeros(h.shape[0], np.uint64)
    acc1 = np.zeros(h.shape[0], np.uint64)
    alive = np.ones(h.shape[0], bool)
    for i in range(K):
        alive &= h[:, i] >= 0
        v = np.where(alive, h[:, i] + 1, 0).astype(np.uint64)
        if i < 3:
            acc = acc | (v << np.uint64(KEY_BITS * i))
        else:
            acc1 = acc1 | (v << np.uint64(KEY_BITS * (i - 3)))
        lo.append(acc[alive])
        hi.append(acc1[alive])
    pairs = np.stack([np.concatenate(hi), np.concatenate(lo)], axis=1)
    u = np.unique(pairs, axis=0)   # rows in lexicographic order: high word, then low word
    out = np.full((u.shape[0], K), -1, np.int32)
    mask = np.uint64((1 << KEY_BITS) - 1)
    for i in range(K):
        w = u[:, 1] if i < 3 else u[:, 0]
        v = ((w >> np.uint64(KEY_BITS * (i if i < 3 else i - 3))) & mask).astype(np.int64)
        prev = out[:, i - 1] >= 0 if i > 0 else np.ones(u.shape[0], bool)
        out[:, i] = np.where((v > 0) & prev, v - 1, -1)
    return out


def exhaustive_candidates(n_surf: int, K: int) -> np.ndarray:
    """Every sequence of at most K surfaces with no immediate repeat, plus
    the empty sequence, in key order."""
    seqs = [[]]
    for k in range(1, K + 1):
        for s in itertools.product(range(n_surf), repeat=k):
            if any(s[i] == s[i + 1] for i in range(k - 1)):
                continue
            seqs.append(list(s))
    seqs.sort(key=seq_key)
    out = np.full((len(seqs), K), -1, np.int32)
    for i, s in enumerate(seqs):
        out[i, :len(s)] = s
    return out


def find_paths(scene, src, cands: np.ndarray, rx: np.ndarray, K: int):
    """Valid, unblocked paths src -> cand -> rx.  Returns (rx_idx, cand_idx,
    points [n, K, 3], triangles [n, K]) in (rx, candidate) order."""
    V = _c(scene.V, np.float32)
    T = _c(scene.T, np.int32)
    SF = _c(scene.surf, np.int32)
    S = _c(src, np.float64)
    cands = _c(cands, np.int32)
    rx = _c(rx, np.float64)
    cap = max(16, 8 * rx.shape[0])
    while True:
        o_rx = np.empty(cap, np.int32)
        o_c = np.empty(cap, np.int32)
        o_p = np.empty((cap, K, 3), np.float64)
        o_t = np.empty((cap, K), np.int32)
        n = lib().or_find_paths(_p(V), _p(T), _p(SF), T.shape[0], _p(S), _p(cands), cands.shape[0],
                                K, _p(rx), rx.shape[0], cap, _p(o_rx), _p(o_c), _p(o_p), _p(o_t))
        if n >= 0:
            return o_rx[:n].copy(), o_c[:n].copy(), o_p[:n].copy(), o_t[:n].copy()
        cap = -n


def ris_paths(scene, tx, elems, rx, uptr, useq, K: int, lit=None):
    """Out side of the RIS paths: for every slot (direct, then the sequences
    of V(rx)) and element, the image-method path m -> seq -> rx, valid and
    unblocked, for the elements a field reaches (the clear direct leg, or
    ``lit`` when the incoming reflections are modelled)."""
    lit_a = None if lit is None else _c(lit, np.uint8)
    V = _c(scene.V, np.float32)
    T = _c(scene.T, np.int32)
    SF = _c(scene.surf, np.int32)
    tx = _c(tx, np.float64)
    elems = _c(elems, np.float64)
    rx = _c(rx, np.float64)
    uptr = _c(uptr, np.int64)
    useq = _c(useq if useq.size else np.zeros((1, K), np.int32), np.int32)
    R, M = rx.shape[0], elems.shape[0]
    n_slots = int(uptr[-1]) + R
    valid = np.zeros((n_slots, M), np.uint8)
    pts = np.zeros((n_slots, M, K, 3), np.float64)
    tri = np.zeros((n_slots, M, K), np.int32)
    txm = np.zeros(M, np.uint8)
    lib().or_ris_paths(_p(V), _p(T), _p(SF), T.shape[0], _p(tx), _p(elems), M, _p(rx), R,
                       _p(uptr), _p(useq), K, _p(valid), _p(pts), _p(tri), _p(txm),
                       None if lit_a is None else _p(lit_a))
    return valid.astype(bool), pts, tri, txm.astype(bool)


# --------------------------------------------------------------------------
# antenna patterns (power patterns, normalised to 1 at the maximum)
# --------------------------------------------------------------------------
def pattern(kind: int, param: float, cos_t: np.ndarray, lam: float) -> np.ndarray:
    """F(theta) from cos(theta).
    ISO: 1.  COSPOW: cos^param for cos > 0, else 0 (eq. (11) with
    param = G_t/2 - 1, eq. (13) with param = 1).  MONOPOLE: eq. (12) with
    height h = param * lambda, 0 at theta = 0 and pi."""
    c = np.clip(np.asarray(cos_t, np.float64), -1.0, 1.0)
    if kind == PAT_ISO:
        return np.ones_like(c)
    if kind == PAT_COSPOW:
        return np.where(c > 0.0, np.power(np.maximum(c, 0.0), param), 0.0)
    if kind == PAT_MONOPOLE:
        kh = 2.0 * math.pi * param
        s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
        with np.errstate(divide="ignore", invalid="ignore"):
            f = ((np.cos(kh * c) - math.cos(kh)) / s) ** 2
        return np.where(s > 0.0, f, 0.0)
    raise ValueError(kind)


def pattern_on(kind: int, cos_t: np.ndarray) -> np.ndarray:
    """Whether F(theta) is nonzero, decided on the FP64 cosine itself rather
    than on the value of F (which can underflow): cos^p is zero exactly for
    cos <= 0, the monopole of eq. (12) exactly at theta = 0 and pi, the
    isotropic pattern never.  A path is emitted when every pattern on it is
    nonzero (reading 15: paths with a zero pattern factor are not emitted)."""
    c = np.clip(np.asarray(cos_t, np.float64), -1.0, 1.0)
    if kind == PAT_ISO:
        return np.ones(c.shape, bool)
    if kind == PAT_COSPOW:
        return c > 0.0
    if kind == PAT_MONOPOLE:
        return 1.0 - c * c > 0.0
    raise ValueError(kind)


def _cos_between(v: np.ndarray, axis: np.ndarray) -> np.ndarray:
    a = np.asarray(axis, np.float64)
    return (v @ a) / (np.linalg.norm(v, axis=-1) * np.linalg.norm(a))


def _phase(total_len: np.ndarray, lam: float) -> np.ndarray:
    """-2 pi frac(d / lambda): the phase of e^{-j 2 pi d / lambda}."""
    x = total_len / lam
    return -2.0 * math.pi * (x - np.floor(x))


def _chain(S: np.ndarray, P: np.ndarray, k: np.ndarray, X: np.ndarray):
    """Per path: total length, first-leg vector, vector from the Rx to the
    last point before it.  S, X: [n, 3]; P: [n, K, 3]; k: [n]."""
    n = X.shape[0]
    D = np.zeros(n)
    first = np.empty((n, 3))
    last = np.empty((n, 3))
    Kmax = P.shape[1] if P.ndim == 3 else 0
    for kk in range(0, Kmax + 1):
        sel = k == kk
        if not np.any(sel):
            continue
        pts = [S[sel]] + [P[sel, j] for j in range(kk)] + [X[sel]]
        for a, b in zip(pts[:-1], pts[1:]):
            D[sel] += np.linalg.norm(b - a, axis=1)
        first[sel] = pts[1] - pts[0]
        last[sel] = pts[-2] - pts[-1]
    return D, first, last


EPS0 = 8.8541878128e-12   # F/m


def fresnel(eps: np.ndarray, cos_i: np.ndarray, pol: int) -> np.ndarray:
    """Fresnel reflection coefficient of a half-space of complex relative
    permittivity eps for a plane wave from free space at incidence angle
    theta (cos_i = cos theta >= 0), Section II-B's specular reflection:
      TE (pol 1, E perpendicular to the plane of incidence):
        (cos - sqrt(eps - sin^2)) / (cos + sqrt(eps - sin^2));
      TM (pol 2, E in the plane of incidence):
        (eps cos - sqrt(eps - sin^2)) / (eps cos + sqrt(eps - sin^2)),
    principal square root (the transmitted wave decays into a lossy medium)."""
    c = np.asarray(cos_i, np.float64)
    e = np.asarray(eps, np.complex128)
    root = np.sqrt(e - (1.0 - c * c))
    if pol == 1:
        return (c - root) / (c + root)
    if pol == 2:
        return (e * c - root) / (e * c + root)
    raise ValueError(pol)


def material_eps(prob, tris: np.ndarray) -> np.ndarray:
    """Complex relative permittivity eps_r - j sigma / (omega eps0) of the
    triangles at the problem's frequency."""
    er = prob.mat_eps_r.astype(np.float64)[tris]
    sg = prob.mat_sigma.astype(np.float64)[tris]
    return er - 1j * sg / (2.0 * math.pi * prob.freq * EPS0)


def bounce_coefs(prob, S: np.ndarray, pts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Product over the bounces of a path of its reflection coefficients: the
    triangle's fixed coefficient, or with ``prob.fresnel`` the Fresnel
    coefficient of its material at the angle between the arriving leg
    (previous point -> reflection point) and the triangle's normal
    (e1 x e2 from its FP64 vertices).  S: [n, 3] path start; pts: [n, K, 3]."""
    if not prob.fresnel:
        return refl_product(prob.scene, tris)
    V = prob.scene.V.astype(np.float64)
    T = prob.scene.T
    n = tris.shape[0]
    out = np.ones(n, np.complex128)
    for j in range(tris.shape[1]):
        t = tris[:, j]
        sel = t >= 0
        if not np.any(sel):
            continue
        tt = t[sel]
        a, b, c = V[T[tt, 0]], V[T[tt, 1]], V[T[tt, 2]]
        nrm = np.cross(b - a, c - a)
        prev = S[sel] if j == 0 else pts[sel, j - 1]
        d = pts[sel, j] - prev
        cos_i = np.abs(np.sum(d * nrm, axis=1)) / (np.linalg.norm(d, axis=1) * np.linalg.norm(nrm, axis=1))
        out[sel] *= fresnel(material_eps(prob, tt), np.minimum(cos_i, 1.0), prob.fresnel)
    return out


def refl_product(scene, tris: np.ndarray) -> np.ndarray:
    """Product of the reflection coefficients of the triangles a path
    reflects on (-1 entries are no reflection)."""
    coef = scene.refl_re.astype(np.float64) + 1j * scene.refl_im.astype(np.float64)
    out = np.ones(tris.shape[0], np.complex128)
    if coef.size == 0:
        return out
    for j in range(tris.shape[1]):
        t = tris[:, j]
        out = out * np.where(t >= 0, coef[np.maximum(t, 0)], 1.0)
    return out


def env_amplitudes(prob, rx_idx, tris, pts):
    """Complex amplitudes of Tx -> environment -> Rx paths (eq. (3) written in
    the form of eq. (8)): A_t(v1) prod(R) S_r lambda / (4 pi D) e^{-jkD}."""
    lam = prob.wavelength
    n = rx_idx.shape[0]
    k = (tris >= 0).sum(axis=1)
    S = np.broadcast_to(prob.tx_pos, (n, 3))
    X = prob.rx_pos[rx_idx]
    D, first, last = _chain(S, pts, k, X)
    ct = _cos_between(first, prob.tx_ant.axis)
    cr = _cos_between(last, prob.rx_ant.axis)
    Ft = pattern(prob.tx_ant.pattern, prob.tx_ant.param, ct, lam)
    Fr = pattern(prob.rx_ant.pattern, prob.rx_ant.param, cr, lam)
    At = np.sqrt(2.0 * ETA0 * prob.tx_power_w * prob.tx_ant.gain * Ft)
    Sr = np.sqrt(prob.rx_ant.gain * Fr)
    a = At * bounce_coefs(prob, S, pts, tris) * Sr * lam / (4.0 * math.pi * D) * np.exp(1j * _phase(D, lam))
    emitted = pattern_on(prob.tx_ant.pattern, ct) & pattern_on(prob.rx_ant.pattern, cr)
    return a, D, emitted


def ris_incoming(prob, c_tx: np.ndarray):
    """Fields reaching every element from the Tx (Section II-B, supporting
    reflections: the image method from the Tx to the RIS, with the same
    centre-point restriction as on the out side).  The sequences tried per
    element are those valid and unblocked from the Tx to the RIS centre; the
    empty sequence is the direct leg.  Per element (eqs. (4)-(6) without
    Gamma_m, F_out and the element factor):
      T_m = sum_p A_t(v1_p) sqrt(F_in(p)) prod(R_p) e^{-jk d_p} / d_p,
    d_p the unfolded length, v1_p the departure and F_in the arrival
    direction of path p.  Returns T [M], lit [M] (some path emitted), the
    sequences valid at the centre (order >= 1), and per emitted path its
    element, sequence row (0 = direct, i = in_seq[i - 1]) and triangles."""
    sc = prob.scene
    K = prob.order
    ris = prob.ris
    lam = prob.wavelength
    M = ris.elems.shape[0]
    _, c_c, _, _ = find_paths(sc, prob.tx_pos, c_tx, ris.centre[None, :], K)
    in_seq = c_tx[c_c]
    in_seq = in_seq[(in_seq >= 0).sum(axis=1) >= 1]
    cands = np.concatenate([np.full((1, K), -1, np.int32), in_seq.astype(np.int32)], axis=0)
    m_idx, j_idx, pts, tris = find_paths(sc, prob.tx_pos, cands, ris.elems, K)
    n = m_idx.shape[0]
    k = (tris >= 0).sum(axis=1)
    D, first, last = _chain(np.broadcast_to(prob.tx_pos, (n, 3)), pts, k, ris.elems[m_idx])
    ct = _cos_between(first, prob.tx_ant.axis)
    ci = _cos_between(last, ris.normal)
    Ft = pattern(prob.tx_ant.pattern, prob.tx_ant.param, ct, lam)
    Fin = pattern(PAT_COSPOW, ris.q, ci, lam)
    At = np.sqrt(2.0 * ETA0 * prob.tx_power_w * prob.tx_ant.gain * Ft)
    a = (At * np.sqrt(Fin) * bounce_coefs(prob, np.broadcast_to(prob.tx_pos, (n, 3)), pts, tris) / D
         * np.exp(1j * _phase(D, lam)))
    on = pattern_on(prob.tx_ant.pattern, ct) & pattern_on(PAT_COSPOW, ci)
    T = np.zeros(M, np.complex128)
    np.add.at(T, m_idx[on], a[on])
    lit = np.zeros(M, bool)
    lit[m_idx[on]] = True
    return T, lit, in_seq, m_idx[on], j_idx[on], tris[on]


def ris_amplitudes_in(prob, T, rx_idx, m_idx, tris, pts):
    """Per-element channel with the incoming field T_m of ``ris_incoming``:
    T_m sqrt(G F_out d_y d_z / 4pi) prod(R) S_r lambda / (4 pi D_r) e^{-jk D_r}."""
    lam = prob.wavelength
    ris = prob.ris
    k = (tris >= 0).sum(axis=1)
    m = ris.elems[m_idx]
    X = prob.rx_pos[rx_idx]
    Dr, first, last = _chain(m, pts, k, X)
    co = _cos_between(first, ris.normal)
    cr = _cos_between(last, prob.rx_ant.axis)
    Fout = pattern(PAT_COSPOW, ris.q, co, lam)
    Fr = pattern(prob.rx_ant.pattern, prob.rx_ant.param, cr, lam)
    elem = np.sqrt(ris.gain * Fout * ris.dy * ris.dz / (4.0 * math.pi))
    Sr = np.sqrt(prob.rx_ant.gain * Fr)
    a = (T[m_idx] * elem * bounce_coefs(prob, m, pts, tris) * Sr * lam / (4.0 * math.pi * Dr)
         * np.exp(1j * _phase(Dr, lam)))
    emitted = pattern_on(PAT_COSPOW, co) & pattern_on(prob.rx_ant.pattern, cr)
    return a, Dr, emitted


def ris_amplitudes(prob, rx_idx, m_idx, tris, pts):
    """Per-element channel (eqs. (4), (7), (8) without Gamma_m):
    A_t(Tx->m) sqrt(G F_in F_out d_y d_z / 4pi) e^{-jk d_t} / d_t prod(R) S_r
    lambda / (4 pi D_r) e^{-jk D_r}."""
    lam = prob.wavelength
    ris = prob.ris
    k = (tris >= 0).sum(axis=1)
    m = ris.elems[m_idx]
    X = prob.rx_pos[rx_idx]
    Dr, first, last = _chain(m, pts, k, X)
    vt = m - prob.tx_pos[None, :]
    dt = np.linalg.norm(vt, axis=1)
    ct = _cos_between(vt, prob.tx_ant.axis)
    ci = _cos_between(-vt, ris.normal)
    co = _cos_between(first, ris.normal)
    cr = _cos_between(last, prob.rx_ant.axis)
    Ft = pattern(prob.tx_ant.pattern, prob.tx_ant.param, ct, lam)
    Fin = pattern(PAT_COSPOW, ris.q, ci, lam)
    Fout = pattern(PAT_COSPOW, ris.q, co, lam)
    Fr = pattern(prob.rx_ant.pattern, prob.rx_ant.param, cr, lam)
    At = np.sqrt(2.0 * ETA0 * prob.tx_power_w * prob.tx_ant.gain * Ft)
    elem = np.sqrt(ris.gain * Fin * Fout * ris.dy * ris.dz / (4.0 * math.pi))
    Sr = np.sqrt(prob.rx_ant.gain * Fr)
    a = (At * elem / dt * bounce_coefs(prob, m, pts, tris) * Sr * lam / (4.0 * math.pi * Dr)
         * np.exp(1j * _phase(dt + Dr, lam)))
    emitted = (pattern_on(prob.tx_ant.pattern, ct) & pattern_on(PAT_COSPOW, ci) & pattern_on(PAT_COSPOW, co)
               & pattern_on(prob.rx_ant.pattern, cr))
    return a, dt + Dr, emitted


# --------------------------------------------------------------------------
# the whole path
# --------------------------------------------------------------------------
def trace(prob, mode: str = "sbr", n_rays: Optional[int] = None, ris_in: bool = False,
          hits=None) -> Dict[str, np.ndarray]:
    """Channel of one problem.

    mode = "sbr": candidate surface sequences from spherical-Fibonacci
      discovery rays from the Tx (full sphere) and from the RIS centre
      (half-space in front of the RIS), n_rays per source;
    mode = "exhaustive": every sequence of at most K surfaces.
    Returns env paths (Tx -> Rx, order 0..K), the sequences V(rx) valid from
    the RIS centre, RIS slots and their validity, H [R, M] and E_env [R].
    ris_in: the field reaching each element also by reflections Tx ->
    surfaces -> m (``ris_incoming``; sequences of the Tx candidates valid at
    the RIS centre); otherwise by the direct leg alone.
    hits: (Tx hit lists, RIS-centre hit lists) of an earlier ``discover`` of
    the oracle with the same scene, sources and n_rays, reused instead of
    tracing the discovery rays again (large scenes).
    """
    K = prob.order
    sc = prob.scene
    n = prob.n_rays if n_rays is None else n_rays
    R = prob.rx_pos.shape[0]
    out: Dict[str, np.ndarray] = {}
    segs = 0
    if mode == "sbr":
        if hits is not None:
            h_tx, s1 = hits[0], 0
        else:
            h_tx, _, s1 = discover(sc, prob.tx_pos, n, K)
        out["hits_tx"] = h_tx
        c_tx = candidates_from_hits_np(surface_hits(sc, h_tx), K)
        segs += s1
        if prob.ris is not None:
            if hits is not None:
                h_u, s2 = hits[1], 0
                launched_u = (h_u >= 0).any(axis=1)
            else:
                h_u, launched_u, s2 = discover(sc, prob.ris.centre, n, K, hemi_normal=prob.ris.normal)
            out["hits_u"] = h_u
            out["launched_u"] = launched_u
            c_u = candidates_from_hits_np(surface_hits(sc, h_u), K)
            segs += s2
    elif mode == "exhaustive":
        c_tx = exhaustive_candidates(sc.n_surf, K)
        c_u = c_tx
    else:
        raise ValueError(mode)
    out["cand_tx"] = c_tx
    e_rx, e_c, e_pts, e_tri = find_paths(sc, prob.tx_pos, c_tx, prob.rx_pos, K)
    a_env, d_env, em = env_amplitudes(prob, e_rx, e_tri, e_pts)
    out["env_rx"] = e_rx[em]
    out["env_seq"] = c_tx[e_c][em]
    out["env_tri"] = e_tri[em]
    out["env_amp"] = a_env[em]
    out["env_len"] = d_env[em]
    out["env_pts"] = e_pts[em]
    E_env = np.zeros(R, np.complex128)
    np.add.at(E_env, e_rx[em], a_env[em])
    out["E_env"] = E_env
    if prob.ris is None:
        out["segments"] = segs
        return out
    out["cand_u"] = c_u
    u_rx, u_c, _, _ = find_paths(sc, prob.ris.centre, c_u, prob.rx_pos, K)
    u_seq = c_u[u_c]
    keep = (u_seq >= 0).sum(axis=1) >= 1
    u_rx, u_seq = u_rx[keep], u_seq[keep]
    uptr = np.zeros(R + 1, np.int64)
    np.add.at(uptr, u_rx + 1, 1)
    uptr = np.cumsum(uptr)
    out["u_rx"] = u_rx
    out["u_seq"] = u_seq
    out["uptr"] = uptr
    M = prob.ris.elems.shape[0]
    T_in = lit = None
    if ris_in:
        T_in, lit, in_seq, in_m, in_j, in_tri = ris_incoming(prob, c_tx)
        out["in_seq"] = in_seq
        out["in_m"] = in_m
        out["in_row"] = in_j
        out["in_tri"] = in_tri
        out["T_in"] = T_in
        out["lit"] = lit
    valid, pts, tri, txm = ris_paths(sc, prob.tx_pos, prob.ris.elems, prob.rx_pos, uptr, u_seq, K, lit)
    n_slots = valid.shape[0]
    slot_rx = np.repeat(np.arange(R), np.diff(uptr) + 1)
    slot_seq = np.full((n_slots, K), -1, np.int32)
    for r in range(R):
        base = uptr[r] + r
        cnt = uptr[r + 1] - uptr[r]
        slot_seq[base + 1: base + 1 + cnt] = u_seq[uptr[r]:uptr[r + 1]]
    sl, mm = np.nonzero(valid)
    if ris_in:
        a, dtot, em = ris_amplitudes_in(prob, T_in, slot_rx[sl], mm, tri[sl, mm], pts[sl, mm])
    else:
        a, dtot, em = ris_amplitudes(prob, slot_rx[sl], mm, tri[sl, mm], pts[sl, mm])
    H = np.zeros((R, M), np.complex128)
    np.add.at(H, (slot_rx[sl][em], mm[em]), a[em])
    emitted = np.zeros_like(valid)
    emitted[sl[em], mm[em]] = True
    out["ris_slot_rx"] = slot_rx
    out["ris_slot_seq"] = slot_seq
    out["ris_valid"] = emitted
    out["ris_tri"] = tri
    out["ris_amp"] = a[em]
    out["ris_amp_idx"] = np.stack([sl[em], mm[em]], axis=1)
    out["ris_len"] = dtot[em]
    out["txm_clear"] = txm
    out["H"] = H
    out["segments"] = segs
    return out


def cir(res, prob, gamma: np.ndarray, bin_s: float, n_bins: int) -> np.ndarray:
    """Delay-binned channel impulse response of one configuration from a
    ``trace`` result (direct incoming legs): bin b of receiver r sums the
    complex amplitudes of its paths with unfolded length d, b = floor(d / L),
    L = c bin_s; environment paths as traced, RIS paths of element m times
    gamma[m]; paths past the last bin are left out."""
    L = C0 * bin_s
    R = prob.rx_pos.shape[0]
    h = np.zeros((R, n_bins), np.complex128)
    b = np.floor(res["env_len"] / L).astype(np.int64)
    keep = b < n_bins
    np.add.at(h, (res["env_rx"][keep], b[keep]), res["env_amp"][keep])
    if prob.ris is not None and res["ris_amp"].size:
        sl, m = res["ris_amp_idx"][:, 0], res["ris_amp_idx"][:, 1]
        b = np.floor(res["ris_len"] / L).astype(np.int64)
        keep = b < n_bins
        np.add.at(h, (res["ris_slot_rx"][sl][keep], b[keep]), gamma[m[keep]] * res["ris_amp"][keep])
    return h


def ris_exact(prob, cands: np.ndarray):
    """The plain definition the centre-point heuristic approximates: for every
    element m, every sequence in ``cands`` is tried from m itself (no
    restriction to sequences valid from the RIS centre).  Returns H [R, M] and
    the number of emitted paths per (rx, m)."""
    K = prob.order
    R = prob.rx_pos.shape[0]
    M = prob.ris.elems.shape[0]
    H = np.zeros((R, M), np.complex128)
    count = np.zeros((R, M), np.int64)
    for m in range(M):
        if not leg_blocked(prob.scene, prob.tx_pos, prob.ris.elems[m]):
            rx, ci, pts, tri = find_paths(prob.scene, prob.ris.elems[m], cands, prob.rx_pos, K)
            a, _, em = ris_amplitudes(prob, rx, np.full(rx.shape[0], m), tri, pts)
            np.add.at(H, (rx[em], np.full(int(em.sum()), m)), a[em])
            np.add.at(count, (rx[em], np.full(int(em.sum()), m)), 1)
    return H, count


def ris_sum(E_env: np.ndarray, H: np.ndarray, gamma: np.ndarray, scale: float = 1.0):
    """eq. (9)/(10): E[r, c] = E_env[r] + scale * sum_m H[r, m] Gamma[m, c];
    P = |E|^2 / (2 eta0).  FP64."""
    E = E_env[:, None] + scale * (H.astype(np.complex128) @ gamma.astype(np.complex128))
    return E, np.abs(E) ** 2 / (2.0 * ETA0)


def ris_sum_loop(E_env, H, gamma, scale: float = 1.0):
    """The same sum as a plain triple loop (small sizes only)."""
    R, M = H.shape
    C = gamma.shape[1]
    E = np.zeros((R, C), np.complex128)
    for r in range(R):
        for c in range(C):
            acc = 0j
            for m in range(M):
                acc += complex(H[r, m]) * complex(gamma[m, c])
            E[r, c] = complex(E_env[r]) + scale * acc
    return E


def power(E) -> np.ndarray:
    return np.abs(E) ** 2 / (2.0 * ETA0)
