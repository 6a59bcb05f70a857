"""Seeded synthetic inputs for the RIS ray tracer.

This module only builds inputs: triangle meshes of rooms and boxes, RIS
element layouts, receiver grids and RIS configurations.  It holds none of the
method's arithmetic (no ray tracing, image method or field evaluation), so
that the oracle and the GPU path can both be fed from it without sharing any
computation.

Conventions
-----------
* Vertices are float32 (``V[n_v, 3]``), triangles int32 (``T[n_t, 3]``).
* Every rectangular face is cut into ``sub x sub`` quads and every quad into
  two triangles along the same diagonal.  Each face is one *surface*
  (``surf[n_t]``, int32): the set of coplanar triangles that the image method
  treats as one planar reflector.
* Positions of sources, receivers and RIS elements are float64.
* A complex reflection coefficient per triangle is stored as two float32
  arrays (``refl_re``, ``refl_im``).
* The RIS is not part of the mesh: its elements sit 1 mm in front of the wall
  that carries them (Section III-A of the paper places a finite RIS in an
  opening of a wall; here the wall stays closed and the elements are free
  points in front of it).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

C0 = 299_792_458.0
BASE_SEED = 2402_13034

PAT_ISO = 0
PAT_COSPOW = 1
PAT_MONOPOLE = 2


@dataclasses.dataclass
class Antenna:
    """An antenna: gain (linear), pattern kind and pattern parameter.

    pattern = PAT_ISO: F = 1; PAT_COSPOW: F = cos^param(theta);
    PAT_MONOPOLE: quarter-wave style monopole of height param * lambda.
    ``axis`` is the pattern's z axis (boresight for a horn, wire axis for a
    monopole).
    """
    axis: np.ndarray
    gain: float = 1.0
    pattern: int = PAT_ISO
    param: float = 0.0


@dataclasses.dataclass
class Ris:
    elems: np.ndarray          # float64 [M, 3]
    normal: np.ndarray         # float64 [3], unit, pointing into the room
    centre: np.ndarray         # float64 [3]
    dy: float
    dz: float
    gain: float                # element gain G (linear)
    q: float                   # element power pattern cos^q(theta)


@dataclasses.dataclass
class Scene:
    V: np.ndarray              # float32 [n_v, 3]
    T: np.ndarray              # int32 [n_t, 3]
    refl_re: np.ndarray        # float32 [n_t]
    refl_im: np.ndarray        # float32 [n_t]
    surf: np.ndarray           # int32 [n_t], surface id of each triangle

    @property
    def n_tri(self) -> int:
        return int(self.T.shape[0])

    @property
    def n_surf(self) -> int:
        return int(self.surf.max()) + 1 if self.surf.size else 0


@dataclasses.dataclass
class Problem:
    name: str
    scene: Scene
    freq: float
    tx_pos: np.ndarray         # float64 [3]
    tx_power_w: float
    tx_ant: Antenna
    ris: Optional[Ris]
    rx_pos: np.ndarray         # float64 [R, 3]
    rx_ant: Antenna
    order: int
    n_rays: int
    seed: int
    gamma: Optional[np.ndarray] = None   # complex128 [M, C]
    # Fresnel reflection instead of the fixed coefficients: 0 off, 1 TE, 2 TM,
    # with a material per triangle (relative permittivity, conductivity S/m)
    fresnel: int = 0
    mat_eps_r: Optional[np.ndarray] = None   # float32 [n_t]
    mat_sigma: Optional[np.ndarray] = None   # float32 [n_t]

    @property
    def wavelength(self) -> float:
        return C0 / self.freq


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
class MeshBuilder:
    def __init__(self) -> None:
        self.verts: list = []
        self.tris: list = []
        self.coef: list = []
        self.surf: list = []
        self.n_surf = 0

    def quad(self, p0, pu, pv, sub: int, coef: complex) -> None:
        """Rectangle p0 + a*pu + b*pv, a, b in [0, 1], cut into sub x sub
        quads, each split along its (0,0)-(1,1) diagonal."""
        p0 = np.asarray(p0, np.float64)
        pu = np.asarray(pu, np.float64)
        pv = np.asarray(pv, np.float64)
        sid = self.n_surf
        self.n_surf += 1
        for i in range(sub):
            for j in range(sub):
                a0, a1 = i / sub, (i + 1) / sub
                b0, b1 = j / sub, (j + 1) / sub
                c00 = p0 + a0 * pu + b0 * pv
                c10 = p0 + a1 * pu + b0 * pv
                c11 = p0 + a1 * pu + b1 * pv
                c01 = p0 + a0 * pu + b1 * pv
                base = len(self.verts)
                self.verts.extend([c00, c10, c11, c01])
                self.tris.append((base, base + 1, base + 2))
                self.tris.append((base, base + 2, base + 3))
                self.coef.extend([coef, coef])
                self.surf.extend([sid, sid])

    def box(self, lo, hi, sub: int, coef: complex, bottom: bool = True,
            top: bool = True) -> None:
        x0, y0, z0 = lo
        x1, y1, z1 = hi
        dx, dy, dz = x1 - x0, y1 - y0, z1 - z0
        self.quad((x0, y0, z0), (0, dy, 0), (0, 0, dz), sub, coef)   # x = x0
        self.quad((x1, y0, z0), (0, dy, 0), (0, 0, dz), sub, coef)   # x = x1
        self.quad((x0, y0, z0), (dx, 0, 0), (0, 0, dz), sub, coef)   # y = y0
        self.quad((x0, y1, z0), (dx, 0, 0), (0, 0, dz), sub, coef)   # y = y1
        if bottom:
            self.quad((x0, y0, z0), (dx, 0, 0), (0, dy, 0), sub, coef)
        if top:
            self.quad((x0, y0, z1), (dx, 0, 0), (0, dy, 0), sub, coef)

    def build(self) -> Scene:
        if not self.tris:
            return empty_scene()
        V = np.asarray(self.verts, np.float64).astype(np.float32)
        T = np.asarray(self.tris, np.int32)
        c = np.asarray(self.coef, np.complex128)
        return Scene(V, T, c.real.astype(np.float32), c.imag.astype(np.float32),
                     np.asarray(self.surf, np.int32))


def empty_scene() -> Scene:
    return Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32),
                 np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.int32))


def box_room(size, coef: complex, sub: int = 1) -> Scene:
    mb = MeshBuilder()
    mb.box((0.0, 0.0, 0.0), size, sub, coef)
    return mb.build()


def concat_scenes(*scenes: Scene) -> Scene:
    Vs, Ts, rr, ri, ss = [], [], [], [], []
    off = 0
    soff = 0
    for s in scenes:
        Vs.append(s.V)
        Ts.append(s.T + off)
        rr.append(s.refl_re)
        ri.append(s.refl_im)
        ss.append(s.surf + soff)
        off += s.V.shape[0]
        soff += s.n_surf
    return Scene(np.concatenate(Vs).astype(np.float32),
                 np.concatenate(Ts).astype(np.int32),
                 np.concatenate(rr).astype(np.float32),
                 np.concatenate(ri).astype(np.float32),
                 np.concatenate(ss).astype(np.int32))


# --------------------------------------------------------------------------
# RIS layouts and receiver sets
# --------------------------------------------------------------------------
def _wall_axes(normal):
    """Two in-plane unit axes (horizontal, vertical) for a vertical wall."""
    n = np.asarray(normal, np.float64)
    up = np.array([0.0, 0.0, 1.0])
    h = np.cross(up, n)
    h /= np.linalg.norm(h)
    v = np.cross(n, h)
    return h, v


def square_ris(nx: int, ny: int, pitch: float, centre, normal) -> np.ndarray:
    h, v = _wall_axes(normal)
    c = np.asarray(centre, np.float64)
    out = []
    for j in range(ny):
        for i in range(nx):
            a = (i - (nx - 1) / 2.0) * pitch
            b = (j - (ny - 1) / 2.0) * pitch
            out.append(c + a * h + b * v)
    return np.asarray(out, np.float64)


def hex_ris(rings: int, pitch: float, centre, normal) -> np.ndarray:
    """Centred hexagonal layout with ``rings`` rings: 1 + 3 r (r + 1)
    elements (127 for 6 rings, the size of the paper's RIS).  Rows run along
    the wall's horizontal axis."""
    h, v = _wall_axes(normal)
    c = np.asarray(centre, np.float64)
    out = []
    row_h = pitch * math.sqrt(3.0) / 2.0
    for r in range(-rings, rings + 1):
        n_in_row = 2 * rings + 1 - abs(r)
        x0 = -(n_in_row - 1) / 2.0 * pitch
        for i in range(n_in_row):
            out.append(c + (x0 + i * pitch) * h + r * row_h * v)
    return np.asarray(out, np.float64)


def hex_count(rings: int) -> int:
    return 1 + 3 * rings * (rings + 1)


def rx_line(p0, p1, n: int, jitter: float, rng) -> np.ndarray:
    p0 = np.asarray(p0, np.float64)
    p1 = np.asarray(p1, np.float64)
    s = np.linspace(0.0, 1.0, n)[:, None]
    pts = p0 + s * (p1 - p0)
    return pts + rng.uniform(-jitter, jitter, size=pts.shape)


def rx_grid(x0, x1, nx, y0, y1, ny, z, jitter: float = 0.0, rng=None) -> np.ndarray:
    """Planar grid, endpoints inclusive, x fastest."""
    xs = np.linspace(x0, x1, nx)
    ys = np.linspace(y0, y1, ny)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)
    if jitter > 0.0:
        pts = pts + rng.uniform(-jitter, jitter, size=pts.shape)
    return pts


def gamma_binary(M: int, C: int, mag: float, rng) -> np.ndarray:
    """mag * e^{j phi}, phi in {0, pi}: mag * (+-1)."""
    s = rng.integers(0, 2, size=(M, C)) * 2 - 1
    return (mag * s).astype(np.complex128)


def gamma_2bit(M: int, C: int, mag: float, rng) -> np.ndarray:
    """mag * j^b, b in {0, 1, 2, 3}."""
    b = rng.integers(0, 4, size=(M, C))
    return mag * (1j ** b)


def unit(v) -> np.ndarray:
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def tiny_box(seed: int = BASE_SEED + 0, n_rays: int = 10_000, order: int = 1,
             n_rx: int = 64, n_cfg: int = 1) -> Problem:
    """5 x 4 x 3 m box (12 triangles, coefficient 0.5), 28 GHz, isotropic Tx
    at (1, 1, 1.5), 7 x 7 RIS at lambda/2 pitch 1 mm in front of the x = 5
    wall, element pattern cos^3, Gamma = 0.9 e^{j phi} with phi in {0, pi},
    64 receivers on a line at z = 1.5."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = C0 / freq
    scene = box_room((5.0, 4.0, 3.0), 0.5 + 0j, sub=1)
    normal = np.array([-1.0, 0.0, 0.0])
    centre = np.array([4.999, 2.0, 1.5])
    elems = square_ris(7, 7, lam / 2, centre, normal)
    ris = Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
    rx = rx_line((0.5, 3.3, 1.5), (4.5, 2.7, 1.5), n_rx, 1e-3, rng)
    tx = np.array([1.0, 1.0, 1.5])
    gamma = gamma_binary(elems.shape[0], n_cfg, 0.9, rng)
    return Problem("tiny_box", scene, freq, tx, 0.01,
                   Antenna(unit(centre - tx), 1.0, PAT_ISO, 0.0), ris, rx,
                   Antenna(np.array([0.0, 0.0, 1.0]), 1.0, PAT_ISO, 0.0),
                   order, n_rays, seed, gamma)


def lab_room_scene(rng, size=(6.0, 5.0, 3.0), n_boxes: int = 20, sub: int = 3,
                   coef_lo: float = 0.3, coef_hi: float = 0.7,
                   max_h: float = 1.0) -> Scene:
    mb = MeshBuilder()
    mb.box((0.0, 0.0, 0.0), size, sub, complex(rng.uniform(coef_lo, coef_hi)))
    for _ in range(n_boxes):
        w = rng.uniform(0.3, 1.2)
        d = rng.uniform(0.3, 1.2)
        h = rng.uniform(0.4, max_h)
        x0 = rng.uniform(0.1, size[0] - 0.1 - w)
        y0 = rng.uniform(0.1, size[1] - 0.1 - d)
        mb.box((x0, y0, 0.0), (x0 + w, y0 + d, h), sub,
               complex(rng.uniform(coef_lo, coef_hi)), bottom=False)
    return mb.build()


def lab_room(seed: int = BASE_SEED + 1, n_rays: int = 1_000_000, order: int = 3,
             nx: int = 64, ny: int = 64, n_cfg: int = 1, sub: int = 3) -> Problem:
    """6 x 5 x 3 m room (walls 3 x 3 subdivided) with 20 seeded furniture
    boxes (~1.9k triangles, coefficients U(0.3, 0.7) per object), 28 GHz,
    127-element hexagonal RIS at lambda/2 pitch on the x = 6 wall with 2-bit
    phases, Tx horn cos^8 (G_t = 18) aimed at the RIS centre, 64 x 64
    isotropic receiver grid at z = 1.2, order <= 3.  ``sub`` subdivides
    every face into sub x sub squares (3 by default; 5 gives ~5.3k
    triangles)."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = C0 / freq
    scene = lab_room_scene(rng, sub=sub)
    normal = np.array([-1.0, 0.0, 0.0])
    centre = np.array([5.999, 2.5, 1.5])
    elems = hex_ris(6, lam / 2, centre, normal)
    ris = Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
    tx = np.array([0.5, 0.5, 2.5])
    rx = rx_grid(0.3, 5.7, nx, 0.3, 4.7, ny, 1.2, 5e-4, rng)
    gamma = gamma_2bit(elems.shape[0], n_cfg, 0.9, rng)
    return Problem("lab_room", scene, freq, tx, 0.01,
                   Antenna(unit(centre - tx), 18.0, PAT_COSPOW, 8.0), ris, rx,
                   Antenna(np.array([0.0, 0.0, 1.0]), 1.0, PAT_ISO, 0.0),
                   order, n_rays, seed, gamma)


def with_materials(prob: Problem, pol: int, seed: int = BASE_SEED + 9, eps_r=(2.0, 8.0), sigma=(0.0, 0.3)) -> Problem:
    """The same problem with Fresnel reflection (pol 1 TE, 2 TM): one seeded
    material per surface, relative permittivity U(eps_r), conductivity
    U(sigma) S/m, copied to its triangles."""
    rng = np.random.default_rng(seed)
    ns = prob.scene.n_surf
    er = rng.uniform(*eps_r, size=ns).astype(np.float32)
    sg = rng.uniform(*sigma, size=ns).astype(np.float32)
    return dataclasses.replace(prob, name=prob.name + ("_te" if pol == 1 else "_tm"), fresnel=pol,
                               mat_eps_r=er[prob.scene.surf], mat_sigma=sg[prob.scene.surf])


def wide_ris_room(seed: int = BASE_SEED + 5, n_rays: int = 20_000, order: int = 2, nx: int = 6,
                  ny: int = 5) -> Problem:
    """The lab room with a sparse 8 x 8 array (0.35 m pitch, 2.45 m across) on
    the x = 6 wall: the legs of one receiver's elements are far apart, the
    opposite of the dense RIS the grouped leg walk is built for."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = C0 / freq
    scene = lab_room_scene(rng)
    normal = np.array([-1.0, 0.0, 0.0])
    centre = np.array([5.999, 2.5, 1.5])
    elems = square_ris(8, 8, 0.35, centre, normal)
    ris = Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
    tx = np.array([0.5, 0.5, 2.5])
    rx = rx_grid(0.3, 5.7, nx, 0.3, 4.7, ny, 1.2, 5e-4, rng)
    gamma = gamma_2bit(elems.shape[0], 1, 0.9, rng)
    return Problem("wide_ris", scene, freq, tx, 0.01,
                   Antenna(unit(centre - tx), 18.0, PAT_COSPOW, 8.0), ris, rx,
                   Antenna(np.array([0.0, 0.0, 1.0]), 1.0, PAT_ISO, 0.0),
                   order, n_rays, seed, gamma)


def precision_problem(seed: int = BASE_SEED + 2, n_side: int = 32, nx: int = 128,
                      ny: int = 128, n_cfg: int = 4096, n_rays: int = 10_000) -> Problem:
    """Channel source for the many-configuration RIS sum: the tiny box room
    with a 32 x 32 RIS (lambda/2) on the x = 5 wall, 128 x 128 receivers at
    z = 1.5, order 1; Gamma = 0.9 s with seeded s in {+-1}."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = C0 / freq
    scene = box_room((5.0, 4.0, 3.0), 0.5 + 0j, sub=1)
    normal = np.array([-1.0, 0.0, 0.0])
    centre = np.array([4.999, 2.0, 1.5])
    elems = square_ris(n_side, n_side, lam / 2, centre, normal)
    ris = Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
    rx = rx_grid(0.25, 4.75, nx, 0.25, 3.75, ny, 1.5, 3e-4, rng)
    tx = np.array([1.0, 1.0, 1.5])
    gamma = gamma_binary(elems.shape[0], n_cfg, 0.9, rng)
    return Problem("precision", scene, freq, tx, 0.01,
                   Antenna(unit(centre - tx), 1.0, PAT_ISO, 0.0), ris, rx,
                   Antenna(np.array([0.0, 0.0, 1.0]), 1.0, PAT_ISO, 0.0),
                   1, n_rays, seed, gamma)


def random_box_room(rng, n_tri_target: int):
    """A random box room for the serving mix: room size U(4..12) m, enough
    3 x 3-subdivided furniture boxes and wall subdivision to reach roughly
    ``n_tri_target`` triangles."""
    L = rng.uniform(4.0, 12.0)
    W = rng.uniform(4.0, 10.0)
    H = 3.0
    sub_wall = 3
    wall_tris = 6 * sub_wall * sub_wall * 2
    per_box_sub = 3 if n_tri_target < 20_000 else 8
    per_box = 5 * per_box_sub * per_box_sub * 2
    n_boxes = max(1, (n_tri_target - wall_tris) // per_box)
    mb = MeshBuilder()
    mb.box((0.0, 0.0, 0.0), (L, W, H), sub_wall, complex(rng.uniform(0.3, 0.7)))
    for _ in range(n_boxes):
        w = rng.uniform(0.1, 0.6)
        d = rng.uniform(0.1, 0.6)
        h = rng.uniform(0.2, 1.0)
        x0 = rng.uniform(0.1, L - 0.7)
        y0 = rng.uniform(0.1, W - 1.0)
        mb.box((x0, y0, 0.0), (x0 + w, y0 + d, h), per_box_sub,
               complex(rng.uniform(0.3, 0.7)), bottom=False)
    return mb.build(), (L, W, H)


def paper_room(reflective: bool = True, grid: str = "coarse", n_rays: int = 100_000,
               seed: int = BASE_SEED + 11) -> Problem:
    """Section III's scenario.  23.8 GHz, P_t = 10 dBm; a horn Tx (G_t = 19 dB,
    cos^(G_t/2 - 1)) at t = (1.86 m, -36 deg, 90 deg) from the RIS centre,
    aimed at it; a 127-element hexagonal RIS (d_y = d_z = 6.6 mm, element
    pitch 6.6 mm, cos theta elements, G = 4 pi d_y d_z / lambda^2) at
    u = (0, 0, 0.5) m facing +x; a lambda/4 monopole Rx (G_r = 0 dB) along +z;
    the 0.9 x 0.05 x 1 m blocking panel at (1.55, -0.475, 0.5) m.  Reflective:
    three metal walls (the sides y = -1.2, 1.2 m and the wall x = 2 m opposite
    the RIS, 1 m high) and the panel, all of the paper's metal (eps_r = 1,
    sigma = 1e7 S/m, TE Fresnel coefficients: the monopole's vertical field
    lies across the plane of incidence on vertical walls), reflections up to
    order 2; anechoic: the panel alone, order 0.  Receivers at z = 11.4 cm:
    grid "coarse" 0.92 <= x <= 1.52, 0.02 <= y <= 0.92 m every 1 cm (61 x 91),
    "fine" 1.1 <= x <= 1.3, 0.25 <= y <= 0.45 m every 2 mm (101 x 101),
    "target" the single point r = (1.33, 0.23, 0.11) m the RIS is configured
    for.  Gamma is left to the caller (on/off with amplitude 1.25)."""
    f = 23.8e9
    lam = C0 / f
    u = np.array([0.0, 0.0, 0.5])
    normal = np.array([1.0, 0.0, 0.0])
    mb = MeshBuilder()
    metal = complex(-1.0, 0.0)   # the fixed coefficient is not used (Fresnel)
    if reflective:
        mb.quad((0.0, -1.2, 0.0), (2.0, 0.0, 0.0), (0.0, 0.0, 1.0), 1, metal)   # y = -1.2
        mb.quad((0.0, 1.2, 0.0), (2.0, 0.0, 0.0), (0.0, 0.0, 1.0), 1, metal)    # y = +1.2
        mb.quad((2.0, -1.2, 0.0), (0.0, 2.4, 0.0), (0.0, 0.0, 1.0), 1, metal)   # x = 2
    pc, ps = np.array([1.55, -0.475, 0.5]), np.array([0.9, 0.05, 1.0])
    mb.box(tuple(pc - ps / 2), tuple(pc + ps / 2), 1, metal)
    scene = mb.build()
    elems = hex_ris(6, 6.6e-3, u, normal)
    ris = Ris(elems, normal, u, 6.6e-3, 6.6e-3, 4.0 * math.pi * 6.6e-3 ** 2 / lam ** 2, 1.0)
    tx = paper_spherical(u, 1.86, -36.0, 90.0)
    gt = 10 ** 1.9
    tx_ant = Antenna(unit(u - tx), gt, PAT_COSPOW, gt / 2.0 - 1.0)
    rx_ant = Antenna(np.array([0.0, 0.0, 1.0]), 1.0, PAT_MONOPOLE, 0.25)
    if grid == "coarse":
        rx = rx_grid(0.92, 1.52, 61, 0.02, 0.92, 91, 0.114)
    elif grid == "fine":
        rx = rx_grid(1.1, 1.3, 101, 0.25, 0.45, 101, 0.114)
    elif grid == "target":
        rx = np.array([[1.33, 0.23, 0.11]])
    else:
        raise ValueError(grid)
    nt = scene.n_tri
    return Problem("paper_" + ("reflective" if reflective else "anechoic") + "_" + grid, scene, f, tx, 0.01,
                   tx_ant, ris, rx, rx_ant, 2 if reflective else 0, n_rays, seed, None,
                   fresnel=1, mat_eps_r=np.full(nt, 1.0, np.float32), mat_sigma=np.full(nt, 1e7, np.float32))


def paper_spherical(u, r: float, phi_deg: float, theta_deg: float) -> np.ndarray:
    """A position given as (r, phi, theta) relative to the RIS centre u in
    the global axes (theta from +z, phi from +x), as used for the Tx and Rx
    of the reflective scenario (Section III, Table I)."""
    ph = math.radians(phi_deg)
    th = math.radians(theta_deg)
    u = np.asarray(u, np.float64)
    return u + r * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph),
                             math.cos(th)])


# --------------------------------------------------------------------------
# large scene: an office floor
# --------------------------------------------------------------------------
def _face_grid(p0, pu, pv, nu: int, nv: int):
    """Vertices and triangles of the rectangle p0 + a pu + b pv, a, b in
    [0, 1], cut into nu x nv quads, each split along its (0,0)-(1,1)
    diagonal (vertices shared inside the face).  Returns float64 vertices
    [(nu+1)(nv+1), 3] and int64 triangles [2 nu nv, 3] (local indices)."""
    a = np.arange(nu + 1) / nu
    b = np.arange(nv + 1) / nv
    V = (np.asarray(p0, np.float64)[None, None, :] + a[:, None, None] * np.asarray(pu, np.float64)
         + b[None, :, None] * np.asarray(pv, np.float64)).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    c00 = (i * (nv + 1) + j).ravel()
    c10 = ((i + 1) * (nv + 1) + j).ravel()
    c11 = ((i + 1) * (nv + 1) + j + 1).ravel()
    c01 = (i * (nv + 1) + j + 1).ravel()
    T = np.stack([np.stack([c00, c10, c11], 1), np.stack([c00, c11, c01], 1)], 1).reshape(-1, 3)
    return V, T


class FastMesh:
    """Mesh accumulated face by face with numpy (one surface per face, one
    reflection coefficient per object): for scenes of 10^5-10^6 triangles."""

    def __init__(self) -> None:
        self.V, self.T, self.surf, self.coef = [], [], [], []
        self.nv = 0
        self.ns = 0

    def face(self, p0, pu, pv, size_u: float, size_v: float, cell: float, coef: complex) -> None:
        nu = max(1, int(round(size_u / cell)))
        nv = max(1, int(round(size_v / cell)))
        V, T = _face_grid(p0, pu, pv, nu, nv)
        self.V.append(V)
        self.T.append(T + self.nv)
        self.surf.append(np.full(T.shape[0], self.ns, np.int32))
        self.coef.append(np.full(T.shape[0], coef, np.complex128))
        self.nv += V.shape[0]
        self.ns += 1

    def box(self, lo, hi, cell: float, coef: complex, bottom: bool = False, top: bool = False) -> None:
        x0, y0, z0 = lo
        x1, y1, z1 = hi
        dx, dy, dz = x1 - x0, y1 - y0, z1 - z0
        self.face((x0, y0, z0), (0, dy, 0), (0, 0, dz), dy, dz, cell, coef)   # x = x0
        self.face((x1, y0, z0), (0, dy, 0), (0, 0, dz), dy, dz, cell, coef)   # x = x1
        self.face((x0, y0, z0), (dx, 0, 0), (0, 0, dz), dx, dz, cell, coef)   # y = y0
        self.face((x0, y1, z0), (dx, 0, 0), (0, 0, dz), dx, dz, cell, coef)   # y = y1
        if bottom:
            self.face((x0, y0, z0), (dx, 0, 0), (0, dy, 0), dx, dy, cell, coef)
        if top:
            self.face((x0, y0, z1), (dx, 0, 0), (0, dy, 0), dx, dy, cell, coef)

    def build(self) -> Scene:
        c = np.concatenate(self.coef)
        return Scene(np.concatenate(self.V).astype(np.float32), np.concatenate(self.T).astype(np.int32),
                     c.real.astype(np.float32), c.imag.astype(np.float32), np.concatenate(self.surf))


def office_floor_scene(rng, nx: int = 20, ny: int = 10, room: float = 2.0, height: float = 3.0,
                       wall: float = 0.1, door: float = 0.8, p_door: float = 0.6, clutter: int = 2,
                       cell_wall: float = 0.18, cell_floor: float = 0.1, cell_clutter: float = 0.08,
                       coef=(0.2, 0.8)) -> Scene:
    """An office floor of nx x ny rooms of room x room metres (40 x 20 x 3 m
    for the defaults), the large indoor configuration: floor and ceiling
    tiles per room; partitions between neighbouring rooms as wall-thick boxes
    from floor to ceiling, a seeded fraction of them with a door gap (two
    boxes); the outer walls as boxes; `clutter` furniture boxes per room
    (desks and cabinets, bottom face omitted).  Faces are meshed with square
    cells of about cell_* metres; each face is one surface; reflection
    coefficient U(coef) per object."""
    fm = FastMesh()
    L, W = nx * room, ny * room

    def cf():
        return complex(rng.uniform(*coef))

    for i in range(nx):
        for j in range(ny):
            x0, y0 = i * room, j * room
            fm.face((x0, y0, 0.0), (room, 0, 0), (0, room, 0), room, room, cell_floor, cf())       # floor tile
            fm.face((x0, y0, height), (room, 0, 0), (0, room, 0), room, room, cell_floor, cf())    # ceiling tile
    h = wall / 2

    def partition(p_lo, p_hi, along_x: bool, with_door: bool):
        c = cf()
        if along_x:   # wall along x at y = p_lo[1]
            (xa, y), (xb, _) = p_lo, p_hi
            segs = [(xa, xb)] if not with_door else [(xa, (xa + xb - door) / 2), ((xa + xb + door) / 2, xb)]
            for a, b in segs:
                fm.box((a, y - h, 0.0), (b, y + h, height), cell_wall, c)
        else:         # wall along y at x = p_lo[0]
            (x, ya), (_, yb) = p_lo, p_hi
            segs = [(ya, yb)] if not with_door else [(ya, (ya + yb - door) / 2), ((ya + yb + door) / 2, yb)]
            for a, b in segs:
                fm.box((x - h, a, 0.0), (x + h, b, height), cell_wall, c)

    # inner partitions (door gaps seeded) and the outer walls (closed)
    for i in range(1, nx):
        for j in range(ny):
            partition((i * room, j * room + h), (i * room, (j + 1) * room - h), False, rng.uniform() < p_door)
    for j in range(1, ny):
        for i in range(nx):
            partition((i * room + h, j * room), ((i + 1) * room - h, j * room), True, rng.uniform() < p_door)
    for j in range(ny):
        partition((0.0, j * room + h), (0.0, (j + 1) * room - h), False, False)
        partition((L, j * room + h), (L, (j + 1) * room - h), False, False)
    for i in range(nx):
        partition((i * room + h, 0.0), ((i + 1) * room - h, 0.0), True, False)
        partition((i * room + h, W), ((i + 1) * room - h, W), True, False)
    # clutter: desks and cabinets, kept 0.3 m off the walls
    for i in range(nx):
        for j in range(ny):
            for _ in range(clutter):
                w, d = rng.uniform(0.4, 1.2), rng.uniform(0.3, 0.8)
                hh = rng.uniform(0.7, 1.8)
                x0 = i * room + rng.uniform(0.3, room - 0.3 - w)
                y0 = j * room + rng.uniform(0.3, room - 0.3 - d)
                fm.box((x0, y0, 0.0), (x0 + w, y0 + d, hh), cell_clutter, cf(), top=True)
    return fm.build()


def office_floor(seed: int = BASE_SEED + 4, n_rays: int = 10_000_000, order: int = 5, n_rx: int = 256,
                 n_side: int = 64, rx_region=None, n_cfg: int = 1, **scene_kw) -> Problem:
    """The large configuration: an office floor (about 10^6 triangles
    with the defaults), 28 GHz, a 64 x 64 square RIS (lambda/2) 1 mm in front
    of the partition wall x = 10 m of room (4, 4) facing -x, a horn Tx
    (cos^8, G_t = 18) in that room aimed at the RIS centre, an n_rx x n_rx
    isotropic receiver grid at 1.2 m over the floor (or over rx_region =
    (x0, x1, y0, y1)), reflections up to `order`, n_rays discovery rays per
    source."""
    rng = np.random.default_rng(seed)
    freq = 28e9
    lam = C0 / freq
    scene = office_floor_scene(rng, **scene_kw)
    normal = np.array([-1.0, 0.0, 0.0])
    centre = np.array([10.0 - 0.05 - 0.001, 9.0, 1.5])
    elems = square_ris(n_side, n_side, lam / 2, centre, normal)
    ris = Ris(elems, normal, centre, lam / 2, lam / 2, math.pi, 3.0)
    tx = np.array([8.35, 8.35, 2.5])
    x0, x1, y0, y1 = rx_region if rx_region is not None else (0.15, 39.85, 0.15, 19.85)
    rx = rx_grid(x0, x1, n_rx, y0, y1, n_rx, 1.2, 3e-4, rng)
    gamma = gamma_binary(elems.shape[0], n_cfg, 0.9, rng)
    return Problem("office_floor", scene, freq, tx, 0.01,
                   Antenna(unit(centre - tx), 18.0, PAT_COSPOW, 8.0), ris, rx,
                   Antenna(np.array([0.0, 0.0, 1.0]), 1.0, PAT_ISO, 0.0),
                   order, n_rays, seed, gamma)


def deep_tree_room(seed: int = BASE_SEED + 6, n_rays: int = 20_000, order: int = 2, chain: int = 48,
                   nx: int = 6, ny: int = 5) -> Problem:
    """The lab room (bounds [0, 6] x [0, 5] x [0, 3] m) with a chain of tiny
    triangles (1 um, each a surface of its own) near its corner (0, 0, 0):
    element i has its centroid at the centre of the Morton cell whose 63-bit
    code is 2^(62 - i), i.e. one axis at (2^(20 - i//3) + 1/2) ext / 2^21 and
    the other two at ext / 2^22.  No other triangle comes within a few cm of
    the corner, so below the first few levels every level of the Morton order
    splits off one chain element and the BVH is about `chain` levels deeper
    than the room's own: the traversal kernels' 64-entry-stack instances."""
    rng = np.random.default_rng(seed)
    base = lab_room(seed=BASE_SEED + 1, n_rays=n_rays, order=order, nx=nx, ny=ny)
    ext = np.array([6.0, 5.0, 3.0])
    V, T = [], []
    for i in range(chain):
        q = np.zeros(3)
        q[i % 3] = 2.0 ** (20 - i // 3)
        c = (q + 0.5) * ext / 2.0 ** 21
        d = 1e-6
        V.extend([c + [d, 0.0, 0.0], c + [-0.5 * d, 0.866 * d, 0.0], c + [-0.5 * d, -0.866 * d, 0.0]])
        T.append([3 * i, 3 * i + 1, 3 * i + 2])
    coef = rng.uniform(0.3, 0.7, size=chain).astype(np.float32)
    tiny = Scene(np.asarray(V, np.float32), np.asarray(T, np.int32), coef, np.zeros(chain, np.float32),
                 np.arange(chain, dtype=np.int32))
    scene = concat_scenes(base.scene, tiny)
    return dataclasses.replace(base, name="deep_tree_room", scene=scene)
