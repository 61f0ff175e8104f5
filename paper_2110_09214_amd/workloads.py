"""Seeded synthetic inputs for the space-charge field path.

This module only builds inputs: triangle meshes of the detector geometries,
particle clouds, loss weights and synthetic gas cross-section tables.  It holds
none of the field, solve or transport arithmetic, so that both the CPU oracle
(tests only) and the HIP library can be fed from it without sharing any of the
method's code.

Geometries follow the paper's description of the set-up (section 2.3: flat
triangular cells, electrodes at applied voltages, dielectric interfaces with
eps_r1 on the side opposite to the normal and eps_r2 on the normal's side).
The paper's own workloads use CAD geometries and measured gas data that are not
available; the generators below are stand-ins with the stated shapes, sizes and
value distributions.

Units are SI throughout (m, V, C, kg, s); cross sections in m^2, energies of the
gas tables in eV.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2018 values (exact or recommended); used here only to express inputs
# (gas density from p/(k_B T), particle masses).
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
K_BOLTZMANN = 1.380649e-23
ATOMIC_MASS = 1.66053906660e-27

KIND_ED = 0  # electrode-to-dielectric cell (Dirichlet row)
KIND_DD = 1  # dielectric-to-dielectric cell (Neumann row)

SPECIES_ELECTRON = 0
SPECIES_CATION = 1
SPECIES_ANION = 2


@dataclasses.dataclass
class Mesh:
    """Flat triangular cells, structure of arrays (all float64 except kind).

    a, b, c : (N, 3) vertices, counter-clockwise about the cell normal n,
              n = (b - a) x (c - a) / |...| points from medium 1 to medium 2.
    kind    : (N,) int8, KIND_ED or KIND_DD.
    eps1    : (N,) relative permittivity on the -n side (dd cells).
    eps2    : (N,) relative permittivity on the +n side (dd cells).
    rhs     : (N,) applied voltage V_i for ed cells, free charge density
              sigma_F,i (C/m^2) for dd cells: the left-hand side of the
              collocation system.
    """

    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    kind: np.ndarray
    eps1: np.ndarray
    eps2: np.ndarray
    rhs: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.a.shape[0])

    def soa(self) -> dict:
        """Contiguous per-coordinate arrays (ax, ay, ..., cz) as float64."""
        out = {}
        for nm, arr in (("a", self.a), ("b", self.b), ("c", self.c)):
            for k, ax in enumerate("xyz"):
                out[nm + ax] = np.ascontiguousarray(arr[:, k], dtype=np.float64)
        return out

    def bbox(self):
        pts = np.concatenate([self.a, self.b, self.c])
        return pts.min(axis=0), pts.max(axis=0)

    @staticmethod
    def concat(parts, name=""):
        return Mesh(
            a=np.concatenate([p.a for p in parts]),
            b=np.concatenate([p.b for p in parts]),
            c=np.concatenate([p.c for p in parts]),
            kind=np.concatenate([p.kind for p in parts]).astype(np.int8),
            eps1=np.concatenate([p.eps1 for p in parts]),
            eps2=np.concatenate([p.eps2 for p in parts]),
            rhs=np.concatenate([p.rhs for p in parts]),
            name=name,
        )


def _make(tris, kind, value, eps1=1.0, eps2=1.0):
    tris = np.asarray(tris, dtype=np.float64).reshape(-1, 3, 3)
    n = tris.shape[0]
    return Mesh(
        a=tris[:, 0].copy(), b=tris[:, 1].copy(), c=tris[:, 2].copy(),
        kind=np.full(n, kind, np.int8),
        eps1=np.full(n, eps1), eps2=np.full(n, eps2),
        rhs=np.full(n, float(value)),
    )


def _rect(p0, u, v, nu, nv):
    """Grid of nu x nv quads on the parallelogram p0 + s u + t v, each split
    along the (i, j) -> (i+1, j+1) diagonal; orientation u x v."""
    p0, u, v = (np.asarray(x, np.float64) for x in (p0, u, v))
    i = np.arange(nu)[:, None]
    j = np.arange(nv)[None, :]

    def P(ii, jj):
        return p0 + (ii / nu)[..., None] * u + (jj / nv)[..., None] * v

    p00 = P(i + 0 * j, j + 0 * i)
    p10 = P(i + 1 + 0 * j, j + 0 * i)
    p11 = P(i + 1 + 0 * j, j + 1 + 0 * i)
    p01 = P(i + 0 * j, j + 1 + 0 * i)
    t1 = np.stack([p00, p10, p11], axis=-2).reshape(-1, 3, 3)
    t2 = np.stack([p00, p11, p01], axis=-2).reshape(-1, 3, 3)
    return np.concatenate([t1, t2])


def _quads_to_tris(P, flip=False):
    """P: (n0+1, n1+1, 3) structured quad grid -> triangles.  Orientation is
    (axis-0 step) x (axis-1 step), reversed if flip."""
    p00 = P[:-1, :-1]
    p10 = P[1:, :-1]
    p11 = P[1:, 1:]
    p01 = P[:-1, 1:]
    if flip:
        t1 = np.stack([p00, p11, p10], axis=-2)
        t2 = np.stack([p00, p01, p11], axis=-2)
    else:
        t1 = np.stack([p00, p10, p11], axis=-2)
        t2 = np.stack([p00, p11, p01], axis=-2)
    return np.concatenate([t1.reshape(-1, 3, 3), t2.reshape(-1, 3, 3)])


def _holed_cell(cx, cy, x0, x1, y0, y1, r, m, n_r, z, up, grading=1.3):
    """Rectangle [x0,x1]x[y0,y1] at height z with a circular hole of radius r
    centred at (cx, cy): an O-grid of 4m angular by n_r radial quads.  Normal
    +z if up else -z."""
    s = np.arange(m) / m
    bx = np.concatenate([x0 + (x1 - x0) * s, np.full(m, x1), x1 - (x1 - x0) * s, np.full(m, x0)])
    by = np.concatenate([np.full(m, y0), y0 + (y1 - y0) * s, np.full(m, y1), y1 - (y1 - y0) * s])
    bx = np.append(bx, bx[0])
    by = np.append(by, by[0])
    th = np.unwrap(np.arctan2(by - cy, bx - cx))
    ix = cx + r * np.cos(th)
    iy = cy + r * np.sin(th)
    g = grading
    sj = (g ** np.arange(n_r + 1) - 1.0) / (g ** n_r - 1.0) if g != 1.0 else np.arange(n_r + 1) / n_r
    X = ix[None, :] + (bx - ix)[None, :] * sj[:, None]
    Y = iy[None, :] + (by - iy)[None, :] * sj[:, None]
    P = np.stack([X, Y, np.full_like(X, z)], axis=-1)  # axis0 radial, axis1 CCW
    return _quads_to_tris(P, flip=not up)


def _wall(cx, cy, rz, n_theta, theta0=0.0):
    """Surface of revolution about the vertical axis through (cx, cy) along the
    profile rz = [(r_0, z_0), ..., (r_k, z_k)] with increasing z; the normal
    points towards the axis for a profile with r constant or r growing with |z|
    away from the waist."""
    rz = np.asarray(rz, np.float64)
    th = theta0 + 2 * np.pi * np.arange(n_theta + 1) / n_theta
    R = rz[:, 0][:, None]
    Z = rz[:, 1][:, None]
    P = np.stack([cx + R * np.cos(th)[None, :], cy + R * np.sin(th)[None, :],
                  np.broadcast_to(Z, (rz.shape[0], n_theta + 1))], axis=-1)
    # axis0: increasing z, axis1: increasing theta -> z x theta = -r (inwards)
    return _quads_to_tris(P)


# --------------------------------------------------------------------------
# Parallel-plate counter
# --------------------------------------------------------------------------
def parallel_plate_mesh(n=32, half=5e-3, gap=1e-3, v_bottom=0.0, v_top=-500.0):
    """Two square plates [-half, half]^2 at z = 0 (v_bottom) and z = gap
    (v_top), each n x n squares split into 2 triangles: 4 n^2 ed cells.
    Zero-thickness sheets carrying the summed charge of both faces."""
    L = 2 * half
    bot = _make(_rect((-half, -half, 0.0), (L, 0, 0), (0, L, 0), n, n), KIND_ED, v_bottom)
    top = _make(_rect((-half, -half, gap), (L, 0, 0), (0, L, 0), n, n), KIND_ED, v_top)
    return Mesh.concat([bot, top], name=f"parallel_plate_{4 * n * n}")


def parallel_plate_electrons(n=4096, seed=0, half=2.5e-3, gap=1e-3):
    """n electrons uniform in [-half, half]^2 x [0, gap] (seed 0)."""
    u = np.random.default_rng(seed).uniform(size=(n, 3))
    x = np.empty_like(u)
    x[:, 0] = -half + 2 * half * u[:, 0]
    x[:, 1] = -half + 2 * half * u[:, 1]
    x[:, 2] = gap * u[:, 2]
    q = np.full(n, -E_CHARGE)
    return x, q


# --------------------------------------------------------------------------
# GEM geometries
# --------------------------------------------------------------------------
@dataclasses.dataclass
class GemGeometry:
    pitch: float = 140e-6
    r_outer: float = 35e-6     # hole radius at the copper faces (70 um diameter)
    r_inner: float = 25e-6     # hole radius at the foil mid-plane (50 um)
    t_kapton: float = 50e-6
    t_cu: float = 5e-6
    half_x: float = 245e-6
    half_y: float = 191.2e-6
    eps_kapton: float = 3.5
    # mesh resolution
    m: int = 12                # O-grid points per cell side (4 m around a hole)
    n_r: int = 6               # radial quads between hole and cell boundary
    n_cone: int = 6            # axial quads per half cone
    n_cu_wall: int = 1         # axial quads on each copper hole wall
    plain_h: float = 12e-6     # target cell size on hole-free face pieces

    def hole_centres(self):
        dy = self.pitch * math.sin(math.pi / 3)
        rows = [(-dy, -35e-6), (0.0, 35e-6), (dy, -35e-6)]
        out = []
        for yr, xo in rows:
            for k in (-1, 0, 1):
                out.append((xo + k * self.pitch, yr))
        return out


def _face(geo: GemGeometry, z):
    """A copper face at height z: 9 holed O-grid cells + hole-free pieces,
    normal +z."""
    dy = geo.pitch * math.sin(math.pi / 3)
    tris = []
    rows = [(-dy, -35e-6), (0.0, 35e-6), (dy, -35e-6)]
    hx = geo.pitch / 2
    for yr, xo in rows:
        y0, y1 = yr - dy / 2, yr + dy / 2
        cells = [xo + k * geo.pitch for k in (-1, 0, 1)]
        for cx in cells:
            tris.append(_holed_cell(cx, yr, cx - hx, cx + hx, y0, y1, geo.r_outer, geo.m, geo.n_r, z, True))
        lo, hi = cells[0] - hx, cells[-1] + hx
        for xa, xb in ((-geo.half_x, lo), (hi, geo.half_x)):
            if xb - xa > 1e-9:
                nu = max(1, int(round((xb - xa) / geo.plain_h)))
                nv = max(1, int(round(dy / geo.plain_h)))
                tris.append(_rect((xa, y0, z), (xb - xa, 0, 0), (0, dy, 0), nu, nv))
    ytop = 1.5 * dy
    for ya, yb in ((-geo.half_y, -ytop), (ytop, geo.half_y)):
        if yb - ya > 1e-9:
            nu = max(1, int(round(2 * geo.half_x / geo.plain_h)))
            nv = max(1, int(round((yb - ya) / geo.plain_h)))
            tris.append(_rect((-geo.half_x, ya, z), (2 * geo.half_x, 0, 0), (0, yb - ya, 0), nu, nv))
    return np.concatenate(tris)


def _face_oriented(geo, z, up):
    t = _face(geo, z)
    if not up:
        t = np.ascontiguousarray(t[:, [0, 2, 1]])
    return t


def _side_strips(geo, z0, z1, nz, h):
    """Four vertical strips on the footprint boundary, outward normals."""
    X, Y = geo.half_x, geo.half_y
    dz = z1 - z0
    nx = max(1, int(round(2 * X / h)))
    ny = max(1, int(round(2 * Y / h)))
    parts = [
        _rect((X, -Y, z0), (0, 2 * Y, 0), (0, 0, dz), ny, nz),     # +x
        _rect((-X, -Y, z0), (0, 0, dz), (0, 2 * Y, 0), nz, ny),    # -x
        _rect((-X, Y, z0), (0, 0, dz), (2 * X, 0, 0), nz, nx),     # +y
        _rect((-X, -Y, z0), (2 * X, 0, 0), (0, 0, dz), nx, nz),    # -y
    ]
    return np.concatenate(parts)


def gem_foil(geo: GemGeometry, z_mid=0.0, v_top=-2400.0, v_bottom=-2000.0):
    """One GEM foil centred at z_mid: two copper layers (closed ed surfaces at
    v_top / v_bottom) and the kapton hole walls and outer sides (dd cells,
    kapton eps on the -n side, gas eps_r = 1 on the +n side)."""
    tk, tc = geo.t_kapton / 2, geo.t_cu
    n_theta = 4 * geo.m
    parts = []
    # copper: top layer z in [tk, tk + tc], bottom layer z in [-tk - tc, -tk]
    for sgn, v in ((+1, v_top), (-1, v_bottom)):
        z_out = z_mid + sgn * (tk + tc)
        z_in = z_mid + sgn * tk
        tris = [_face_oriented(geo, z_out, up=(sgn > 0)),
                _face_oriented(geo, z_in, up=(sgn < 0))]
        zl, zh = sorted((z_in, z_out))
        for (cx, cy) in geo.hole_centres():
            prof = [(geo.r_outer, zl + (zh - zl) * k / geo.n_cu_wall) for k in range(geo.n_cu_wall + 1)]
            tris.append(_wall(cx, cy, prof, n_theta))
        tris.append(_side_strips(geo, zl, zh, 1, geo.plain_h))
        parts.append(_make(np.concatenate(tris), KIND_ED, v))
    # kapton biconical walls: r from r_outer at |z|=tk to r_inner at z=0
    tris = []
    zs = np.concatenate([np.linspace(-tk, 0.0, geo.n_cone + 1), np.linspace(0.0, tk, geo.n_cone + 1)[1:]])
    rs = geo.r_inner + (geo.r_outer - geo.r_inner) * np.abs(zs) / tk
    for (cx, cy) in geo.hole_centres():
        tris.append(_wall(cx, cy, np.stack([rs, z_mid + zs], axis=1), n_theta))
    tris.append(_side_strips(geo, z_mid - tk, z_mid + tk, max(1, int(round(2 * tk / geo.plain_h))), geo.plain_h))
    parts.append(_make(np.concatenate(tris), KIND_DD, 0.0, eps1=geo.eps_kapton, eps2=1.0))
    return Mesh.concat(parts, name="gem_foil")


def _plane(geo, z, v, n=32):
    X, Y = geo.half_x, geo.half_y
    return _make(_rect((-X, -Y, z), (2 * X, 0, 0), (0, 2 * Y, 0), n, n), KIND_ED, v)


def gem_cell_mesh(geo: GemGeometry | None = None, v_drift=-3000.0, v_top=-2400.0,
                  v_bottom=-2000.0, v_ind=0.0, drift_gap=3e-3, ind_gap=2e-3):
    """Single GEM unit cell (3x3 holes on a 140 um hexagonal pitch) with a
    drift plane drift_gap above the top copper face and an induction plane
    ind_gap below the bottom copper face; about 40k cells by default."""
    geo = geo or GemGeometry()
    top = geo.t_kapton / 2 + geo.t_cu
    foil = gem_foil(geo, 0.0, v_top, v_bottom)
    m = Mesh.concat([foil, _plane(geo, top + drift_gap, v_drift), _plane(geo, -top - ind_gap, v_ind)],
                    name="gem_cell")
    return m


def gem_cell_refined_geometry():
    """Refinement of the GEM cell used for the adjoint workload (~50k cells)."""
    return GemGeometry(m=13, n_r=7, n_cone=7)


def double_gem_mesh(geo: GemGeometry | None = None, sep=2e-3, drift_gap=3e-3, ind_gap=2e-3,
                    v=(-3800.0, -3200.0, -2800.0, -2400.0, -2000.0, 0.0)):
    """Two GEM foils with mid-planes sep apart (upper foil at z = 0), drift
    plane drift_gap above the upper foil, induction plane ind_gap below the
    lower one.  Voltages: drift, GEM1 top/bottom, GEM2 top/bottom, induction."""
    geo = geo or GemGeometry(m=10, n_r=5, n_cone=6)
    top = geo.t_kapton / 2 + geo.t_cu
    f1 = gem_foil(geo, 0.0, v[1], v[2])
    f2 = gem_foil(geo, -sep, v[3], v[4])
    return Mesh.concat([f1, f2, _plane(geo, top + drift_gap, v[0]), _plane(geo, -sep - top - ind_gap, v[5])],
                       name="double_gem")


def gem_cell_points(n=1_000_000, seed=1, geo: GemGeometry | None = None, drift_gap=3e-3, ind_gap=2e-3):
    """n field points uniform in footprint x [-(top+ind_gap), top+drift_gap] (seed 1)."""
    geo = geo or GemGeometry()
    top = geo.t_kapton / 2 + geo.t_cu
    u = np.random.default_rng(seed).uniform(size=(n, 3))
    x = np.empty_like(u)
    x[:, 0] = geo.half_x * (2 * u[:, 0] - 1)
    x[:, 1] = geo.half_y * (2 * u[:, 1] - 1)
    x[:, 2] = -(top + ind_gap) + (2 * top + ind_gap + drift_gap) * u[:, 2]
    return x


def gaussian_clouds(n_e, n_i, centre_e, centre_i, sigma, rng):
    """Electrons then singly charged cations, each an isotropic 3D Gaussian;
    returns positions (n_e + n_i, 3), charges, species."""
    xe = rng.normal(size=(n_e, 3)) * sigma + np.asarray(centre_e)
    xi = rng.normal(size=(n_i, 3)) * sigma + np.asarray(centre_i)
    x = np.concatenate([xe, xi])
    q = np.concatenate([np.full(n_e, -E_CHARGE), np.full(n_i, E_CHARGE)])
    sp = np.concatenate([np.full(n_e, SPECIES_ELECTRON, np.int8), np.full(n_i, SPECIES_CATION, np.int8)])
    return x, q, sp


def space_charge_cloud(n_e=2_000_000, n_i=2_000_000, seed=2):
    """2M electrons ~ N((0,0,230um), (50um)^2 I) then 2M cations ~
    N((0,0,210um), (50um)^2 I), drawn in that order (seed 2)."""
    rng = np.random.default_rng(seed)
    return gaussian_clouds(n_e, n_i, (0, 0, 230e-6), (0, 0, 210e-6), 50e-6, rng)


def adjoint_workload(n_e=500_000, n_i=500_000, seed=3):
    """Clouds as in space_charge_cloud (positions first), then loss weights
    w ~ N(0,1)^(n x 3), all from seed 3."""
    rng = np.random.default_rng(seed)
    x, q, sp = gaussian_clouds(n_e, n_i, (0, 0, 230e-6), (0, 0, 210e-6), 50e-6, rng)
    w = rng.normal(size=(n_e + n_i, 3))
    return x, q, sp, w


def double_gem_initial(n_pairs=200_000, seed=4, geo: GemGeometry | None = None, height=60e-6):
    """Initial population for the double-GEM run: n_pairs electrons and
    n_pairs cations drawn independently from N(c, (20um)^2 I), c on the axis of
    the central hole of the upper foil, `height` above its top copper face.
    Velocities zero.  Returns positions, species, ids (electrons first)."""
    geo = geo or GemGeometry(m=10, n_r=5, n_cone=6)
    top = geo.t_kapton / 2 + geo.t_cu
    cx, cy = geo.hole_centres()[4]
    rng = np.random.default_rng(seed)
    c = np.array([cx, cy, top + height])
    x = np.concatenate([rng.normal(size=(n_pairs, 3)) * 20e-6 + c, rng.normal(size=(n_pairs, 3)) * 20e-6 + c])
    sp = np.concatenate([np.full(n_pairs, SPECIES_ELECTRON, np.int8), np.full(n_pairs, SPECIES_CATION, np.int8)])
    return x, sp


def double_gem_avalanche_start(n_e=200_000, seed=4, geo: GemGeometry | None = None, margin=0.9):
    """Initial population of the double-GEM tracking run: n_e electrons at
    rest inside the 9 holes of the upper foil (the electrons an avalanche
    starts from), no ions.  Per electron: a hole (uniform), a height z
    uniform over the foil (copper and kapton), a point uniform over the disk
    of `margin` times the hole radius at that height (biconical in the
    kapton, r_outer in the copper).  Returns positions, species."""
    geo = geo or GemGeometry(m=10, n_r=5, n_cone=6)
    tk, tc = geo.t_kapton / 2, geo.t_cu
    rng = np.random.default_rng(seed)
    cen = np.array(geo.hole_centres())
    h = rng.integers(0, len(cen), n_e)
    z = rng.uniform(-(tk + tc), tk + tc, n_e)
    r_hole = np.where(np.abs(z) < tk, geo.r_inner + (geo.r_outer - geo.r_inner) * np.abs(z) / tk, geo.r_outer)
    r = margin * r_hole * np.sqrt(rng.uniform(size=n_e))
    t = rng.uniform(0.0, 2 * math.pi, n_e)
    x = np.stack([cen[h, 0] + r * np.cos(t), cen[h, 1] + r * np.sin(t), z], axis=1)
    return x, np.full(n_e, SPECIES_ELECTRON, np.int8)


# --------------------------------------------------------------------------
# Test fixtures
# --------------------------------------------------------------------------
def icosphere(radius, subdiv, centre=(0.0, 0.0, 0.0)):
    """Triangulated sphere, outward normals."""
    t = (1.0 + 5 ** 0.5) / 2
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
                  [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], float)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
                  [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
                  [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    verts = list(v)
    for _ in range(subdiv):
        cache = {}
        nf = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                p = verts[i] + verts[j]
                verts.append(p / np.linalg.norm(p))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf)
    V = np.array(verts) * radius + np.asarray(centre)
    tris = V[f]
    # orient outwards
    n = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    cen = tris.mean(axis=1) - np.asarray(centre)
    flip = np.einsum("ij,ij->i", n, cen) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def sphere_in_shell_mesh(a=1.0, b=2.0, eps_shell=4.0, v=1.0, subdiv=3):
    """Conducting sphere (radius a, potential v) inside a concentric dielectric
    shell (eps_shell, outer radius b) in vacuum: ed sphere + two dd spheres?
    No: the inner sphere surface is an electrode in contact with the shell,
    so only the outer shell surface is a dd interface (eps_shell inside on the
    -n side, vacuum outside)."""
    s = _make(icosphere(a, subdiv), KIND_ED, v)
    d = _make(icosphere(b, subdiv), KIND_DD, 0.0, eps1=eps_shell, eps2=1.0)
    return Mesh.concat([s, d], name="sphere_in_shell")


def plates_with_slab_mesh(n=24, half=5e-3, gap=1e-3, t=0.4e-3, eps=3.0, v_top=-500.0, nz=2):
    """Parallel plates (z = 0 at 0 V, z = gap at v_top) with a dielectric slab
    eps filling [-half, half]^2 x [0, t]: the slab's top face and its four
    sides are dd cells (slab on the -n side)."""
    L = 2 * half
    bot = _make(_rect((-half, -half, 0.0), (L, 0, 0), (0, L, 0), n, n), KIND_ED, 0.0)
    top = _make(_rect((-half, -half, gap), (L, 0, 0), (0, L, 0), n, n), KIND_ED, v_top)
    geo = GemGeometry(half_x=half, half_y=half)
    faces = [_rect((-half, -half, t), (L, 0, 0), (0, L, 0), n, n),
             _side_strips(geo, 0.0, t, nz, L / n)]
    slab = _make(np.concatenate(faces), KIND_DD, 0.0, eps1=eps, eps2=1.0)
    return Mesh.concat([bot, top, slab], name="plates_with_slab")


def dielectric_box_mesh(half=5e-3, depth=5e-3, eps=4.0, n=24, nz=12):
    """Closed dielectric box [-half, half]^2 x [-depth, 0] in vacuum: all dd
    cells, outward normals (dielectric on the -n side)."""
    L = 2 * half
    top = _rect((-half, -half, 0.0), (L, 0, 0), (0, L, 0), n, n)
    bot = _rect((-half, -half, -depth), (0, L, 0), (L, 0, 0), n, n)
    geo = GemGeometry(half_x=half, half_y=half)
    sides = _side_strips(geo, -depth, 0.0, nz, L / n)
    return _make(np.concatenate([top, bot, sides]), KIND_DD, 0.0, eps1=eps, eps2=1.0)


# --------------------------------------------------------------------------
# Synthetic gas
# --------------------------------------------------------------------------
@dataclasses.dataclass
class GasTables:
    """Electron cross sections on log-spaced nodes (interpolated linearly in
    the normalised lethargy of eq. (leth) by the consumers), process order
    elastic, exc1, exc2, ionisation, attachment; ion cross sections constant."""
    energies: np.ndarray          # (n,) eV, log-spaced
    xs: np.ndarray                # (5, n) m^2
    thresholds: np.ndarray        # (5,) eV
    e_min: float
    e_max: float
    density: float                # m^-3
    temperature: float            # K
    m_gas: float                  # kg (mass-weighted molecule of the mixture)
    m_cation: float
    m_anion: float
    ion_xs_iso: float             # m^2
    ion_xs_back: float            # m^2
    xi: np.ndarray | None = None  # (n,) anisotropy parameter of the elastic angle, None = isotropic
    penning_prob: float = 0.0     # Penning transfer probability (0 = off)
    penning_level: float = 0.0    # eV, ionisation potential of the quenching species


def synthetic_ar_co2(n_nodes=2000, e_min=0.01, e_max=1000.0, pressure=1e5, temperature=300.0, anisotropic=False,
                     penning_prob=0.0, penning_level=12.5):
    """Smooth Ar/CO2-like (70/30) electron cross sections: elastic with a
    resonance-like bump, two excitations (11.55, 13.0 eV), a Lotz-like
    ionisation (15.7 eV) and a Gaussian attachment band at 8.2 eV.  With
    anisotropic=True the elastic angle's anisotropy parameter rises smoothly
    with energy, xi(E) = 0.9 E / (E + 5 eV); penning_prob > 0 turns on Penning
    transfer from excited states at or above penning_level (eV)."""
    E = e_min * (e_max / e_min) ** (np.arange(n_nodes) / (n_nodes - 1))
    x = E / 12.0
    el = 1e-20 * (0.3 + 35.0 * x ** 2 / (1.0 + x ** 2) ** 1.35)

    def exc(T, smax):
        u = np.where(E > T, T / E, 1.0)
        return np.where(E > T, smax * (1 - u) ** 1.5 * u ** 0.5 / 0.3248, 0.0)

    T_ion = 15.7
    ion = np.where(E > T_ion, 1.876e-17 * np.log(np.maximum(E / T_ion, 1.0)) / (E * T_ion), 0.0)
    att = 2e-22 * np.exp(-0.5 * ((E - 8.2) / 1.2) ** 2)
    xs = np.stack([el, exc(11.55, 1.0e-20), exc(13.0, 0.5e-20), ion, att])
    m_gas = (0.7 * 39.948 + 0.3 * 44.0095) * ATOMIC_MASS
    return GasTables(
        energies=E, xs=np.ascontiguousarray(xs), thresholds=np.array([0.0, 11.55, 13.0, T_ion, 0.0]),
        e_min=e_min, e_max=e_max, density=pressure / (K_BOLTZMANN * temperature),
        temperature=temperature, m_gas=m_gas, m_cation=m_gas, m_anion=15.999 * ATOMIC_MASS,
        ion_xs_iso=2.5e-19, ion_xs_back=2.5e-19,
        xi=(0.9 * E / (E + 5.0)) if anisotropic else None, penning_prob=penning_prob, penning_level=penning_level,
    )


def constant_nu_gas(nu, n_nodes=2000, e_min=0.01, e_max=1000.0, density=2.4143e25):
    """Test gas: elastic only with sigma ∝ 1/v (constant collision frequency
    nu), infinitely heavy molecules (no recoil loss), no inelastic channels."""
    E = e_min * (e_max / e_min) ** (np.arange(n_nodes) / (n_nodes - 1))
    v = np.sqrt(2 * E * E_CHARGE / M_ELECTRON)
    xs = np.zeros((5, n_nodes))
    xs[0] = nu / (density * v)
    return GasTables(
        energies=E, xs=xs, thresholds=np.array([0.0, 11.55, 13.0, 15.7, 0.0]), e_min=e_min, e_max=e_max,
        density=density, temperature=300.0, m_gas=1e30, m_cation=40 * ATOMIC_MASS,
        m_anion=16 * ATOMIC_MASS, ion_xs_iso=0.0, ion_xs_back=0.0,
    )
