"""Seeded synthetic workloads: scenes, surface samples, queries, signs, trajectories.

This module draws geometry and points only.  It holds none of the regression
method's arithmetic (no kernel, no fit, no distance mapping), so both the GPU
path and the FP64 CPU oracle may consume its outputs.

The scenes stand in for the paper's indoor (Replica / Cow&Lady) and outdoor
(Newer College) workloads (Sec. V, Table III), which are not available here.
Hyperparameters follow the workload definitions (length-scale 0.2 m, noise
variance 1e-4) instead of the paper's per-dataset lambda (App. I).

Every draw comes from ``numpy.random.default_rng`` on a sub-stream spawned from
``SeedSequence(config_id)``: geometry, sampling jitter, normal noise, queries,
trajectories and per-cell sample caps each have their own stream.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional

import numpy as np

ELL = 0.2          # RBF length-scale (m)
NOISE_VAR = 1e-4   # uniform surface-sample noise variance sigma^2
K_FUSE = 8         # number of nearest local GPs fused by the min

# sub-stream indices
_S_GEOM, _S_JITTER, _S_NOISE, _S_QUERY, _S_TRAJ, _S_CAP, _S_DENS = range(7)


def _rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(cfg_id).spawn(8)[stream])


@dataclasses.dataclass
class Workload:
    """One synthetic workload.

    points      [N,3] surface samples (float64 for the FP64 sphere, else float32)
    origin, h   cell lattice: key = floor((x - origin) / h)
    margin      collection-box growth on each side of a cell (h/2)
    m_max       cap on samples per cell; m_min drops smaller cells
    m_cap_grid  optional uint8 per-lattice-key cap (uneven m), with key_lo
    queries     [Q,3] query points (same dtype as points)
    sign        [Q] int8 sign of the analytic scene (+1 free space)
    """
    cfg_id: int
    name: str
    points: np.ndarray
    origin: tuple
    h: float
    margin: float
    m_max: int
    m_min: int
    queries: np.ndarray
    sign: np.ndarray
    m_cap_grid: Optional[np.ndarray] = None
    key_lo: tuple = (0, 0, 0)
    traj_shape: Optional[tuple] = None    # (n_traj, n_waypoints) when queries are trajectories
    ell: float = ELL
    noise_var: float = NOISE_VAR
    k_fuse: int = K_FUSE
    scene: object = None

    @property
    def dtype(self):
        return self.points.dtype

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.points, self.queries, self.sign):
            h.update(np.ascontiguousarray(a).tobytes())
        if self.m_cap_grid is not None:
            h.update(self.m_cap_grid.tobytes())
        return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# primitive geometry (solids), used for sampling, dropping and the sign
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Box:
    lo: np.ndarray
    hi: np.ndarray

    def inside(self, p, tol=1e-9):
        return np.all((p >= self.lo - tol) & (p <= self.hi + tol), axis=-1)

    def bounds(self):
        return np.asarray(self.lo, np.float64), np.asarray(self.hi, np.float64)


@dataclasses.dataclass
class Cylinder:        # vertical
    cx: float
    cy: float
    r: float
    z0: float
    z1: float

    def inside(self, p, tol=1e-9):
        d2 = (p[..., 0] - self.cx) ** 2 + (p[..., 1] - self.cy) ** 2
        return (d2 <= (self.r + tol) ** 2) & (p[..., 2] >= self.z0 - tol) & (p[..., 2] <= self.z1 + tol)

    def bounds(self):
        return (np.array([self.cx - self.r, self.cy - self.r, self.z0]),
                np.array([self.cx + self.r, self.cy + self.r, self.z1]))


@dataclasses.dataclass
class RoomWalls:       # the solid outside an axis-aligned room box
    lo: np.ndarray
    hi: np.ndarray

    def inside(self, p, tol=1e-9):
        return ~np.all((p > self.lo + tol) & (p < self.hi - tol), axis=-1)


@dataclasses.dataclass
class Terrain:         # solid below a value-noise heightfield
    field: "ValueNoise"

    def inside(self, p, tol=1e-9):
        return p[..., 2] <= self.field.height(p[..., 0], p[..., 1]) + tol


class ValueNoise:
    """Four-octave value noise on a 100 m square, smoothstep-interpolated."""

    def __init__(self, rng, extent=100.0, spacings=(25.0, 12.5, 6.25, 3.125),
                 amps=(1.0, 0.5, 0.25, 0.125), zmax=20.0):
        self.extent, self.spacings, self.amps, self.zmax = extent, spacings, amps, zmax
        self.tables = [rng.random((int(round(extent / s)) + 2,) * 2) for s in spacings]
        self.norm = zmax / sum(amps)

    def height(self, x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for s, a, t in zip(self.spacings, self.amps, self.tables):
            u, v = np.clip(x / s, 0, t.shape[0] - 1.0001), np.clip(y / s, 0, t.shape[1] - 1.0001)
            i, j = np.floor(u).astype(np.int64), np.floor(v).astype(np.int64)
            fu, fv = u - i, v - j
            su, sv = fu * fu * (3 - 2 * fu), fv * fv * (3 - 2 * fv)
            v00, v10, v01, v11 = t[i, j], t[i + 1, j], t[i, j + 1], t[i + 1, j + 1]
            out += a * ((v00 * (1 - su) + v10 * su) * (1 - sv) + (v01 * (1 - su) + v11 * su) * sv)
        return out * self.norm


# ---------------------------------------------------------------------------
# stratified surface sampling (noiseless point, unit normal)
# ---------------------------------------------------------------------------

def _rect(rng, origin, e1, e2, spacing):
    """Stratified jitter on the rectangle origin + s*e1 + t*e2, s,t in [0,1]."""
    l1, l2 = np.linalg.norm(e1), np.linalg.norm(e2)
    n1, n2 = max(1, int(np.ceil(l1 / spacing))), max(1, int(np.ceil(l2 / spacing)))
    i, j = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    s = (i.ravel() + rng.random(i.size)) / n1
    t = (j.ravel() + rng.random(j.size)) / n2
    p = origin[None, :] + s[:, None] * e1[None, :] + t[:, None] * e2[None, :]
    n = np.cross(e1, e2)
    n = n / np.linalg.norm(n)
    return p, np.broadcast_to(n, p.shape).copy()


def _box_surface(rng, box: Box, spacing, bottom=False):
    lo, hi = box.lo, box.hi
    d = hi - lo
    ex, ey, ez = np.array([d[0], 0, 0]), np.array([0, d[1], 0]), np.array([0, 0, d[2]])
    faces = [
        (lo + ez, ex, ey),                 # top (normal +z)
        (lo, ey, ex),                      # bottom (normal -z)
        (lo, ez, ey),                      # x- face (normal -x)
        (lo + ex, ey, ez),                 # x+ face (normal +x)
        (lo, ex, ez),                      # y- face (normal -y)
        (lo + ey, ez, ex),                 # y+ face (normal +y)
    ]
    if not bottom:
        faces.pop(1)
    ps, ns = zip(*[_rect(rng, o, a, b, spacing) for o, a, b in faces])
    return np.concatenate(ps), np.concatenate(ns)


def _room_surface(rng, lo, hi, spacing_per_face):
    """The six interior faces of the room, normals pointing into the room."""
    d = hi - lo
    ex, ey, ez = np.array([d[0], 0, 0]), np.array([0, d[1], 0]), np.array([0, 0, d[2]])
    faces = [(lo, ex, ey), (lo + ez, ey, ex), (lo, ey, ez), (lo + ex, ez, ey),
             (lo, ez, ex), (lo + ey, ex, ez)]
    ps, ns = [], []
    for (o, a, b), sp in zip(faces, spacing_per_face):
        p, n = _rect(rng, o, a, b, sp)
        ps.append(p)
        ns.append(n)
    return ps, ns


def _cyl_surface(rng, c: Cylinder, spacing, bottom=False):
    h = c.z1 - c.z0
    nt = max(3, int(np.ceil(2 * np.pi * c.r / spacing)))
    nh = max(1, int(np.ceil(h / spacing)))
    i, j = np.meshgrid(np.arange(nt), np.arange(nh), indexing="ij")
    th = 2 * np.pi * (i.ravel() + rng.random(i.size)) / nt
    z = c.z0 + h * (j.ravel() + rng.random(j.size)) / nh
    side_n = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], 1)
    side_p = np.stack([c.cx + c.r * np.cos(th), c.cy + c.r * np.sin(th), z], 1)
    caps = [(c.z1, 1.0)] + ([(c.z0, -1.0)] if bottom else [])
    ps, ns = [side_p], [side_n]
    for zc, sgn in caps:
        n1 = max(1, int(np.ceil(2 * c.r / spacing)))
        a, b = np.meshgrid(np.arange(n1), np.arange(n1), indexing="ij")
        u = -c.r + 2 * c.r * (a.ravel() + rng.random(a.size)) / n1
        v = -c.r + 2 * c.r * (b.ravel() + rng.random(b.size)) / n1
        keep = u * u + v * v <= c.r * c.r
        p = np.stack([c.cx + u[keep], c.cy + v[keep], np.full(keep.sum(), zc)], 1)
        ps.append(p)
        ns.append(np.broadcast_to(np.array([0, 0, sgn]), p.shape).copy())
    return np.concatenate(ps), np.concatenate(ns)


def _inside_any(p, solids, tol=1e-9):
    """Mask of the points of p inside any of the solids (each solid's own test, with
    its tolerance); solids with an axis-aligned bound only test the points whose x
    falls in that bound (points sorted by x once)."""
    out = np.zeros(len(p), bool)
    bounded = [s for s in solids if hasattr(s, "bounds")]
    for s in solids:
        if not hasattr(s, "bounds"):
            out |= s.inside(p, tol=tol)
    if bounded and len(p):
        order = np.argsort(p[:, 0], kind="stable")
        xs = p[order, 0]
        pad = tol + 1e-6
        for s in bounded:
            lo, hi = s.bounds()
            a = np.searchsorted(xs, lo[0] - pad, "left")
            b = np.searchsorted(xs, hi[0] + pad, "right")
            idx = order[a:b]
            if len(idx):
                out[idx[s.inside(p[idx], tol=tol)]] = True
    return out


def _drop_inside(parts, solids):
    """Union surface: drop each part's samples that lie in another part's solid."""
    keep_p, keep_n = [], []
    for k, (p, n) in enumerate(parts):
        mask = ~_inside_any(p, [s for j, s in enumerate(solids) if j != k])
        keep_p.append(p[mask])
        keep_n.append(n[mask])
    return keep_p, keep_n


def _add_normal_noise(rng, p, n, std):
    return p + n * rng.normal(0.0, std, size=(len(p), 1))


# ---------------------------------------------------------------------------
# scenes
# ---------------------------------------------------------------------------

ROOM_LO = np.array([0.0, 0.0, 0.0])
ROOM_HI = np.array([10.0, 8.0, 3.0])


class RoomScene:
    """Box room [0,10]x[0,8]x[0,3] with floor-standing boxes and cylinders."""

    def __init__(self, rng, n_boxes=20, n_cyl=10):
        self.walls = RoomWalls(ROOM_LO, ROOM_HI)
        self.boxes, self.cyls = [], []
        for _ in range(n_boxes):
            s = rng.uniform(0.3, 1.5, 3)
            x0 = rng.uniform(0, ROOM_HI[0] - s[0])
            y0 = rng.uniform(0, ROOM_HI[1] - s[1])
            self.boxes.append(Box(np.array([x0, y0, 0.0]), np.array([x0 + s[0], y0 + s[1], s[2]])))
        for _ in range(n_cyl):
            r = rng.uniform(0.1, 0.5)
            h = rng.uniform(0.5, 3.0)
            cx = rng.uniform(r, ROOM_HI[0] - r)
            cy = rng.uniform(r, ROOM_HI[1] - r)
            self.cyls.append(Cylinder(cx, cy, r, 0.0, h))

    def solids(self):
        return [self.walls] + self.boxes + self.cyls

    def free(self, p):
        """True where p lies in free space (inside the room, outside every object)."""
        return ~_inside_any(p, [self.walls] + self.boxes + self.cyls, tol=0.0)

    def sample(self, rng_j, rng_n, spacing, noise_std, density=None):
        """density: optional per-object multiplier (room faces first, then boxes, cylinders)."""
        n_obj = 6 + len(self.boxes) + len(self.cyls)
        dens = np.ones(n_obj) if density is None else density
        sp = spacing / np.sqrt(dens)
        room_ps, room_ns = _room_surface(rng_j, ROOM_LO, ROOM_HI, sp[:6])
        parts = [(np.concatenate(room_ps), np.concatenate(room_ns))]
        for k, b in enumerate(self.boxes):
            parts.append(_box_surface(rng_j, b, sp[6 + k]))
        for k, c in enumerate(self.cyls):
            parts.append(_cyl_surface(rng_j, c, sp[6 + len(self.boxes) + k]))
        ps, ns = _drop_inside(parts, self.solids())
        p, n = np.concatenate(ps), np.concatenate(ns)
        return _add_normal_noise(rng_n, p, n, noise_std)


class TerrainScene:
    """100x100 m value-noise terrain (heights in [0,20] m) with boxes and cylinders."""

    def __init__(self, rng, n_boxes=250, n_cyl=250, size_scale=1.0):
        self.field = ValueNoise(rng)
        self.terrain = Terrain(self.field)
        self.boxes, self.cyls = [], []
        for _ in range(n_boxes):
            sx, sy = rng.uniform(1.0, 4.0, 2) * size_scale
            hz = rng.uniform(1.0, 5.0) * size_scale
            x0, y0 = rng.uniform(0, 100 - sx), rng.uniform(0, 100 - sy)
            xs, ys = np.array([x0, x0 + sx, x0, x0 + sx, x0 + sx / 2]), np.array([y0, y0, y0 + sy, y0 + sy, y0 + sy / 2])
            z0 = float(self.field.height(xs, ys).min())
            self.boxes.append(Box(np.array([x0, y0, z0]), np.array([x0 + sx, y0 + sy, z0 + hz])))
        for _ in range(n_cyl):
            r = rng.uniform(0.1, 0.5) * size_scale
            hz = rng.uniform(1.0, 6.0) * size_scale
            cx, cy = rng.uniform(r, 100 - r), rng.uniform(r, 100 - r)
            ang = np.linspace(0, 2 * np.pi, 9)
            z0 = float(self.field.height(cx + r * np.cos(ang), cy + r * np.sin(ang)).min())
            self.cyls.append(Cylinder(cx, cy, r, z0, z0 + hz))

    def solids(self):
        return [self.terrain] + self.boxes + self.cyls

    def free(self, p):
        return ~_inside_any(p, [self.terrain] + self.boxes + self.cyls, tol=0.0)

    def sample(self, rng_j, rng_n, spacing, noise_std):
        n1 = int(np.ceil(100.0 / spacing))
        parts = []
        # terrain: stratified over xy, normal from a central difference of the heightfield
        rows = []
        for i0 in range(0, n1, 256):       # chunked to bound memory
            i = np.arange(i0, min(n1, i0 + 256))
            ii, jj = np.meshgrid(i, np.arange(n1), indexing="ij")
            x = 100.0 * (ii.ravel() + rng_j.random(ii.size)) / n1
            y = 100.0 * (jj.ravel() + rng_j.random(jj.size)) / n1
            z = self.field.height(x, y)
            e = 1e-3
            gx = (self.field.height(x + e, y) - self.field.height(x - e, y)) / (2 * e)
            gy = (self.field.height(x, y + e) - self.field.height(x, y - e)) / (2 * e)
            nrm = np.stack([-gx, -gy, np.ones_like(gx)], 1)
            nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
            rows.append((np.stack([x, y, z], 1), nrm))
        parts.append((np.concatenate([r[0] for r in rows]), np.concatenate([r[1] for r in rows])))
        for b in self.boxes:
            parts.append(_box_surface(rng_j, b, spacing))
        for c in self.cyls:
            parts.append(_cyl_surface(rng_j, c, spacing))
        ps, ns = _drop_inside(parts, self.solids())
        p, n = np.concatenate(ps), np.concatenate(ns)
        return _add_normal_noise(rng_n, p, n, noise_std)


class SphereScene:
    def __init__(self, radius=1.0):
        self.radius = radius

    def free(self, p):
        return np.linalg.norm(p, axis=-1) > self.radius

    def distance(self, p):
        """Analytic unsigned distance to the sphere surface."""
        return np.abs(np.linalg.norm(p, axis=-1) - self.radius)


# ---------------------------------------------------------------------------
# per-cell caps, queries, trajectories
# ---------------------------------------------------------------------------

def _cap_grid(rng, key_lo, key_hi, lo=8, hi=128):
    """Log-uniform per-lattice-key sample cap on [lo, hi]."""
    dims = tuple(int(b - a + 1) for a, b in zip(key_lo, key_hi))
    u = rng.random(dims)
    m = np.floor(lo * np.exp(u * np.log((hi + 1) / lo))).astype(np.int64)
    return np.clip(m, lo, hi).astype(np.uint8)


def _keys_bounds(points, origin, h, pad=1):
    k = np.floor((points.astype(np.float64) - np.asarray(origin)) / h).astype(np.int64)
    return tuple(k.min(0) - pad), tuple(k.max(0) + pad)


def _sign(free_mask):
    return np.where(free_mask, 1, -1).astype(np.int8)


def _grid_queries(lo, hi, n, dtype):
    axes = [lo[d] + (np.arange(n) + 0.5) * (hi[d] - lo[d]) / n for d in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    return g.astype(dtype)


def _trajectories(rng, scene, n_traj, n_way, lo, hi, dtype):
    ends = []
    need = 2 * n_traj
    while sum(len(e) for e in ends) < need:
        p = rng.uniform(lo, hi, size=(need, 3))
        ends.append(p[scene.free(p)])
    e = np.concatenate(ends)[:need].reshape(n_traj, 2, 3)
    t = (np.arange(n_way) / (n_way - 1))[None, :, None]
    w = e[:, :1, :] * (1 - t) + e[:, 1:, :] * t
    return w.reshape(-1, 3).astype(dtype)


def sphere_workload(n_samples=2000, n_queries=10000, cfg_id=1):
    """Plain method, FP64: unit sphere, 2,000 samples with N(0, 0.01 m) radial noise."""
    g = _rng(cfg_id, _S_GEOM).normal(size=(n_samples, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = 1.0 + _rng(cfg_id, _S_NOISE).normal(0.0, 0.01, size=(n_samples, 1))
    pts = (g * r).astype(np.float64)
    q = _rng(cfg_id, _S_QUERY).uniform(-2.0, 2.0, size=(n_queries, 3)).astype(np.float64)
    scene = SphereScene()
    return Workload(cfg_id, "sphere_fp64", pts, (0.0, 0.0, 0.0), 0.5, 0.25, 32, 1, q,
                    _sign(scene.free(q)), scene=scene)


def room_workload(variant="grid", grid_n=256, n_random=4_194_304, n_traj=4096, n_way=64,
                  spacing=0.02, cfg_id=None):
    """Indoor room.  variant: 'grid' (256^3 mean/grad/var grid), 'batch' (uneven
    density and uneven m, random queries), 'traj' (trajectories for the cost)."""
    cfg_id = cfg_id if cfg_id is not None else {"grid": 2, "batch": 3, "traj": 4}[variant]
    scene_rng = _rng(2, _S_GEOM)               # one room shared by the three indoor workloads
    scene = RoomScene(scene_rng)
    density = None
    if variant == "batch":
        n_obj = 6 + len(scene.boxes) + len(scene.cyls)
        density = np.exp(_rng(cfg_id, _S_DENS).uniform(np.log(0.1), np.log(4.0), n_obj))
    pts = scene.sample(_rng(cfg_id if variant == "batch" else 2, _S_JITTER),
                       _rng(cfg_id if variant == "batch" else 2, _S_NOISE), spacing, 0.005, density)
    pts = pts.astype(np.float32)
    origin = (-0.125, -0.125, -0.125)
    h = 0.25
    cap, key_lo, m_max, m_min = None, (0, 0, 0), 64, 1
    if variant == "grid":
        q = _grid_queries(ROOM_LO, ROOM_HI, grid_n, np.float32)
        traj = None
    elif variant == "batch":
        q = _rng(cfg_id, _S_QUERY).uniform(ROOM_LO, ROOM_HI, size=(n_random, 3)).astype(np.float32)
        key_lo, key_hi = _keys_bounds(pts, origin, h)
        cap = _cap_grid(_rng(cfg_id, _S_CAP), key_lo, key_hi)
        m_max, m_min = 128, 8
        traj = None
    else:
        q = _trajectories(_rng(cfg_id, _S_TRAJ), scene, n_traj, n_way, ROOM_LO, ROOM_HI, np.float32)
        traj = (n_traj, n_way)
    return Workload(cfg_id, f"room_{variant}", pts, origin, h, h / 2, m_max, m_min, q,
                    _sign(scene.free(q.astype(np.float64))), m_cap_grid=cap, key_lo=key_lo,
                    traj_shape=traj, scene=scene)


def room_trajectories(wl: Workload, n_traj=4096, n_way=64):
    """The trajectory queries of the 'traj' room workload, for a room workload already
    built (same scene and samples), without sampling the surfaces again."""
    q = _trajectories(_rng(4, _S_TRAJ), wl.scene, n_traj, n_way, ROOM_LO, ROOM_HI, np.float32)
    return q, _sign(wl.scene.free(q.astype(np.float64)))


def terrain_workload(grid_n=256, n_traj=16384, n_way=64, spacing=0.03, cfg_id=5,
                     size_scale=1.0, with_grid=True):
    """Large outdoor: value-noise terrain with buildings and trees; 3 cm spacing."""
    scene = TerrainScene(_rng(cfg_id, _S_GEOM), size_scale=size_scale)
    pts = scene.sample(_rng(cfg_id, _S_JITTER), _rng(cfg_id, _S_NOISE), spacing, 0.01).astype(np.float32)
    origin, h = (0.0, 0.0, 0.0), 0.5
    key_lo, key_hi = _keys_bounds(pts, origin, h)
    cap = _cap_grid(_rng(cfg_id, _S_CAP), key_lo, key_hi)
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([100.0, 100.0, 25.0])
    q = _grid_queries(lo, hi, grid_n, np.float32) if with_grid else np.zeros((0, 3), np.float32)
    return Workload(cfg_id, "terrain", pts, origin, h, h / 2, 128, 8, q,
                    _sign(scene.free(q.astype(np.float64))), m_cap_grid=cap, key_lo=key_lo,
                    scene=scene)


def terrain_trajectories(wl: Workload, n_traj=16384, n_way=64):
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([100.0, 100.0, 25.0])
    q = _trajectories(_rng(wl.cfg_id, _S_TRAJ), wl.scene, n_traj, n_way, lo, hi, np.float32)
    return q, _sign(wl.scene.free(q.astype(np.float64)))


def small_room_workload(n_queries=4096, cfg_id=12, spacing=0.04, n_boxes=3, n_cyl=2,
                        m_max=64, uneven=False):
    """A reduced room (fewer objects, coarser sampling) for tests the oracle finishes
    in seconds; same cell lattice and hyperparameters as the full room."""
    scene = RoomScene(_rng(cfg_id, _S_GEOM), n_boxes=n_boxes, n_cyl=n_cyl)
    density = None
    if uneven:
        n_obj = 6 + len(scene.boxes) + len(scene.cyls)
        density = np.exp(_rng(cfg_id, _S_DENS).uniform(np.log(0.1), np.log(4.0), n_obj))
    pts = scene.sample(_rng(cfg_id, _S_JITTER), _rng(cfg_id, _S_NOISE), spacing, 0.005,
                       density).astype(np.float32)
    origin, h = (-0.125, -0.125, -0.125), 0.25
    q = _rng(cfg_id, _S_QUERY).uniform(ROOM_LO, ROOM_HI, size=(n_queries, 3)).astype(np.float32)
    cap, key_lo, m_min = None, (0, 0, 0), 1
    if uneven:
        key_lo, key_hi = _keys_bounds(pts, origin, h)
        cap = _cap_grid(_rng(cfg_id, _S_CAP), key_lo, key_hi)
        m_max, m_min = 128, 8
    return Workload(cfg_id, "small_room", pts, origin, h, h / 2, m_max, m_min, q,
                    _sign(scene.free(q.astype(np.float64))), m_cap_grid=cap, key_lo=key_lo,
                    scene=scene)


def bhm_weights(wl, box=0.16, hinges=7, ell_bhm=0.016, weight=2.0):
    """Synthetic local Bayesian-Hilbert-map weights standing in for a trained front-end:
    a map for every box of edge `box` that holds a surface sample, its hinges^3 hinge
    points at the box's lattice points weighted +weight inside a solid and -weight in
    free space (the scene's analytic test), bias 0; kernel exp(-gamma |x - h|^2) with
    gamma = 1 / (2 ell_bhm^2).  Box size, hinge count and kernel scale follow the
    paper's indoor settings (two 0.08 m voxels, 7 hinges per axis, 0.016 m)."""
    pts = np.asarray(wl.points, np.float64)
    origin = pts.min(0) - box
    dims = np.ceil((pts.max(0) + box - origin) / box).astype(np.int64)
    keys = np.floor((pts - origin) / box).astype(np.int64)
    flat = np.unique((keys[:, 0] * dims[1] + keys[:, 1]) * dims[2] + keys[:, 2])
    box_bhm = np.full(int(np.prod(dims)), -1, np.int32)
    box_bhm[flat] = np.arange(len(flat), dtype=np.int32)
    kk = np.stack([flat // (dims[1] * dims[2]), (flat // dims[2]) % dims[1], flat % dims[2]], 1)
    g = np.arange(hinges) * (box / (hinges - 1))
    off = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    h = (origin + kk * box)[:, None, :] + off[None, :, :]
    free = wl.scene.free(h.reshape(-1, 3)).reshape(len(flat), -1)
    w = np.where(free, -weight, weight)
    weights = np.concatenate([w, np.zeros((len(flat), 1))], 1)
    return dict(origin=tuple(origin), box=box, dims=tuple(int(d) for d in dims), hinges=hinges,
                gamma=1.0 / (2 * ell_bhm * ell_bhm), box_bhm=box_bhm,
                weights=np.ascontiguousarray(weights.reshape(-1)))
