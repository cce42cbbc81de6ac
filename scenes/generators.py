"""Seeded synthetic inputs: triangle meshes, vehicle placement, radar arrays, waveforms.

This module produces input data only. It evaluates nothing of the scattering model,
the echo or the range-Doppler processing; the FP64 oracle and the GPU library both
consume the arrays it returns, each with its own arithmetic.

Conventions (the paper's intersection frame, Table 1): the radar sits on a pole at
(0, 0, 6) m, Y runs along the lanes, Z is up, X is across the lanes. Lane centres
are at x = 2, 5.75 and 9.5 m. Mesh vertices are float32 in the body frame (metres),
triangles are int32 with counter-clockwise order giving the outward normal.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Used only to place array elements on a half-wavelength grid (input geometry).
_C0 = 299_792_458.0

RADAR_POS = np.array([0.0, 0.0, 6.0])
LANE_CENTRES_X = (2.0, 5.75, 9.5)

VEHICLE_CLASSES = {
    # name: (length, width, height, n_wheels)
    "car": (4.5, 1.8, 1.5, 4),
    "bus": (12.0, 2.5, 3.0, 4),
    "truck": (8.0, 2.4, 3.2, 4),
    "motorcycle": (2.0, 0.8, 1.4, 2),
}


@dataclass
class Mesh:
    verts: np.ndarray  # float32 [V, 3], body frame
    tris: np.ndarray  # int32 [F, 3], CCW = outward
    name: str = ""

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


@dataclass
class Instance:
    mesh: int
    rot: np.ndarray  # float64 [3, 3], body -> world
    pos0: np.ndarray  # float64 [3], world position of the body origin at t = 0
    vel: np.ndarray  # float64 [3], world velocity (rigid translation)


@dataclass
class Points:
    pos0: np.ndarray  # float64 [n, 3]
    vel: np.ndarray  # float64 [n, 3]
    amp: np.ndarray  # complex128 [n], scattering amplitude in m^2

    @property
    def n(self) -> int:
        return int(self.pos0.shape[0])


@dataclass
class Scene:
    meshes: List[Mesh]
    instances: List[Instance]
    points: Optional[Points] = None

    @property
    def n_tris(self) -> int:
        return int(sum(self.meshes[i.mesh].n_tris for i in self.instances))


@dataclass
class Waveform:
    f0: float  # start frequency, Hz
    slope: float  # chirp slope mu, Hz/s
    fs: float  # ADC sample rate, Hz
    chirp_period: float  # T_c, s
    n_samples: int  # M
    n_chirps: int  # N


@dataclass
class RadarArray:
    tx: np.ndarray  # float64 [P, 3] world positions
    rx: np.ndarray  # float64 [Q, 3] world positions

    @property
    def n_channels(self) -> int:
        return int(self.tx.shape[0] * self.rx.shape[0])


@dataclass
class Config:
    name: str
    scenes: List[Scene]
    waveform: Waveform
    array: RadarArray
    seed: int
    notes: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------------
# waveforms
# ----------------------------------------------------------------------------------

def paper_waveform(n_samples: int, n_chirps: int) -> Waveform:
    """Experiment waveform of the paper's setup: fs 5.12 Msps, slope 12.5 MHz/us,
    start 77 GHz, chirp period = sampling time + 10 us idle (reproduces Table 2)."""
    fs = 5.12e6
    return Waveform(f0=77e9, slope=12.5e12, fs=fs,
                    chirp_period=n_samples / fs + 10e-6,
                    n_samples=n_samples, n_chirps=n_chirps)


def literal_77_81_waveform(n_samples: int = 128, n_chirps: int = 32) -> Waveform:
    """77-81 GHz swept in n_samples steps at 5.12 Msps (slope = 4 GHz * fs / M)."""
    fs = 5.12e6
    df = 4e9 / n_samples
    return Waveform(f0=77e9, slope=df * fs, fs=fs,
                    chirp_period=n_samples / fs + 10e-6,
                    n_samples=n_samples, n_chirps=n_chirps)


def _band_centre_wavelength(wf: Waveform) -> float:
    bw = wf.n_samples * wf.slope / wf.fs
    return _C0 / (wf.f0 + 0.5 * bw)


# ----------------------------------------------------------------------------------
# arrays
# ----------------------------------------------------------------------------------

def ula_1tx4rx(wf: Waveform, centre=RADAR_POS) -> RadarArray:
    """1 Tx + 4 Rx half-wavelength ULA along x (the paper's 1TX4RX layout)."""
    h = 0.5 * _band_centre_wavelength(wf)
    centre = np.asarray(centre, dtype=np.float64)
    rx = np.stack([centre + np.array([(i - 1.5) * h, 0.0, 0.0]) for i in range(4)])
    tx = (centre + np.array([-4.0 * h, 0.0, 0.0]))[None, :]
    return RadarArray(tx=tx.astype(np.float64), rx=rx.astype(np.float64))


def sparse_mimo_12x16(wf: Waveform, seed: int, centre=RADAR_POS) -> RadarArray:
    """Seeded sparse planar array in the x-z plane, boresight +Y.

    Rx: 16 of the first 32 half-wavelength x-slots. Tx: 12 of 24 slots laid out as
    8 x-positions at a 16-half-wavelength pitch times 3 z-rows {0, h, 2h}.
    """
    rng = np.random.default_rng(seed)
    h = 0.5 * _band_centre_wavelength(wf)
    centre = np.asarray(centre, dtype=np.float64)
    rx_slots = np.sort(rng.choice(32, size=16, replace=False))
    rx = np.stack([centre + np.array([(s - 15.5) * h, 0.0, 0.0]) for s in rx_slots])
    tx_slots = np.sort(rng.choice(24, size=12, replace=False))
    tx = []
    for s in tx_slots:
        ix, iz = divmod(int(s), 3)
        tx.append(centre + np.array([(ix - 3.5) * 16.0 * h, 0.0, (iz - 1) * h]))
    return RadarArray(tx=np.stack(tx), rx=rx)


# ----------------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------------

def _orient(verts: np.ndarray, tris: np.ndarray, normal_hint) -> np.ndarray:
    """Flip triangles whose winding disagrees with the wanted outward direction.
    normal_hint(centroids) -> [F,3] directions the normals should point along."""
    v = verts.astype(np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    nrm = np.cross(b - a, c - a)
    want = normal_hint((a + b + c) / 3.0)
    flip = np.einsum("ij,ij->i", nrm, want) < 0
    out = tris.copy()
    out[flip] = out[flip][:, [0, 2, 1]]
    return out


def _weld(verts: np.ndarray, tris: np.ndarray):
    uniq, inv = np.unique(verts, axis=0, return_inverse=True)
    return uniq, inv.reshape(-1)[tris]


def _grid_quads(p_of_ij, nu: int, nv: int):
    """Vertices [ (nu+1)(nv+1), 3 ] and triangles of an nu x nv quad grid patch."""
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nv + 1), indexing="ij")
    pts = p_of_ij(ii.reshape(-1), jj.reshape(-1))
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
    a = idx[:-1, :-1].reshape(-1)
    b = idx[1:, :-1].reshape(-1)
    c = idx[1:, 1:].reshape(-1)
    d = idx[:-1, 1:].reshape(-1)
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return pts, tris


def box_mesh(lo, hi, n) -> Mesh:
    """Closed axis-aligned box [lo, hi] with an n = (nx, ny, nz) quad grid per axis.
    Triangles: 4 (ny nz + nx nz + nx ny). The vertex grid along each axis is one
    linspace, so edges shared by two faces weld exactly."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    nx, ny, nz = (int(k) for k in n)
    ax = [np.linspace(lo[d], hi[d], (nx, ny, nz)[d] + 1) for d in range(3)]
    verts, tris, off = [], [], 0
    for d in range(3):
        u, w = [k for k in range(3) if k != d]
        for side in (0, 1):
            fixed = (lo, hi)[side][d]

            def p(i, j, d=d, u=u, w=w, fixed=fixed):
                out = np.empty((i.shape[0], 3))
                out[:, d] = fixed
                out[:, u] = ax[u][i]
                out[:, w] = ax[w][j]
                return out

            pts, t = _grid_quads(p, (nx, ny, nz)[u], (nx, ny, nz)[w])
            verts.append(pts)
            tris.append(t + off)
            off += pts.shape[0]
    verts = np.concatenate(verts).astype(np.float32)
    tris = np.concatenate(tris)
    verts, tris = _weld(verts, tris)
    centre = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)

    def hint(cen):
        r = (cen - centre) / half
        k = np.argmax(np.abs(r), axis=1)
        out = np.zeros_like(cen)
        out[np.arange(cen.shape[0]), k] = np.sign(r[np.arange(cen.shape[0]), k])
        return out

    tris = _orient(verts, tris, hint)
    return Mesh(verts=verts.astype(np.float32), tris=tris.astype(np.int32), name="box")


def cylinder_y_mesh(centre, radius, half_width, n_theta, n_len, n_rings) -> Mesh:
    """Capped cylinder with its axis along y (a wheel). Lateral grid n_theta x n_len,
    each cap a polar grid of n_rings rings (the innermost ring is a fan)."""
    cx, cy, cz = (float(x) for x in centre)
    th = np.linspace(0.0, 2.0 * np.pi, n_theta + 1)[:-1]
    ys = np.linspace(cy - half_width, cy + half_width, n_len + 1)
    verts, tris = [], []
    # lateral: vertex (k, i) = ring k along y, angle i
    lat = np.array([[cx + radius * np.cos(t), y, cz + radius * np.sin(t)]
                    for y in ys for t in th])
    idx = np.arange((n_len + 1) * n_theta).reshape(n_len + 1, n_theta)
    a = idx[:-1, :].reshape(-1)
    b = idx[:-1, np.r_[1:n_theta, 0]].reshape(-1)
    c = idx[1:, np.r_[1:n_theta, 0]].reshape(-1)
    d = idx[1:, :].reshape(-1)
    verts.append(lat)
    tris.append(np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]))
    off = lat.shape[0]
    for yc in (cy - half_width, cy + half_width):
        pts = [[cx, yc, cz]]
        for r in range(1, n_rings + 1):
            rr = radius * r / n_rings
            pts += [[cx + rr * np.cos(t), yc, cz + rr * np.sin(t)] for t in th]
        pts = np.array(pts)
        t = []
        nxt = np.r_[1:n_theta, 0]
        ring1 = 1 + np.arange(n_theta)
        t.append(np.stack([np.zeros(n_theta, int), ring1, 1 + nxt], 1))
        for r in range(1, n_rings):
            inner = 1 + (r - 1) * n_theta + np.arange(n_theta)
            outer = 1 + r * n_theta + np.arange(n_theta)
            inner_n = 1 + (r - 1) * n_theta + nxt
            outer_n = 1 + r * n_theta + nxt
            t.append(np.stack([inner, outer, outer_n], 1))
            t.append(np.stack([inner, outer_n, inner_n], 1))
        verts.append(pts)
        tris.append(np.concatenate(t) + off)
        off += pts.shape[0]
    verts = np.concatenate(verts).astype(np.float32)
    tris = np.concatenate(tris)

    def hint(cen):
        out = np.zeros_like(cen)
        on_cap = np.abs(np.abs(cen[:, 1] - cy) - half_width) < 1e-6
        out[on_cap, 1] = np.sign(cen[on_cap, 1] - cy)
        lat_ = ~on_cap
        out[lat_, 0] = cen[lat_, 0] - cx
        out[lat_, 2] = cen[lat_, 2] - cz
        return out

    tris = _orient(verts, tris, hint)
    return Mesh(verts=verts, tris=tris.astype(np.int32), name="cylinder")


def merge_meshes(parts: List[Mesh], name: str = "") -> Mesh:
    verts, tris, off = [], [], 0
    for m in parts:
        verts.append(m.verts)
        tris.append(m.tris.astype(np.int64) + off)
        off += m.verts.shape[0]
    return Mesh(verts=np.concatenate(verts).astype(np.float32),
                tris=np.concatenate(tris).astype(np.int32), name=name)


def _hull_parts(length, width, height, n_wheels, cell):
    """Body box + cabin box + capped wheel cylinders at cell size `cell` (metres)."""
    rw = 0.2 * height
    hw = 0.1 * width
    zb0, zb1 = 0.8 * rw, 0.62 * height
    parts = []

    def nseg(extent):
        return max(1, int(np.ceil(extent / cell)))

    body_lo = (-0.5 * length, -0.5 * width, zb0)
    body_hi = (0.5 * length, 0.5 * width, zb1)
    parts.append(box_mesh(body_lo, body_hi,
                          (nseg(length), nseg(width), nseg(zb1 - zb0))))
    # the cabin floor sits 2 cm inside the body and the wheels stand 2 cm proud of the
    # body sides, so no two parts share a plane (no coplanar overlapping triangles)
    cab_lo = (-0.30 * length, -0.45 * width, zb1 - 0.02)
    cab_hi = (0.25 * length, 0.45 * width, height)
    parts.append(box_mesh(cab_lo, cab_hi,
                          (nseg(0.55 * length), nseg(0.9 * width), nseg(height - zb1 + 0.02))))
    n_theta = max(8, nseg(2 * np.pi * rw))
    n_len = nseg(2 * hw)
    n_rings = max(1, nseg(rw))
    if n_wheels == 2:
        spots = [(-0.35 * length, 0.0), (0.35 * length, 0.0)]
    else:
        spots = [(sx * 0.32 * length, sy * (0.5 * width - hw + 0.02))
                 for sx in (-1, 1) for sy in (-1, 1)]
    for (x, y) in spots:
        parts.append(cylinder_y_mesh((x, y, rw), rw, hw, n_theta, n_len, n_rings))
    return parts


def _hull_count(length, width, height, n_wheels, cell):
    rw = 0.2 * height
    hw = 0.1 * width
    zb0, zb1 = 0.8 * rw, 0.62 * height

    def nseg(extent):
        return max(1, int(np.ceil(extent / cell)))

    def box(nx, ny, nz):
        return 4 * (ny * nz + nx * nz + nx * ny)

    n = box(nseg(length), nseg(width), nseg(zb1 - zb0))
    n += box(nseg(0.55 * length), nseg(0.9 * width), nseg(height - zb1 + 0.02))
    n_theta = max(8, nseg(2 * np.pi * rw))
    n_len = nseg(2 * hw)
    n_rings = max(1, nseg(rw))
    n += n_wheels * (2 * n_theta * n_len + 2 * n_theta * (2 * n_rings - 1))
    return n


def hull_mesh(length, width, height, n_wheels, target_tris) -> Mesh:
    """Procedural vehicle hull with about target_tris triangles (exact count varies).

    Overlapping parts are allowed: wheels poke into the body, the cabin sits on it;
    interior faces end up shadowed by the visibility test."""
    lo, hi = 1e-3, 2.0
    for _ in range(60):
        mid = np.sqrt(lo * hi)
        if _hull_count(length, width, height, n_wheels, mid) > target_tris:
            lo = mid
        else:
            hi = mid
    cands = [lo, hi]
    cell = min(cands, key=lambda c: abs(_hull_count(length, width, height, n_wheels, c)
                                        - target_tris))
    return merge_meshes(_hull_parts(length, width, height, n_wheels, cell),
                        name=f"hull{length}x{width}x{height}")


def vehicle_mesh(cls: str, target_tris: int) -> Mesh:
    L, W, H, nw = VEHICLE_CLASSES[cls]
    m = hull_mesh(L, W, H, nw, target_tris)
    m.name = cls
    return m


def ground_grid(x0, x1, y0, y1, cell) -> Mesh:
    nx = int(round((x1 - x0) / cell))
    ny = int(round((y1 - y0) / cell))
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)

    def p(i, j):
        return np.stack([xs[i], ys[j], np.zeros(i.shape[0])], 1)

    pts, tris = _grid_quads(p, nx, ny)
    tris = _orient(pts, tris, lambda c: np.tile([0.0, 0.0, 1.0], (c.shape[0], 1)))
    return Mesh(verts=pts.astype(np.float32), tris=tris.astype(np.int32), name="ground")


# ----------------------------------------------------------------------------------
# placement
# ----------------------------------------------------------------------------------

def yaw_matrix(yaw: float) -> np.ndarray:
    """Rotation about +z taking body +x (vehicle length) to heading (cos yaw, sin yaw)."""
    c, s = np.cos(yaw), np.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _instance_from(mesh_idx, x, y, yaw, speed):
    rot = yaw_matrix(yaw)
    heading = rot[:, 0]
    return Instance(mesh=mesh_idx, rot=rot, pos0=np.array([x, y, 0.0]),
                    vel=speed * heading)


def place_single(rng, height, range_lo, range_hi, az_deg=45.0, yaw_dev_deg=10.0,
                 speed_max=15.0):
    """Seeded pose for one vehicle: slant range from the radar to the body centre,
    azimuth within +-az_deg of boresight, heading along +-Y +- yaw_dev_deg."""
    r = rng.uniform(range_lo, range_hi)
    az = np.deg2rad(rng.uniform(-az_deg, az_deg))
    dz = RADAR_POS[2] - 0.5 * height
    rho = np.sqrt(max(r * r - dz * dz, 1.0))
    x, y = rho * np.sin(az), rho * np.cos(az)
    yaw = (np.pi / 2 if rng.uniform() < 0.5 else -np.pi / 2) + np.deg2rad(
        rng.uniform(-yaw_dev_deg, yaw_dev_deg))
    speed = rng.uniform(-speed_max, speed_max)
    return x, y, yaw, speed


def place_many(rng, classes, max_slant=58.0, gap=0.5, box=(-30.0, 30.0, 0.0, 60.0),
               p_along_y=0.7, speed_max=15.0, max_tries=20000):
    """Rejection-sampled non-overlapping footprints inside box, slant range <= max_slant."""
    placed = []  # (x, y, yaw, speed, half_x, half_y) axis-aligned footprint extents
    for cls in classes:
        L, W, H, _ = VEHICLE_CLASSES[cls]
        for _ in range(max_tries):
            x = rng.uniform(box[0], box[1])
            y = rng.uniform(box[2], box[3])
            along_y = rng.uniform() < p_along_y
            yaw = (np.pi / 2 if along_y else 0.0) + (np.pi if rng.uniform() < 0.5 else 0.0)
            hx, hy = ((0.5 * W, 0.5 * L) if along_y else (0.5 * L, 0.5 * W))
            if x - hx < box[0] or x + hx > box[1] or y - hy < box[2] or y + hy > box[3]:
                continue
            slant = np.sqrt(x * x + y * y + (RADAR_POS[2] - 0.5 * H) ** 2)
            if slant > max_slant or np.hypot(x, y) < 3.0:
                continue
            ok = all(abs(x - px) >= hx + phx + gap or abs(y - py) >= hy + phy + gap
                     for (px, py, _, _, phx, phy) in placed)
            if ok:
                placed.append((x, y, yaw, rng.uniform(-speed_max, speed_max), hx, hy))
                break
        else:
            raise RuntimeError("placement failed; box too crowded")
    return [(p[0], p[1], p[2], p[3]) for p in placed]


# ----------------------------------------------------------------------------------
# simple scenes used by tests
# ----------------------------------------------------------------------------------

def point_scene(ranges, range_rates, amps=None, az_deg=None, height=1.0) -> Scene:
    """Point scatterers at the given slant ranges (m) with the given range rates
    (m/s, positive = receding), on bearings az_deg (default 0) from boresight."""
    ranges = np.atleast_1d(np.asarray(ranges, np.float64))
    rates = np.atleast_1d(np.asarray(range_rates, np.float64))
    n = ranges.shape[0]
    az = np.zeros(n) if az_deg is None else np.deg2rad(np.atleast_1d(az_deg))
    dz = height - RADAR_POS[2]
    rho = np.sqrt(ranges ** 2 - dz ** 2)
    pos = np.stack([rho * np.sin(az), rho * np.cos(az), np.full(n, height)], 1)
    u = (pos - RADAR_POS) / ranges[:, None]
    vel = rates[:, None] * u
    a = np.ones(n, np.complex128) if amps is None else np.asarray(amps, np.complex128)
    return Scene(meshes=[], instances=[], points=Points(pos0=pos, vel=vel, amp=a))


def plate_scene(a, b, n_a, n_b, distance, tilt_rad=0.0, centre=RADAR_POS) -> Scene:
    """Flat a x b plate facing the radar along +Y at `distance`, tilted by tilt_rad
    about the world z axis (the plate's b-edge). Mesh in the body x-z plane, normal -Y."""
    xs = np.linspace(-0.5 * a, 0.5 * a, n_a + 1)
    zs = np.linspace(-0.5 * b, 0.5 * b, n_b + 1)

    def p(i, j):
        return np.stack([xs[i], np.zeros(i.shape[0]), zs[j]], 1)

    pts, tris = _grid_quads(p, n_a, n_b)
    tris = _orient(pts, tris, lambda c: np.tile([0.0, -1.0, 0.0], (c.shape[0], 1)))
    mesh = Mesh(verts=pts.astype(np.float32), tris=tris.astype(np.int32), name="plate")
    rot = yaw_matrix(tilt_rad)
    pos0 = np.asarray(centre, np.float64) + np.array([0.0, distance, 0.0])
    inst = Instance(mesh=0, rot=rot, pos0=pos0, vel=np.zeros(3))
    return Scene(meshes=[mesh], instances=[inst])


def dihedral_scene(a, b, distance, n_a=1, n_b=1, centre=RADAR_POS) -> Scene:
    """Right-angle dihedral (two a x b plates meeting on a fold line of length a along
    world x) at `distance` along +Y from `centre`, opening towards it: the plates leave the
    fold at +45 and -45 degrees from the line of sight in the y-z plane, with normals
    facing into the corner. Each plate is an n_a x n_b grid of quads (two triangles each)."""
    xs = np.linspace(-0.5 * a, 0.5 * a, n_a + 1)
    ss = np.linspace(0.0, b, n_b + 1)
    h = np.sqrt(0.5)
    meshes_pts, meshes_tris = [], []
    for sign in (1.0, -1.0):
        def p(i, j, sign=sign):
            return np.stack([xs[i], -h * ss[j], sign * h * ss[j]], 1)
        pts, tris = _grid_quads(p, n_a, n_b)
        nrm = np.array([0.0, -h, -sign * h])
        tris = _orient(pts, tris, lambda c, nrm=nrm: np.tile(nrm, (c.shape[0], 1)))
        meshes_pts.append(pts)
        meshes_tris.append(tris)
    off = meshes_pts[0].shape[0]
    pts = np.concatenate(meshes_pts)
    tris = np.concatenate([meshes_tris[0], meshes_tris[1] + off])
    mesh = Mesh(verts=pts.astype(np.float32), tris=tris.astype(np.int32), name="dihedral")
    pos0 = np.asarray(centre, np.float64) + np.array([0.0, distance, 0.0])
    inst = Instance(mesh=0, rot=np.eye(3), pos0=pos0, vel=np.zeros(3))
    return Scene(meshes=[mesh], instances=[inst])


# ----------------------------------------------------------------------------------
# synthetic range-Doppler cubes for the detection stage
# ----------------------------------------------------------------------------------

def synthetic_y_cube(arr: RadarArray, wf: Waveform, seed: int, targets, noise_sigma: float = 1.0):
    """Seeded complex cube Y[O, N, M] standing in for the Doppler-FFT output: circular
    complex Gaussian noise of standard deviation noise_sigma per element plus, for each
    target (row, bin, amplitude, u, w), a plane wave over the virtual array at that cell,
    amplitude * exp(-j 2 pi (u x + w z) / lambda_c) with (x, z) the virtual element
    positions tx_p + rx_q. Returns complex64."""
    rng = np.random.default_rng(seed)
    O = arr.n_channels
    N, M = wf.n_chirps, wf.n_samples
    Y = (rng.normal(size=(O, N, M)) + 1j * rng.normal(size=(O, N, M))) * (noise_sigma / np.sqrt(2.0))
    lam = _band_centre_wavelength(wf)
    v = (arr.tx[:, None, :] + arr.rx[None, :, :]).reshape(-1, 3)
    for row, col, amp, u, w in targets:
        Y[:, row, col] += amp * np.exp(-2j * np.pi * (u * v[:, 0] + w * v[:, 2]) / lam)
    return Y.astype(np.complex64)


def scene_digest(scene: Scene) -> str:
    """Short hash of a scene's generated geometry and motion (vertices, triangles,
    rotations, start positions, velocities), so that stored expectations can detect
    generator drift."""
    import hashlib
    h = hashlib.sha256()
    for m in scene.meshes:
        h.update(np.ascontiguousarray(m.verts, np.float32).tobytes())
        h.update(np.ascontiguousarray(m.tris, np.int32).tobytes())
    for i in scene.instances:
        for a in (i.rot, i.pos0, i.vel):
            h.update(np.ascontiguousarray(a, np.float64).tobytes())
    return h.hexdigest()[:16]
