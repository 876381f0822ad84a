"""Seeded synthetic inputs: Gaussian scenes, cameras and target images.

This module is shared by the tests, the benchmark and the oracle checks. It only
draws inputs (positions, scales, rotations, opacities, SH coefficients, camera
poses); it holds none of the rendering arithmetic. Every array is drawn in
float64 with NumPy's PCG64 generator and then cast to float32, the precision the
splatting model takes its parameters in (Sec. 3.2: position p, opacity o, SH
coefficients k, scale s, rotation quaternion q).

Layouts (structure of arrays, one column per Gaussian):
  mean    [3][N]          world-space centre p
  scale   [3][N]          linear scales s (> 0)
  quat    [4][N]          rotation quaternion (w, x, y, z), any non-zero norm
  opacity [N]             o in (0, 1)
  sh      [(d+1)^2*3][N]  SH coefficients, row (k*3 + c) holds coefficient k of
                          colour channel c; d is the SH degree (0..3)

Cameras are pinhole, world-to-camera p_c = R p + t with x right, y down and z
forward; pixel (px, py) is sampled at its centre (px + 0.5, py + 0.5).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

SEED_GAUSSIANS = 0
SEED_TARGETS = 1
SEED_CAMERAS = 2
SEED_KMEANS = 3
SEED_IMAGES = 4


@dataclass
class Scene:
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.mean[:, idx]), np.ascontiguousarray(self.scale[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]), np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, idx]), self.sh_degree)

    def concat(self, other: "Scene") -> "Scene":
        assert other.sh_degree == self.sh_degree
        return Scene(np.concatenate([self.mean, other.mean], 1), np.concatenate([self.scale, other.scale], 1),
                     np.concatenate([self.quat, other.quat], 1), np.concatenate([self.opacity, other.opacity]),
                     np.concatenate([self.sh, other.sh], 1), self.sh_degree)


@dataclass
class Camera:
    R: np.ndarray            # (3, 3) float32, world -> camera rotation
    t: np.ndarray            # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def position(self) -> np.ndarray:
        """Camera centre in world coordinates (float64)."""
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclass
class Params:
    """Model constants the paper leaves open; defaults follow the readings in the design notes."""
    lowpass: float = 0.3
    kappa: float = 3.0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    guard: float = 1.3
    bg: List[float] = field(default_factory=lambda: [0.0, 0.0, 0.0])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def uniform_cube_scene(n=2000, seed=SEED_GAUSSIANS) -> Scene:
    """Plain forward-render scene: means U[-1,1]^3, log-scales N(-3, 0.5), uniform rotations,
    opacity sigmoid(N(0,1)), SH degree 0 whose evaluation gives an RGB drawn from U(0,1)."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, (3, n))
    scale = np.exp(rng.normal(-3.0, 0.5, (3, n)))
    quat = _unit_quats(rng, n)
    opacity = _sigmoid(rng.standard_normal(n))
    rgb = rng.uniform(0.0, 1.0, (3, n))
    # degree-0 band is the constant 1/(2 sqrt(pi)); pick k0 so that k0 * Y00 + 0.5 = rgb
    sh = (rgb - 0.5) * (2.0 * np.sqrt(np.pi))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), 0)


def _random_rotation(rng):
    a = rng.standard_normal((3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))[None, :]
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def mixture_scene(n, seed=SEED_GAUSSIANS, n_clusters=32, radius=10.0, log_scale_mu=-4.0,
                  log_scale_sigma=0.7, sh_degree=3, sh_sigma=0.2) -> Scene:
    """Unbounded-360-like scene: a mixture of anisotropic 3D Gaussian clusters in a ball.

    32 cluster centres uniform in a ball of the given radius; per-cluster axis standard
    deviations log-uniform in [0.5, 3] under a random rotation; equal weights; samples
    outside the ball are redrawn. Log-scales N(mu, sigma), uniform rotations, opacity
    sigmoid(N(0,1)), every SH coefficient N(0, sh_sigma). Storage order is random
    (labels are drawn independently), as in a scene grown by densification.
    """
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n_clusters, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = d * (radius * rng.uniform(0.0, 1.0, (n_clusters, 1)) ** (1.0 / 3.0))
    stds = np.exp(rng.uniform(np.log(0.5), np.log(3.0), (n_clusters, 3)))
    rots = np.stack([_random_rotation(rng) for _ in range(n_clusters)])
    labels = rng.integers(0, n_clusters, n)
    pts = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        lab = labels[todo]
        z = rng.standard_normal((todo.size, 3)) * stds[lab]
        p = centres[lab] + np.einsum("nij,nj->ni", rots[lab], z)
        ok = np.linalg.norm(p, axis=1) <= radius
        pts[todo[ok]] = p[ok]
        todo = todo[~ok]
    scale = np.exp(rng.normal(log_scale_mu, log_scale_sigma, (3, n)))
    quat = _unit_quats(rng, n)
    opacity = _sigmoid(rng.standard_normal(n))
    rows = (sh_degree + 1) ** 2 * 3
    sh = rng.normal(0.0, sh_sigma, (rows, n))
    return Scene(_f32(pts.T), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), sh_degree)


def look_at_camera(position, target, width, height, fx=None, fy=None, znear=0.2) -> Camera:
    """Pinhole camera at `position` looking at `target`, world up = -y (image y points down)."""
    pos = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    down = np.array([0.0, 1.0, 0.0])
    y = down - np.dot(down, fwd) * fwd
    if np.linalg.norm(y) < 1e-9:
        y = np.array([0.0, 0.0, 1.0]) - fwd[2] * fwd
    y /= np.linalg.norm(y)
    x = np.cross(y, fwd)
    R = np.stack([x, y, fwd])
    t = -R @ pos
    if fx is None:
        fx = 0.78 * width
    if fy is None:
        fy = fx
    return Camera(_f32(R), _f32(t), float(np.float32(fx)), float(np.float32(fy)), float(np.float32(width / 2.0)),
                  float(np.float32(height / 2.0)), int(width), int(height), float(np.float32(znear)))


def orbit_camera(azimuth, elevation, radius, width, height, fx=None) -> Camera:
    """Orbit pose: centre radius*(cos e sin a, -sin e, -cos e cos a), looking at the origin."""
    pos = radius * np.array([np.cos(elevation) * np.sin(azimuth), -np.sin(elevation),
                             -np.cos(elevation) * np.cos(azimuth)])
    return look_at_camera(pos, np.zeros(3), width, height, fx)


def plain_view() -> Camera:
    """The 128x96 view, fx = fy = 100, camera at (0, 0, -4) looking at the origin (R = I)."""
    return Camera(np.eye(3, dtype=np.float32), np.array([0, 0, 4], np.float32), 100.0, 100.0, 64.0, 48.0, 128, 96,
                  float(np.float32(0.2)))


def orbit_views(n_views, width=1256, height=828, radius=4.0, seed=SEED_CAMERAS) -> List[Camera]:
    """Orbit of n views: azimuth 2 pi k / n, elevation U(-15, 30) degrees, radius 4."""
    rng = np.random.default_rng(seed)
    elev = np.deg2rad(rng.uniform(-15.0, 30.0, n_views))
    return [orbit_camera(2 * np.pi * k / n_views, elev[k], radius, width, height) for k in range(n_views)]


UNEVEN_SIZES = [(640, 480), (800, 600), (1024, 768), (1256, 828), (1280, 720), (1440, 960), (1600, 1064),
                (1920, 1080)]


def uneven_views(sizes=UNEVEN_SIZES, elevation_deg=10.0, radius=4.0) -> List[Camera]:
    """Batch of views of uneven resolution: azimuths k * 45 degrees, elevation 10 degrees."""
    return [orbit_camera(np.deg2rad(45.0 * k), np.deg2rad(elevation_deg), radius, w, h)
            for k, (w, h) in enumerate(sizes)]


def target_images(cams, seed=SEED_TARGETS) -> List[np.ndarray]:
    """U(0,1) target images, planar [3][H][W] float32 per view."""
    rng = np.random.default_rng(seed)
    return [_f32(rng.uniform(0.0, 1.0, (3, c.height, c.width))) for c in cams]


def image_pair(n_planes, height, width, seed=SEED_IMAGES):
    """Render-like image x and target y, [n_planes][height][width] float32 in [0, 1]: smooth
    low-frequency content (a few random sinusoids), pixel noise, a flat patch (zero local
    variance) and saturated regions at 0 and 1; y is x with a smooth shift, its own noise and a
    flat patch of another value."""
    rng = np.random.default_rng(seed)
    i = np.arange(height, dtype=np.float64)[:, None]
    j = np.arange(width, dtype=np.float64)[None, :]

    def smooth():
        f = np.zeros((height, width))
        for _ in range(4):
            ky, kx = rng.uniform(0.01, 0.2, 2)
            f += rng.uniform(0.1, 0.3) * np.sin(ky * i + kx * j + rng.uniform(0, 2 * np.pi))
        return f

    x = np.empty((n_planes, height, width))
    y = np.empty_like(x)
    for p in range(n_planes):
        x[p] = 0.5 + smooth() + rng.normal(0.0, 0.05, (height, width))
        y[p] = x[p] + 0.3 * smooth() + rng.normal(0.0, 0.05, (height, width))
        h0, w0 = height // 3, width // 3
        x[p, h0:h0 + max(1, height // 4), w0:w0 + max(1, width // 4)] = 0.25
        y[p, h0:h0 + max(1, height // 5), w0:w0 + max(1, width // 5)] = 0.75
    return _f32(np.clip(x, 0.0, 1.0)), _f32(np.clip(y, 0.0, 1.0))


# ---------------------------------------------------------------------------------------------
# House-scale scene: two floors of 3 x 2 rooms (10 x 10 x 3 m each) in a 30 x 20 x 6 m box.
# ---------------------------------------------------------------------------------------------

ROOM = 10.0
FLOOR_H = 3.0


def _room_origin(floor, rx, rz):
    # world y points down: floor f occupies y in [-(f+1)*3, -f*3]
    return np.array([rx * ROOM, -floor * FLOOR_H, rz * ROOM])


def house_scene(n, seed=SEED_GAUSSIANS, sh_degree=3) -> Scene:
    """House-like scene of 12 rooms. About 60% of the Gaussians lie flat on walls, floors and
    ceilings (normal log-scale -6, tangent log-scales N(-3.5, 0.5), opacity sigmoid(N(2,1))),
    with 1 x 2 m doorways left open in the interior walls; the other 40% form clutter clusters
    inside the rooms (log-scales N(-4, 0.7), opacity sigmoid(N(0,1)))."""
    rng = np.random.default_rng(seed)
    rooms = [(f, rx, rz) for f in range(2) for rx in range(3) for rz in range(2)]
    n_surf = int(round(0.6 * n))
    n_clut = n - n_surf
    # faces: kind 0 floor, 1 ceiling, 2 wall x = x0, 3 wall x = x0 + 10, 4 wall z = z0, 5 wall z = z0 + 10
    f_org, f_kind, f_inner, f_area = [], [], [], []
    for (f, rx, rz) in rooms:
        o = _room_origin(f, rx, rz)
        for kind in range(6):
            inner = {2: rx > 0, 3: rx < 2, 4: rz > 0, 5: rz < 1}.get(kind, False)
            f_org.append(o)
            f_kind.append(kind)
            f_inner.append(inner)
            f_area.append(ROOM * ROOM if kind < 2 else ROOM * FLOOR_H)
    f_org, f_kind, f_inner, f_area = (np.array(f_org), np.array(f_kind), np.array(f_inner), np.array(f_area))
    which = rng.choice(len(f_kind), n_surf, p=f_area / f_area.sum())
    pts = np.empty((n_surf, 3))
    normal_axis = np.empty(n_surf, np.int64)
    todo = np.arange(n_surf)
    while todo.size:
        fc = which[todo]
        a = rng.uniform(0, 1, todo.size)
        b = rng.uniform(0, 1, todo.size)
        o, kind = f_org[fc], f_kind[fc]
        p = np.empty((todo.size, 3))
        ax = np.empty(todo.size, np.int64)
        flat = kind < 2
        p[flat, 0] = o[flat, 0] + a[flat] * ROOM
        p[flat, 1] = o[flat, 1] - FLOOR_H * (kind[flat] == 1)
        p[flat, 2] = o[flat, 2] + b[flat] * ROOM
        ax[flat] = 1
        h = o[:, 1] - b * FLOOR_H  # wall height coordinate (y points down)
        xw = (kind == 2) | (kind == 3)
        p[xw, 0] = o[xw, 0] + ROOM * (kind[xw] == 3)
        p[xw, 1] = h[xw]
        p[xw, 2] = o[xw, 2] + a[xw] * ROOM
        ax[xw] = 0
        zw = (kind == 4) | (kind == 5)
        p[zw, 0] = o[zw, 0] + a[zw] * ROOM
        p[zw, 1] = h[zw]
        p[zw, 2] = o[zw, 2] + ROOM * (kind[zw] == 5)
        ax[zw] = 2
        # 1 m wide, 2 m high doorway in the middle of each interior wall
        door = f_inner[fc] & ~flat & (np.abs(a * ROOM - ROOM / 2) < 0.5) & ((o[:, 1] - h) < 2.0)
        keep = ~door
        pts[todo[keep]] = p[keep]
        normal_axis[todo[keep]] = ax[keep]
        todo = todo[door]
    surf_scale = np.exp(rng.normal(-3.5, 0.5, (3, n_surf)))
    surf_scale[normal_axis, np.arange(n_surf)] = np.exp(-6.0)
    surf_quat = np.zeros((4, n_surf))
    # rotation about the surface normal only keeps the thin axis on the normal
    ang = rng.uniform(0, np.pi, n_surf)
    surf_quat[0] = np.cos(ang)
    surf_quat[1 + normal_axis, np.arange(n_surf)] = np.sin(ang)
    surf_opac = _sigmoid(rng.normal(2.0, 1.0, n_surf))
    # clutter: 8 clusters per room, std 0.2 - 0.8 m, inside the room
    centres = []
    for (f, rx, rz) in rooms:
        o = _room_origin(f, rx, rz)
        for _ in range(8):
            centres.append(o + np.array([rng.uniform(1, ROOM - 1), -rng.uniform(0.3, 2.0), rng.uniform(1, ROOM - 1)]))
    centres = np.array(centres)
    cstd = rng.uniform(0.2, 0.8, len(centres))
    lab = rng.integers(0, len(centres), n_clut)
    clut = centres[lab] + rng.standard_normal((n_clut, 3)) * cstd[lab, None]
    clut_scale = np.exp(rng.normal(-4.0, 0.7, (3, n_clut)))
    clut_quat = _unit_quats(rng, n_clut)
    clut_opac = _sigmoid(rng.standard_normal(n_clut))
    mean = np.concatenate([pts, clut]).T
    scale = np.concatenate([surf_scale, clut_scale], 1)
    quat = np.concatenate([surf_quat, clut_quat], 1)
    opac = np.concatenate([surf_opac, clut_opac])
    perm = rng.permutation(n)
    rows = (sh_degree + 1) ** 2 * 3
    sh = rng.normal(0.0, 0.2, (rows, n))
    return Scene(_f32(mean[:, perm]), _f32(scale[:, perm]), _f32(quat[:, perm]), _f32(opac[perm]), _f32(sh),
                 sh_degree)


def house_training_views(n_views=640, width=1920, height=1080, seed=SEED_CAMERAS) -> List[Camera]:
    """Training cameras spread over the 12 rooms: position uniform in the room inset by 1 m, eye
    height floor + U(1.2, 1.8) m, yaw U(0, 360) degrees, pitch U(-15, 15) degrees."""
    rng = np.random.default_rng(seed)
    rooms = [(f, rx, rz) for f in range(2) for rx in range(3) for rz in range(2)]
    cams = []
    for k in range(n_views):
        f, rx, rz = rooms[k % len(rooms)]
        o = _room_origin(f, rx, rz)
        pos = o + np.array([rng.uniform(1, ROOM - 1), -rng.uniform(1.2, 1.8), rng.uniform(1, ROOM - 1)])
        yaw = rng.uniform(0, 2 * np.pi)
        pitch = np.deg2rad(rng.uniform(-15, 15))
        d = np.array([np.cos(pitch) * np.sin(yaw), -np.sin(pitch), np.cos(pitch) * np.cos(yaw)])
        cams.append(look_at_camera(pos, pos + d, width, height))
    return cams


def house_camera_positions(m, seed=SEED_CAMERAS) -> np.ndarray:
    """[m][3] float64 camera centres drawn like house_training_views (room k mod 12, uniform in
    the room inset by 1 m, eye height floor + U(1.2, 1.8) m), for camera sets too large to
    build views for, such as the frames of a long capture."""
    rng = np.random.default_rng(seed)
    rooms = np.array([_room_origin(f, rx, rz) for f in range(2) for rx in range(3) for rz in range(2)])
    o = rooms[np.arange(m) % len(rooms)]
    off = np.stack([rng.uniform(1, ROOM - 1, m), -rng.uniform(1.2, 1.8, m), rng.uniform(1, ROOM - 1, m)], 1)
    return np.ascontiguousarray(o + off, np.float64)


def house_test_path(n_frames=300, width=1920, height=1080) -> List[Camera]:
    """Closed path per floor through the room centres and doorways at eye height 1.6 m, looking
    along the direction of travel; half the frames on each floor."""
    cams = []
    per_floor = n_frames // 2
    loop = [(0, 0), (0, 1), (1, 1), (2, 1), (2, 0), (1, 0)]
    for f in range(2):
        way = []
        for i, (rx, rz) in enumerate(loop):
            c = _room_origin(f, rx, rz) + np.array([ROOM / 2, -1.6, ROOM / 2])
            way.append(c)
            nx, nz = loop[(i + 1) % len(loop)]
            nc = _room_origin(f, nx, nz) + np.array([ROOM / 2, -1.6, ROOM / 2])
            way.append(0.5 * (c + nc))  # doorway between the two rooms
        way = np.array(way)
        seg = np.linalg.norm(np.roll(way, -1, 0) - way, axis=1)
        s_tot = seg.sum()
        for j in range(per_floor):
            s = s_tot * j / per_floor
            k = 0
            while s > seg[k]:
                s -= seg[k]
                k += 1
            a, b = way[k], way[(k + 1) % len(way)]
            pos = a + (b - a) * (s / seg[k])
            cams.append(look_at_camera(pos, pos + (b - a), width, height))
    return cams
