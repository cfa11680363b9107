"""Seeded synthetic scene generators.

This module produces plain NumPy arrays describing an animated triangle
scene (materials, meshes, keyframed rigid instances, optional point lights,
a keyframed pinhole camera).  It holds none of the renderer's arithmetic:
no instance transform is applied here, no ray is traced, nothing is
sampled.  The same arrays feed both the GPU library and the CPU oracle.

The paper evaluates on four scenes (two made in Blender, two public pbrt
scenes; Sec. 4) that are not available here, so these procedural scenes
stand in for them:

* ``tiny_box``   -- an open box with a ceiling light and a small moving cube
  (stands in for the paper's "two boxes"), 64x64.
* ``sensor``     -- a displaced heightfield floor with 20 icospheres moving
  rigidly and three area lights (an occluder-rich stand-in for the paper's
  larger scenes), 640x480, ~98k triangles.
* closed-form test scenes (white furnace, plane under a point light, plane
  under a triangle area light) and random triangle soups.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Scene:
    albedo: np.ndarray          # float32 [n_mat]
    emission: np.ndarray        # float32 [n_mat]
    xyz: np.ndarray             # float32 [n_vert, 3] object-space vertices
    tri_idx: np.ndarray         # uint32 [n_tri, 3] (global vertex indices)
    tri_mat: np.ndarray         # uint32 [n_tri]
    mesh_tri_off: np.ndarray    # uint32 [n_mesh + 1]
    inst_mesh: np.ndarray       # uint32 [n_inst]
    inst_key_off: np.ndarray    # uint32 [n_inst + 1]
    key_t: np.ndarray           # float64 [n_keys]
    key_xform: np.ndarray       # float64 [n_keys, 3, 4]
    pl_pos: np.ndarray          # float32 [n_plight, 3]
    pl_intensity: np.ndarray    # float32 [n_plight]
    width: int
    height: int
    vfov_deg: float
    cam_t: np.ndarray           # float64 [n_cam_keys]
    cam_elu: np.ndarray         # float64 [n_cam_keys, 9] eye, look-at, up
    # Environment cube map (grey radiance, faces +x, -x, +y, -y, +z, -z,
    # [6, N, N] rows j then columns i; None: black background) and thin lens
    # (aperture radius 0: pinhole; distance of the plane in focus).
    env: Optional[np.ndarray] = None
    lens_radius: float = 0.0
    focus_dist: float = 1.0
    # RGB radiance (None: grey): per material albedo_rgb [n_mat, 3] in
    # [0, 1) and emission_rgb [n_mat, 3] >= 0 (linear Rec. 709 primaries),
    # optional per point light pl_rgb [n_plight, 3] (None: the grey
    # intensity in every channel).  albedo / emission are then unused.
    albedo_rgb: Optional[np.ndarray] = None
    emission_rgb: Optional[np.ndarray] = None
    pl_rgb: Optional[np.ndarray] = None

    @property
    def n_tri_world(self) -> int:
        per_mesh = np.diff(self.mesh_tri_off.astype(np.int64))
        return int(per_mesh[self.inst_mesh.astype(np.int64)].sum()) if len(self.inst_mesh) else 0

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


class SceneBuilder:
    """Accumulates meshes, instances, materials and the camera."""

    def __init__(self) -> None:
        self.albedo: List[float] = []
        self.emission: List[float] = []
        self.verts: List[np.ndarray] = []
        self.tris: List[np.ndarray] = []
        self.mats: List[np.ndarray] = []
        self.mesh_off = [0]
        self.n_vert = 0
        self.inst_mesh: List[int] = []
        self.inst_keys: List[tuple] = []
        self.pl_pos: List[Sequence[float]] = []
        self.pl_int: List[float] = []
        self.camera = None

    def material(self, albedo: float, emission: float = 0.0) -> int:
        self.albedo.append(float(albedo))
        self.emission.append(float(emission))
        return len(self.albedo) - 1

    def mesh(self, verts: np.ndarray, tris: np.ndarray, mat) -> int:
        verts = np.asarray(verts, dtype=np.float32).reshape(-1, 3)
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        mats = np.broadcast_to(np.asarray(mat, dtype=np.uint32), (len(tris),)).copy()
        self.verts.append(verts)
        self.tris.append((tris + self.n_vert).astype(np.uint32))
        self.mats.append(mats)
        self.n_vert += len(verts)
        self.mesh_off.append(self.mesh_off[-1] + len(tris))
        return len(self.mesh_off) - 2

    def instance(self, mesh_id: int, key_t: Sequence[float], xforms: Sequence[np.ndarray]) -> int:
        kt = np.asarray(key_t, dtype=np.float64).reshape(-1)
        kx = np.asarray(xforms, dtype=np.float64).reshape(-1, 3, 4)
        assert len(kt) == len(kx) and len(kt) >= 1
        assert np.all(np.diff(kt) > 0)
        self.inst_mesh.append(mesh_id)
        self.inst_keys.append((kt, kx))
        return len(self.inst_mesh) - 1

    def static(self, mesh_id: int) -> int:
        return self.instance(mesh_id, [0.0], [identity()])

    def point_light(self, pos, intensity: float) -> None:
        self.pl_pos.append(list(pos))
        self.pl_int.append(float(intensity))

    def set_camera(self, width: int, height: int, vfov_deg: float, key_t, eye_look_up) -> None:
        kt = np.asarray(key_t, dtype=np.float64).reshape(-1)
        elu = np.asarray(eye_look_up, dtype=np.float64).reshape(-1, 9)
        assert len(kt) == len(elu)
        self.camera = (int(width), int(height), float(vfov_deg), kt, elu)

    def build(self) -> Scene:
        assert self.camera is not None
        key_t = [k[0] for k in self.inst_keys]
        key_x = [k[1] for k in self.inst_keys]
        off = np.zeros(len(self.inst_keys) + 1, dtype=np.uint32)
        off[1:] = np.cumsum([len(k) for k in key_t])
        w, h, fov, ct, celu = self.camera
        return Scene(
            albedo=np.asarray(self.albedo, dtype=np.float32),
            emission=np.asarray(self.emission, dtype=np.float32),
            xyz=np.concatenate(self.verts).astype(np.float32) if self.verts else np.zeros((0, 3), np.float32),
            tri_idx=np.concatenate(self.tris) if self.tris else np.zeros((0, 3), np.uint32),
            tri_mat=np.concatenate(self.mats) if self.mats else np.zeros((0,), np.uint32),
            mesh_tri_off=np.asarray(self.mesh_off, dtype=np.uint32),
            inst_mesh=np.asarray(self.inst_mesh, dtype=np.uint32),
            inst_key_off=off,
            key_t=np.concatenate(key_t) if key_t else np.zeros((0,), np.float64),
            key_xform=np.concatenate(key_x) if key_x else np.zeros((0, 3, 4), np.float64),
            pl_pos=np.asarray(self.pl_pos, dtype=np.float32).reshape(-1, 3),
            pl_intensity=np.asarray(self.pl_int, dtype=np.float32),
            width=w, height=h, vfov_deg=fov, cam_t=ct, cam_elu=celu,
        )


# ---------------------------------------------------------------------------
# Small geometry helpers (input construction only).

def identity() -> np.ndarray:
    return np.hstack([np.eye(3), np.zeros((3, 1))])


def translation(v) -> np.ndarray:
    m = identity()
    m[:, 3] = np.asarray(v, dtype=np.float64)
    return m


def rotation_axis_angle(axis, angle_rad: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle_rad) * k + (1 - math.cos(angle_rad)) * (k @ k)


def compose(r3: np.ndarray, t, scale: float = 1.0) -> np.ndarray:
    """3x4 matrix x -> R (scale * x) + t."""
    m = np.zeros((3, 4))
    m[:, :3] = r3 * scale
    m[:, 3] = np.asarray(t, dtype=np.float64)
    return m


def oriented_quad(corners, normal):
    """Two triangles over 4 corners (in perimeter order), wound so that
    cross(v1 - v0, v2 - v0) points along ``normal``."""
    c = np.asarray(corners, dtype=np.float64)
    tris = np.array([[0, 1, 2], [0, 2, 3]])
    n = np.cross(c[1] - c[0], c[2] - c[0])
    if np.dot(n, np.asarray(normal, dtype=np.float64)) < 0:
        tris = tris[:, ::-1]
    return c.astype(np.float32), tris


def box_mesh(lo, hi, outward: bool = True, faces=("-x", "+x", "-y", "+y", "-z", "+z")):
    """Axis-aligned box faces (two triangles each), normals outward or inward."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    verts, tris = [], []
    for f in faces:
        ax = "xyz".index(f[1])
        sgn = 1.0 if f[0] == "+" else -1.0
        u, v = [a for a in range(3) if a != ax]
        val = hi[ax] if sgn > 0 else lo[ax]
        cs = []
        for (a, b) in ((lo[u], lo[v]), (hi[u], lo[v]), (hi[u], hi[v]), (lo[u], hi[v])):
            p = np.zeros(3)
            p[ax] = val
            p[u] = a
            p[v] = b
            cs.append(p)
        nrm = np.zeros(3)
        nrm[ax] = sgn if outward else -sgn
        c, t = oriented_quad(cs, nrm)
        tris.append(t + 4 * len(verts))
        verts.append(c)
    return np.concatenate(verts), np.concatenate(tris)


def icosphere(subdiv: int):
    """Unit icosphere: an icosahedron with each face split in four
    ``subdiv`` times, new vertices projected to the sphere; outward winding."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts)
    F = np.array(faces, dtype=np.int64)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", n, V[F].mean(axis=1)) < 0
    F[flip] = F[flip][:, ::-1]
    return V.astype(np.float32), F


# ---------------------------------------------------------------------------
# Benchmark scenes.

def tiny_box(seed: int = 0, width: int = 64, height: int = 64) -> Scene:
    """64x64 open box: floor, ceiling, back, left and right faces (10 inward
    triangles; albedo U[0.2, 0.8] per face, in that order, seed 0), a 0.5 x 0.5
    ceiling light at y = 1.98 facing down (Le = 10, albedo 0), and a 0.5-unit
    cube centred at (-0.2, 0.25, -0.2) that moves by +0.05 along x between
    t = 0 and t = 1.  Pinhole camera at (0, 1, 3.4) looking at (0, 1, 0),
    40 degree vertical field of view."""
    rng = np.random.default_rng(seed)
    draws = rng.uniform(0.2, 0.8, size=6)
    b = SceneBuilder()
    face_specs = [("-y", (0, 1, 0)), ("+y", (0, -1, 0)), ("-z", (0, 0, 1)),
                  ("-x", (1, 0, 0)), ("+x", (-1, 0, 0))]
    for k, (face, _) in enumerate(face_specs):
        m = b.material(draws[k])
        v, t = box_mesh((-1, 0, -1), (1, 2, 1), outward=False, faces=(face,))
        b.static(b.mesh(v, t, m))
    light = b.material(0.0, 10.0)
    lv, lt = oriented_quad([(-0.25, 1.98, -0.25), (0.25, 1.98, -0.25), (0.25, 1.98, 0.25),
                            (-0.25, 1.98, 0.25)], (0, -1, 0))
    b.static(b.mesh(lv, lt, light))
    cube_m = b.material(draws[5])
    cv, ct = box_mesh((-0.25, -0.25, -0.25), (0.25, 0.25, 0.25), outward=True)
    cube = b.mesh(cv, ct, cube_m)
    c0 = np.array([-0.2, 0.25, -0.2])
    b.instance(cube, [0.0, 1.0], [translation(c0), translation(c0 + [0.05, 0, 0])])
    b.set_camera(width, height, 40.0, [0.0], [[0, 1, 3.4, 0, 1, 0, 0, 1, 0]])
    return b.build()


def heightfield_y(x, z, phi1: float, phi2: float):
    return 0.05 * np.sin(1.7 * x + phi1) * np.cos(2.3 * z + phi2)


def sensor(seed: int = 0, width: int = 640, height: int = 480, n_spheres: int = 20,
           grid: int = 190, subdiv: int = 3, n_moving: Optional[int] = None,
           sky: Optional[float] = None) -> Scene:
    """640x480: a 190x190-quad displaced floor on [-4, 4]^2 (72,200 triangles,
    h = 0.05 sin(1.7x + phi1) cos(2.3z + phi2)), 20 icospheres (subdivision 3,
    1,280 triangles each) of radius U[0.1, 0.5] resting on the floor at
    centres U[-3, 3]^2, albedo U[0.1, 0.9] per object, three 1x1 area lights
    at y = 4 facing down (Le = 10).  Between t = 0 and t = 1 every sphere
    moves rigidly by a translation U[-0.02, 0.02]^3 and a rotation of U[0, 2]
    degrees about a random axis through its centre.  Static camera at
    (0, 2.5, 7) looking at (0, 0.3, 0), 40 degree vertical field of view.
    Variants: only the first n_moving spheres move (the others keep their
    t = 0 placement; the random draws are the same), and a uniform grey sky
    of radiance `sky` (an environment map) lights the scene besides the
    three lights."""
    rng = np.random.default_rng(seed)
    phi1, phi2 = rng.uniform(0, 2 * math.pi, size=2)
    b = SceneBuilder()
    floor_m = b.material(rng.uniform(0.1, 0.9))
    g = grid
    xs = np.linspace(-4.0, 4.0, g + 1)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    Y = heightfield_y(X, Z, phi1, phi2)
    fv = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    i = np.arange(g)[:, None]
    j = np.arange(g)[None, :]
    v00 = (i * (g + 1) + j).reshape(-1)
    v10 = ((i + 1) * (g + 1) + j).reshape(-1)
    v01 = (i * (g + 1) + j + 1).reshape(-1)
    v11 = ((i + 1) * (g + 1) + j + 1).reshape(-1)
    ft = np.stack([np.stack([v00, v01, v11], 1), np.stack([v00, v11, v10], 1)], 1).reshape(-1, 3)
    b.static(b.mesh(fv, ft, floor_m))
    sv, st = icosphere(subdiv)
    for k in range(n_spheres):
        m = b.material(rng.uniform(0.1, 0.9))
        mesh = b.mesh(sv, st, m)
        r = rng.uniform(0.1, 0.5)
        cx, cz = rng.uniform(-3.0, 3.0, size=2)
        c = np.array([cx, float(heightfield_y(cx, cz, phi1, phi2)) + r, cz])
        dt = rng.uniform(-0.02, 0.02, size=3)
        axis = rng.normal(size=3)
        ang = math.radians(rng.uniform(0.0, 2.0))
        rot = rotation_axis_angle(axis, ang)
        if n_moving is None or k < n_moving:
            b.instance(mesh, [0.0, 1.0], [compose(np.eye(3), c, r), compose(rot, c + dt, r)])
        else:
            b.instance(mesh, [0.0], [compose(np.eye(3), c, r)])
    light_m = b.material(0.0, 10.0)
    for (lx, lz) in ((-2.0, -1.0), (0.0, 1.0), (2.0, -0.5)):
        lv, lt = oriented_quad([(lx - 0.5, 4.0, lz - 0.5), (lx + 0.5, 4.0, lz - 0.5),
                                (lx + 0.5, 4.0, lz + 0.5), (lx - 0.5, 4.0, lz + 0.5)], (0, -1, 0))
        b.static(b.mesh(lv, lt, light_m))
    b.set_camera(width, height, 40.0, [0.0], [[0, 2.5, 7.0, 0, 0.3, 0, 0, 1, 0]])
    sc = b.build()
    if sky is not None:
        sc.env = np.full((6, 8, 8), sky, np.float32)
    return sc


def diff_scene(seed: int = 0, width: int = 256, height: int = 256, floor_n: int = 50,
               n_spheres: int = 12, subdiv: int = 2) -> Scene:
    """Workload of the event-loss gradient (256x256, 9,648 triangles, 32
    Lambertian materials of albedo U[0.2, 0.8] and 4 emitters of radiance
    U[1, 20]): a floor_n x floor_n-quad floor on [-3, 3]^2 in 4x4 tiles of 16
    materials, a 20x20-quad back wall at z = -3 in 2x2 tiles of 4 materials,
    12 icospheres (subdivision 2, 320 triangles) of radius U[0.2, 0.5] and
    one material each resting on the floor at centres U[-2.2, 2.2]^2, and
    four 0.8 x 0.8 lights at y = 3 facing down, one material each.  Every
    sphere translates by U[-0.05, 0.05]^3 between t = 0 and t = 1.  Static
    camera at (0, 2.2, 5.5) looking at (0, 0.4, 0), 45 degrees."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    floor_m = [b.material(rng.uniform(0.2, 0.8)) for _ in range(16)]
    wall_m = [b.material(rng.uniform(0.2, 0.8)) for _ in range(4)]
    sphere_m = [b.material(rng.uniform(0.2, 0.8)) for _ in range(n_spheres)]
    light_m = [b.material(0.0, rng.uniform(1.0, 20.0)) for _ in range(4)]

    def grid(n, corner, du, dv, tile_mats, tiles):
        u = np.arange(n + 1)
        U, V = np.meshgrid(u, u, indexing="ij")
        P = (np.asarray(corner)[None, None, :] + U[..., None] * np.asarray(du)[None, None, :] / n
             + V[..., None] * np.asarray(dv)[None, None, :] / n).reshape(-1, 3)
        i = np.arange(n)[:, None]
        j = np.arange(n)[None, :]
        v00 = (i * (n + 1) + j).reshape(-1)
        v10 = ((i + 1) * (n + 1) + j).reshape(-1)
        v01 = (i * (n + 1) + j + 1).reshape(-1)
        v11 = ((i + 1) * (n + 1) + j + 1).reshape(-1)
        tr = np.stack([np.stack([v00, v01, v11], 1), np.stack([v00, v11, v10], 1)], 1).reshape(-1, 3)
        ti = (i * tiles // n) * tiles + (j * tiles // n)
        mats = np.repeat(np.asarray(tile_mats)[ti.reshape(-1)], 2)
        return P, tr, mats

    # Floor facing +y (corner, du along +z, dv along +x), wall facing +z.
    fv, ft, fm = grid(floor_n, (-3.0, 0.0, -3.0), (0.0, 0.0, 6.0), (6.0, 0.0, 0.0), floor_m, 4)
    b.static(b.mesh(fv, ft, fm))
    wv, wt, wm = grid(20, (-3.0, 0.0, -3.0), (6.0, 0.0, 0.0), (0.0, 3.5, 0.0), wall_m, 2)
    b.static(b.mesh(wv, wt, wm))
    sv, st = icosphere(subdiv)
    for k in range(n_spheres):
        mesh = b.mesh(sv, st, sphere_m[k])
        r = rng.uniform(0.2, 0.5)
        cx, cz = rng.uniform(-2.2, 2.2, size=2)
        c = np.array([cx, r, cz])
        dt = rng.uniform(-0.05, 0.05, size=3)
        b.instance(mesh, [0.0, 1.0], [compose(np.eye(3), c, r), compose(np.eye(3), c + dt, r)])
    for k, (lx, lz) in enumerate(((-1.2, -1.0), (1.2, -1.0), (-1.2, 1.0), (1.2, 1.0))):
        lv, lt = oriented_quad([(lx - 0.4, 3.0, lz - 0.4), (lx + 0.4, 3.0, lz - 0.4),
                                (lx + 0.4, 3.0, lz + 0.4), (lx - 0.4, 3.0, lz + 0.4)], (0, -1, 0))
        b.static(b.mesh(lv, lt, light_m[k]))
    b.set_camera(width, height, 45.0, [0.0], [[0, 2.2, 5.5, 0, 0.4, 0, 0, 1, 0]])
    return b.build()


def _pan_keys(eye, look, up, n_frames: int, deg_per_frame: float):
    """Camera keys at t = 0, 1, ..., n_frames - 1: the view direction turns
    about the vertical axis through the eye by deg_per_frame per frame."""
    eye = np.asarray(eye, np.float64)
    d0 = np.asarray(look, np.float64) - eye
    keys = []
    for k in range(n_frames):
        a = math.radians(deg_per_frame * k)
        c, s_ = math.cos(a), math.sin(a)
        d = np.array([c * d0[0] + s_ * d0[2], d0[1], -s_ * d0[0] + c * d0[2]])
        keys.append(list(eye) + list(eye + d) + list(up))
    return np.arange(n_frames, dtype=np.float64), np.asarray(keys, np.float64)


def panning(sc: Scene, n_frames: int, deg_per_frame: float) -> Scene:
    """The scene with every instance frozen at its first key and the camera
    turning by deg_per_frame per frame at t = 0, 1, ..., n_frames - 1."""
    import dataclasses
    koff = sc.inst_key_off.astype(np.int64)
    key_t = np.zeros(len(sc.inst_mesh), np.float64)
    key_x = np.stack([sc.key_xform[koff[i]] for i in range(len(sc.inst_mesh))]) if len(sc.inst_mesh) else \
        np.zeros((0, 3, 4))
    e = sc.cam_elu[0]
    ct, ce = _pan_keys(e[0:3], e[3:6], e[6:9], n_frames, deg_per_frame)
    return dataclasses.replace(sc, key_t=key_t, key_xform=key_x,
                               inst_key_off=np.arange(len(sc.inst_mesh) + 1, dtype=np.uint32),
                               cam_t=ct, cam_elu=ce)


def moving_panning(width: int = 32, height: int = 24, n_frames: int = 5, deg_per_frame: float = 2.0,
                   step: float = 0.05) -> Scene:
    """The tiny box with its cube moving by `step` in x per frame and the
    camera turning by deg_per_frame per frame, both keyed at t = 0, 1, ...,
    n_frames - 1 (geometry and camera change every frame)."""
    import dataclasses
    sc = tiny_box(width=width, height=height)
    koff = sc.inst_key_off.astype(np.int64)
    cube = len(sc.inst_mesh) - 1
    key_t, key_x = [], []
    for i in range(len(sc.inst_mesh)):
        if i == cube:
            c0 = sc.key_xform[koff[i]][:, 3].copy()
            key_t += [0.0, float(n_frames - 1)]
            key_x += [translation(c0), translation(c0 + [step * (n_frames - 1), 0, 0])]
        else:
            key_t.append(0.0)
            key_x.append(sc.key_xform[koff[i]])
    off = np.concatenate([[0], np.cumsum([2 if i == cube else 1 for i in range(len(sc.inst_mesh))])])
    e = sc.cam_elu[0]
    ct, ce = _pan_keys(e[0:3], e[3:6], e[6:9], n_frames, deg_per_frame)
    return dataclasses.replace(sc, key_t=np.asarray(key_t, np.float64), key_xform=np.asarray(key_x, np.float64),
                               inst_key_off=off.astype(np.uint32), cam_t=ct, cam_elu=ce)


def tessellated_box(n: int = 3):
    """Unit box [0, 1]^3 with every face cut into n x n quads (12 n^2
    triangles), faces wound outward."""
    verts, tris = [], []
    u = np.linspace(0.0, 1.0, n + 1)
    faces = [((0, 1, 2), 0.0, -1), ((0, 1, 2), 1.0, 1), ((1, 2, 0), 0.0, -1), ((1, 2, 0), 1.0, 1),
             ((2, 0, 1), 0.0, -1), ((2, 0, 1), 1.0, 1)]
    for (a, b, c), cval, sgn in faces:
        base = len(verts)
        for i in range(n + 1):
            for j in range(n + 1):
                p = [0.0, 0.0, 0.0]
                p[a], p[b], p[c] = u[i], u[j], cval
                verts.append(p)
        for i in range(n):
            for j in range(n):
                v00 = base + i * (n + 1) + j
                v10, v01, v11 = v00 + n + 1, v00 + 1, v00 + n + 2
                for t in ((v00, v10, v11), (v00, v11, v01)):
                    P = np.array([verts[k] for k in t])
                    nrm = np.cross(P[1] - P[0], P[2] - P[0])
                    want = np.zeros(3)
                    want[c] = sgn
                    tris.append(t if nrm @ want > 0 else (t[0], t[2], t[1]))
    return np.asarray(verts, np.float32), np.asarray(tris, np.int64)


def city(seed: int = 0, width: int = 1920, height: int = 1080, grid: int = 200, n_frames: int = 121,
         n_moving: int = 50, n_lights: int = 16) -> Scene:
    """Stress workload (about 4.3M triangles): a grid x grid city of boxes
    (footprint 0.6, pitch 1.0, height U[0.3, 4.0]) whose faces are cut 3 x 3
    (108 triangles a box), 16 box materials of albedo U[0.1, 0.9], a ground
    plane, n_lights 2 x 2 area lights at y = 12 (Le = 25) facing down,
    n_moving boxes that each move by U[-0.03, 0.03] in x and z per frame,
    and a camera flying over the city (eye from (-20, 9, 40) toward
    (-20, 9, 28), looking 20 units ahead and 8 down), keyed at t = 0, 1,
    ..., n_frames - 1; 50 degrees."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    ground_m = b.material(0.4)
    gv, gt = oriented_quad([(-110, 0, -110), (110, 0, -110), (110, 0, 110), (-110, 0, 110)], (0, 1, 0))
    b.static(b.mesh(gv, gt, ground_m))
    bv, bt = tessellated_box(3)
    box_meshes = [b.mesh(bv, bt, b.material(rng.uniform(0.1, 0.9))) for _ in range(16)]
    off = (grid - 1) / 2.0
    heights = rng.uniform(0.3, 4.0, size=(grid, grid))
    mesh_pick = rng.integers(0, 16, size=(grid, grid))
    moving = set(map(int, rng.choice(grid * grid, size=n_moving, replace=False)))
    last = float(n_frames - 1)
    for i in range(grid):
        for j in range(grid):
            x, z = i - off - 0.3, j - off - 0.3
            m = compose(np.diag([0.6, heights[i, j], 0.6]), (x, 0.0, z))
            if i * grid + j in moving:
                v = rng.uniform(-0.03, 0.03, size=2)
                m1 = m.copy()
                m1[0, 3] += v[0] * last
                m1[2, 3] += v[1] * last
                b.instance(box_meshes[mesh_pick[i, j]], [0.0, last], [m, m1])
            else:
                b.instance(box_meshes[mesh_pick[i, j]], [0.0], [m])
    lm = b.material(0.0, 25.0)
    for k in range(n_lights):
        lx, lz = rng.uniform(-60, 60, size=2)
        lv, lt = oriented_quad([(lx - 1, 12.0, lz - 1), (lx + 1, 12.0, lz - 1), (lx + 1, 12.0, lz + 1),
                                (lx - 1, 12.0, lz + 1)], (0, -1, 0))
        b.static(b.mesh(lv, lt, lm))
    kt = np.arange(n_frames, dtype=np.float64)
    keys = []
    for k in range(n_frames):
        ez = 40.0 - 12.0 * k / max(1, n_frames - 1)
        keys.append([-20.0, 9.0, ez, -20.0, 1.0, ez - 20.0, 0.0, 1.0, 0.0])
    b.set_camera(width, height, 50.0, kt, keys)
    return b.build()


# Stress workload: 120 pairs of the city, depth 12, schedule 64/64/4096,
# C = 0.2, alpha = 0.001.
CITY_PARAMS = dict(seed=0, max_depth=12, rr_start_depth=2, minibatch=4, log_eps=1e-4, nee=1, jitter=1,
                   spp_init=64, spp_batch=64, spp_max=4096, C=0.2, alpha=0.001)


def batch_scene(seed: int = 0, width: int = 1280, height: int = 720, grid: int = 24, n_cubes: int = 20000,
                subdiv: int = 3, n_frames: int = 65, deg_per_frame: float = 0.5) -> Scene:
    """Frame-batch workload (1280x720, 977,290 triangles): a 40 x 40 ground
    quad, a grid x grid lattice of icospheres (subdivision 3, 1,280
    triangles, radius U[0.25, 0.45]) on a 1.2-unit pitch, n_cubes small
    cubes (12 triangles, edge U[0.1, 0.3], random yaw) scattered over
    [-16, 16]^2, 16 Lambertian materials of albedo U[0.1, 0.9], four 2 x 2
    lights at y = 8 (Le = 15).  All geometry static; the camera at
    (0, 4, 18) looking at (0, 0.5, 0) turns by deg_per_frame per frame about
    the vertical axis, keyed at t = 0 ... n_frames - 1; 45 degrees."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    mats = [b.material(rng.uniform(0.1, 0.9)) for _ in range(16)]
    gv, gt = oriented_quad([(-20, 0, -20), (20, 0, -20), (20, 0, 20), (-20, 0, 20)], (0, 1, 0))
    b.static(b.mesh(gv, gt, mats[0]))
    sv, st = icosphere(subdiv)
    sphere_meshes = [b.mesh(sv, st, m) for m in mats[1:9]]
    off = (grid - 1) * 1.2 / 2.0
    for i in range(grid):
        for j in range(grid):
            r = rng.uniform(0.25, 0.45)
            c = np.array([i * 1.2 - off, r, j * 1.2 - off])
            b.instance(sphere_meshes[int(rng.integers(0, 8))], [0.0], [compose(np.eye(3), c, r)])
    cv, ct = box_mesh((-0.5, 0.0, -0.5), (0.5, 1.0, 0.5))
    cube_meshes = [b.mesh(cv, ct, m) for m in mats[9:16]]
    for _ in range(n_cubes):
        e = rng.uniform(0.1, 0.3)
        x, z = rng.uniform(-16.0, 16.0, size=2)
        rot = rotation_axis_angle((0, 1, 0), rng.uniform(0.0, 2 * math.pi))
        b.instance(cube_meshes[int(rng.integers(0, 7))], [0.0], [compose(rot, (x, 0.0, z), e)])
    light_m = b.material(0.0, 15.0)
    for (lx, lz) in ((-6.0, -4.0), (6.0, -4.0), (-6.0, 6.0), (6.0, 6.0)):
        lv, lt = oriented_quad([(lx - 1, 8.0, lz - 1), (lx + 1, 8.0, lz - 1), (lx + 1, 8.0, lz + 1),
                                (lx - 1, 8.0, lz + 1)], (0, -1, 0))
        b.static(b.mesh(lv, lt, light_m))
    ct_, ce = _pan_keys((0.0, 4.0, 18.0), (0.0, 0.5, 0.0), (0, 1, 0), n_frames, deg_per_frame)
    b.set_camera(width, height, 45.0, list(ct_), [list(r) for r in ce])
    return b.build()


def sky_cube_map(res: int = 32, sun_dir=(0.5, 0.6, -0.62), sun_radiance: float = 60.0,
                 sky: float = 1.2, ground: float = 0.25) -> np.ndarray:
    """Grey cube map [6, res, res] (faces +x, -x, +y, -y, +z, -z; row j,
    column i) of a sky: brighter toward the zenith, a dim ground below the
    horizon and a small bright sun, evaluated at texel centres."""
    sc = 2.0 * (np.arange(res) + 0.5) / res - 1.0
    tc = sc[:, None]
    s_ = sc[None, :]
    one = np.ones((res, res))
    dirs = [np.stack([one, -tc * one, -s_ * one], -1), np.stack([-one, -tc * one, s_ * one], -1),
            np.stack([s_ * one, one, tc * one], -1), np.stack([s_ * one, -one, -tc * one], -1),
            np.stack([s_ * one, -tc * one, one], -1), np.stack([-s_ * one, -tc * one, -one], -1)]
    d = np.stack(dirs)
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    up = d[..., 1]
    env = np.where(up > 0, sky * (0.4 + 0.6 * up), ground)
    sd = np.asarray(sun_dir, np.float64)
    sd = sd / np.linalg.norm(sd)
    env = np.where(d @ sd > 0.995, sun_radiance, env)
    return env.astype(np.float32)


def lens_env(seed: int = 0, width: int = 96, height: int = 64, lens_radius: float = 0.08,
             focus_dist: float = 5.0) -> Scene:
    """The setting of the paper's failure case (Sec. 5): a background given
    by an environment map (the sky cube map above), static boxes at several
    depths whose contours stand against it, one sphere that moves by 0.1 in
    x between t = 0 and t = 1 at the distance in focus, a floor, a small
    area light, and a thin-lens camera (aperture radius lens_radius, focus
    at focus_dist) at (0, 1.2, 5) looking at (0, 0.8, 0), 50 degrees."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    floor_m = b.material(0.5)
    v, t = oriented_quad([(-6, 0, -6), (6, 0, -6), (6, 0, 6), (-6, 0, 6)], (0, 1, 0))
    b.static(b.mesh(v, t, floor_m))
    cv, ct = box_mesh((-0.5, 0.0, -0.5), (0.5, 1.0, 0.5))
    for (x, z, hgt) in ((-1.6, 2.0, 1.4), (1.3, -1.0, 2.0), (-0.6, -3.0, 2.6), (2.4, 1.5, 0.9)):
        m = b.material(rng.uniform(0.2, 0.8))
        b.instance(b.mesh(cv, ct, m), [0.0], [compose(np.diag([0.7, hgt, 0.7]), (x, 0.0, z))])
    sv, st = icosphere(3)
    sm = b.material(0.7)
    b.instance(b.mesh(sv, st, sm), [0.0, 1.0], [compose(np.eye(3), (-0.2, 0.45, 0.0), 0.45),
                                                compose(np.eye(3), (-0.1, 0.45, 0.0), 0.45)])
    lm = b.material(0.0, 8.0)
    lv, lt = oriented_quad([(-0.4, 3.5, -0.4), (0.4, 3.5, -0.4), (0.4, 3.5, 0.4), (-0.4, 3.5, 0.4)], (0, -1, 0))
    b.static(b.mesh(lv, lt, lm))
    b.set_camera(width, height, 50.0, [0.0], [[0.0, 1.2, 5.0, 0.0, 0.8, 0.0, 0, 1, 0]])
    sc = b.build()
    sc.env = sky_cube_map()
    sc.lens_radius = float(lens_radius)
    sc.focus_dist = float(focus_dist)
    return sc


# Frame-batch workload: 64 pairs, schedule 16/16/2048, depth 8.
BATCH_PARAMS = dict(seed=0, max_depth=8, rr_start_depth=2, minibatch=4, log_eps=1e-4, nee=1, jitter=1,
                    spp_init=16, spp_batch=16, spp_max=2048, C=0.2, alpha=0.01)


# Event loss of the differentiation workload: 256 paths per pixel and
# instant, loss sum softplus((|Delta| - C) / tau).
DIFF_PARAMS = dict(seed=0, max_depth=4, rr_start_depth=2, minibatch=4, log_eps=1e-4, nee=1, jitter=1,
                   C=0.2, tau=0.05, spp=256)


# ---------------------------------------------------------------------------
# Closed-form and structural test scenes.

def furnace(albedo: float, emission: float, width: int = 16, height: int = 16) -> Scene:
    """Closed cube [-1, 1]^3 of inward triangles that all have the same albedo
    and emission, camera inside at the centre."""
    b = SceneBuilder()
    m = b.material(albedo, emission)
    v, t = box_mesh((-1, -1, -1), (1, 1, 1), outward=False)
    b.static(b.mesh(v, t, m))
    b.set_camera(width, height, 60.0, [0.0], [[0.0, 0.0, 0.0, 0.3, 0.1, -1.0, 0, 1, 0]])
    return b.build()


def plane_point_light(albedo: float = 0.7, intensity: float = 5.0, h: float = 1.5,
                      width: int = 24, height: int = 16) -> Scene:
    """Plane y = 0 (two triangles, 100 units wide) under a point light at
    (0.3, h, -0.2); the camera at (0, 2, 3) looks at the origin."""
    b = SceneBuilder()
    m = b.material(albedo)
    v, t = oriented_quad([(-50, 0, -50), (50, 0, -50), (50, 0, 50), (-50, 0, 50)], (0, 1, 0))
    b.static(b.mesh(v, t, m))
    b.point_light((0.3, h, -0.2), intensity)
    b.set_camera(width, height, 50.0, [0.0], [[0.0, 2.0, 3.0, 0, 0, 0, 0, 1, 0]])
    return b.build()


def single_triangle(albedo: float = 0.6, intensity: float = 4.0, width: int = 12,
                    height: int = 10) -> Scene:
    """One triangle in the plane y = 0 (the whole scene is a single leaf)
    under a point light at (0.2, 1.2, 0.1); the camera at (0, 2, 2.5)."""
    b = SceneBuilder()
    m = b.material(albedo)
    tri = np.array([[-1.5, 0.0, -1.0], [0.0, 0.0, 1.5], [1.5, 0.0, -1.0]], dtype=np.float32)
    b.static(b.mesh(tri, np.array([[0, 1, 2]]), m))
    b.point_light((0.2, 1.2, 0.1), intensity)
    b.set_camera(width, height, 60.0, [0.0], [[0.0, 2.0, 2.5, 0, 0, 0, 0, 1, 0]])
    return b.build()


def plane_area_light(albedo: float = 0.6, emission: float = 4.0, width: int = 8,
                     height: int = 8) -> Scene:
    """Plane y = 0 under one triangular emitter at y = 1 facing down."""
    b = SceneBuilder()
    m = b.material(albedo)
    v, t = oriented_quad([(-50, 0, -50), (50, 0, -50), (50, 0, 50), (-50, 0, 50)], (0, 1, 0))
    b.static(b.mesh(v, t, m))
    lm = b.material(0.0, emission)
    tri = np.array([[-0.4, 1.0, -0.3], [0.5, 1.0, -0.2], [0.0, 1.0, 0.6]], dtype=np.float64)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    if n[1] > 0:
        tri = tri[[0, 2, 1]]
    b.static(b.mesh(tri.astype(np.float32), np.array([[0, 1, 2]]), lm))
    b.set_camera(width, height, 30.0, [0.0], [[0.0, 2.5, 2.5, 0, 0, 0, 0, 1, 0]])
    return b.build()


def triangle_soup(n_tri: int, seed: int = 0, extent: float = 2.0, size: float = 0.4,
                  width: int = 32, height: int = 32, moving: bool = False,
                  emitters: int = 0) -> Scene:
    """Random triangles in [-extent, extent]^3 (plus some coplanar pairs that
    share an edge), optionally with a moving half and a few emitters."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    mats = [b.material(rng.uniform(0.1, 0.9)) for _ in range(4)]
    emit_m = b.material(0.0, 5.0) if emitters else None
    cen = rng.uniform(-extent, extent, size=(n_tri, 1, 3))
    tri = cen + rng.uniform(-size, size, size=(n_tri, 3, 3))
    half = n_tri // 2
    tm = rng.integers(0, 4, size=n_tri)
    if emitters:
        tm[:emitters] = -1
    mat_ids = np.array([emit_m if x < 0 else mats[x] for x in tm], dtype=np.uint32)
    idx = np.arange(3 * n_tri).reshape(-1, 3)
    s = b.mesh(tri[:half].reshape(-1, 3), idx[:half], mat_ids[:half])
    d = b.mesh(tri[half:].reshape(-1, 3), idx[half:] - 3 * half, mat_ids[half:])
    b.static(s)
    if moving:
        rot = rotation_axis_angle(rng.normal(size=3), math.radians(3.0))
        b.instance(d, [0.0, 1.0], [identity(), compose(rot, (0.05, -0.03, 0.02))])
    else:
        b.static(d)
    b.set_camera(width, height, 45.0, [0.0], [[0.0, 0.0, 6.0, 0, 0, 0, 0, 1, 0]])
    return b.build()


def colorize(sc: Scene, seed: int = 0, spread: float = 0.5) -> Scene:
    """The same scene with RGB radiance: each material's albedo and emission
    scaled per channel by factors in [1 - spread, 1 + spread] (albedo
    clamped below 1), each point light's intensity likewise."""
    rng = np.random.default_rng(seed)
    n = len(sc.albedo)
    fa = rng.uniform(1.0 - spread, 1.0 + spread, size=(n, 3))
    fe = rng.uniform(1.0 - spread, 1.0 + spread, size=(n, 3))
    out = dataclasses.replace(sc)
    out.albedo_rgb = np.minimum(np.asarray(sc.albedo, np.float64)[:, None] * fa, 0.99).astype(np.float32)
    out.emission_rgb = (np.asarray(sc.emission, np.float64)[:, None] * fe).astype(np.float32)
    if len(sc.pl_intensity):
        fl = rng.uniform(1.0 - spread, 1.0 + spread, size=(len(sc.pl_intensity), 3))
        out.pl_rgb = (np.asarray(sc.pl_intensity, np.float64)[:, None] * fl).astype(np.float32)
    return out


def empty(width: int = 8, height: int = 8) -> Scene:
    """No geometry at all: every path escapes."""
    b = SceneBuilder()
    b.material(0.5)
    b.set_camera(width, height, 40.0, [0.0], [[0, 0, 5, 0, 0, 0, 0, 1, 0]])
    return b.build()


# ---------------------------------------------------------------------------
# Render parameter presets for the two plain-method workloads.

TINY_PARAMS = dict(seed=0, spp_init=16, spp_batch=16, spp_max=256, max_depth=4,
                   rr_start_depth=2, minibatch=4, log_eps=1e-4, C=0.2, alpha=0.01,
                   nee=1, jitter=1, mode=0, df_mode=0, ref_mode=0)

SENSOR_PARAMS = dict(seed=0, spp_init=64, spp_batch=16, spp_max=1024, max_depth=8,
                     rr_start_depth=2, minibatch=4, log_eps=1e-4, C=0.15, alpha=0.01,
                     nee=1, jitter=1, mode=0, df_mode=0, ref_mode=0)


def subset_every(width: int, height: int, step: int = 8) -> np.ndarray:
    """Pixel indices of every ``step``-th pixel in x and y (row-major)."""
    ys = np.arange(0, height, step)
    xs = np.arange(0, width, step)
    return (ys[:, None] * width + xs[None, :]).reshape(-1).astype(np.uint32)
