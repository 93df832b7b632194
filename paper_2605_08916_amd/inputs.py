"""Seeded synthetic inputs: procedural scenes, chain states, per-chain sigma.

This module generates inputs only.  It holds none of the method's arithmetic
(no path sampling, no chain dynamics) and is the one module both the HIP
library's callers and the CPU oracle's callers take their inputs from.

A scene is a dict of numpy arrays:
  vertices     (V, 3) float32
  indices      (T, 3) uint32
  tri_material (T,)   uint32
  materials    (M, 12) float32: kind (0 Lambertian, 1 GGX conductor,
               2 smooth conductor, 3 smooth dielectric), albedo[3],
               roughness (GGX alpha), f0[3], Le[3], eta (dielectric index
               of refraction on the side opposite e1 x e2)
  lights       (NL, 12) float32: parallelogram p0[3], e1[3], e2[3], Le[3];
               it emits on the side of e1 x e2 and also appears in the mesh
               as two triangles wound the same way with an emissive material
  camera       (10,) float32: eye[3], at[3], up[3], vertical fov in degrees
  width, height, name

The paper evaluates on dataset scenes that are not available here; these
procedural scenes stand in for them at the paper's working scale (one chain
per pixel).
"""
from __future__ import annotations

import math

import numpy as np

KIND_LAMBERT, KIND_GGX, KIND_MIRROR, KIND_GLASS = 0, 1, 2, 3


def material(kind=KIND_LAMBERT, albedo=(0.5, 0.5, 0.5), rough=0.0, f0=(0.0, 0.0, 0.0), Le=(0.0, 0.0, 0.0),
             eta=1.5):
    return [float(kind), *map(float, albedo), float(rough), *map(float, f0), *map(float, Le), float(eta)]


class _Builder:
    def __init__(self):
        self.V: list[np.ndarray] = []
        self.I: list[np.ndarray] = []
        self.TM: list[np.ndarray] = []
        self.mats: list[list[float]] = []
        self.lights: list[list[float]] = []
        self.nv = 0

    def add_material(self, m) -> int:
        self.mats.append(m)
        return len(self.mats) - 1

    def add_mesh(self, V, I, mat):
        V = np.asarray(V, np.float64).reshape(-1, 3)
        I = np.asarray(I, np.int64).reshape(-1, 3)
        self.V.append(V)
        self.I.append(I + self.nv)
        self.TM.append(np.broadcast_to(np.asarray(mat, np.int64), (I.shape[0],)).copy())
        self.nv += V.shape[0]

    def add_quad(self, p0, e1, e2, mat):
        p0, e1, e2 = (np.asarray(a, np.float64) for a in (p0, e1, e2))
        V = np.stack([p0, p0 + e1, p0 + e1 + e2, p0 + e2])
        self.add_mesh(V, [[0, 1, 2], [0, 2, 3]], mat)

    def add_light(self, p0, e1, e2, Le, albedo=(0.0, 0.0, 0.0)):
        # store the light in float32 first so that mesh and light agree exactly
        p0, e1, e2 = (np.asarray(a, np.float32).astype(np.float64) for a in (p0, e1, e2))
        m = self.add_material(material(KIND_LAMBERT, albedo=albedo, Le=Le))
        self.add_quad(p0, e1, e2, m)
        self.lights.append([*p0, *e1, *e2, *map(float, Le)])

    def finish(self, camera, width, height, name) -> dict:
        return dict(
            vertices=np.concatenate(self.V).astype(np.float32),
            indices=np.concatenate(self.I).astype(np.uint32),
            tri_material=np.concatenate(self.TM).astype(np.uint32),
            materials=np.asarray(self.mats, np.float32),
            lights=np.asarray(self.lights, np.float32).reshape(-1, 12),
            camera=np.asarray(camera, np.float32),
            width=int(width), height=int(height), name=name,
        )


def _box_faces(center, size, angle_deg):
    """Top and four sides of a y-rotated axis-aligned box (no bottom)."""
    cx, cy, cz = center
    sx, sy, sz = (s / 2 for s in size)
    a = math.radians(angle_deg)
    ca, sa = math.cos(a), math.sin(a)

    def P(x, y, z):
        return np.array([cx + ca * x + sa * z, cy + y, cz - sa * x + ca * z])

    c = {k: P(*k) for k in [(i * sx, j * sy, k * sz) for i in (-1, 1) for j in (-1, 1) for k in (-1, 1)]}
    faces = [
        (c[(-sx, sy, -sz)], c[(sx, sy, -sz)], c[(sx, sy, sz)], c[(-sx, sy, sz)]),      # top
        (c[(-sx, -sy, sz)], c[(sx, -sy, sz)], c[(sx, sy, sz)], c[(-sx, sy, sz)]),      # +z
        (c[(sx, -sy, -sz)], c[(-sx, -sy, -sz)], c[(-sx, sy, -sz)], c[(sx, sy, -sz)]),  # -z
        (c[(sx, -sy, sz)], c[(sx, -sy, -sz)], c[(sx, sy, -sz)], c[(sx, sy, sz)]),      # +x
        (c[(-sx, -sy, -sz)], c[(-sx, -sy, sz)], c[(-sx, sy, sz)], c[(-sx, sy, -sz)]),  # -x
    ]
    return faces


def cornell_tiny(seed: int = 1, width: int = 64, height: int = 64) -> dict:
    """32-triangle Cornell-style box built procedurally: 5 wall quads, one
    ceiling quad light, two 5-face boxes; Lambertian albedo per face, each
    channel U[0.3, 0.8]; light radiance 15."""
    rng = np.random.default_rng(seed)
    B = _Builder()

    def lam():
        return B.add_material(material(KIND_LAMBERT, albedo=rng.uniform(0.3, 0.8, 3)))

    B.add_quad([0, 0, 0], [1, 0, 0], [0, 0, 1], lam())     # floor
    B.add_quad([0, 1, 0], [0, 0, 1], [1, 0, 0], lam())     # ceiling
    B.add_quad([0, 0, 0], [0, 1, 0], [1, 0, 0], lam())     # back wall
    B.add_quad([0, 0, 0], [0, 0, 1], [0, 1, 0], lam())     # left wall
    B.add_quad([1, 0, 0], [0, 1, 0], [0, 0, 1], lam())     # right wall
    for center, size, ang in [((0.32, 0.15, 0.62), (0.3, 0.3, 0.3), -17.0),
                              ((0.67, 0.30, 0.36), (0.28, 0.6, 0.28), 16.0)]:
        for q in _box_faces(center, size, ang):
            m = lam()
            B.add_mesh(np.stack(q), [[0, 1, 2], [0, 2, 3]], m)
    # ceiling light: emits downward (e1 x e2 = -y)
    B.add_light([0.4, 0.999, 0.4], [0.2, 0, 0], [0, 0, 0.2], (15.0, 15.0, 15.0))
    cam = [0.5, 0.5, 2.2, 0.5, 0.5, 0.0, 0.0, 1.0, 0.0, 40.0]
    sc = B.finish(cam, width, height, "cornell_tiny")
    assert sc["indices"].shape[0] == 32
    return sc


def specular_box(seed: int = 2, width: int = 64, height: int = 64, subdiv: int = 2) -> dict:
    """Cornell-style box with the delta materials: a smooth-dielectric
    icosphere (eta 1.5, outward winding), a tall box of smooth conductor
    (f0 per channel U[0.6, 0.95]) and a smooth-conductor back wall panel, so
    that paths run through glass (caustics on the floor, total internal
    reflection) and chains of mirror bounces.  Walls Lambertian, albedo per
    channel U[0.3, 0.8]; ceiling light of radiance 15."""
    rng = np.random.default_rng(seed)
    B = _Builder()

    def lam():
        return B.add_material(material(KIND_LAMBERT, albedo=rng.uniform(0.3, 0.8, 3)))

    B.add_quad([0, 0, 0], [1, 0, 0], [0, 0, 1], lam())     # floor
    B.add_quad([0, 1, 0], [0, 0, 1], [1, 0, 0], lam())     # ceiling
    B.add_quad([0, 0, 0], [0, 1, 0], [1, 0, 0], lam())     # back wall
    B.add_quad([0, 0, 0], [0, 0, 1], [0, 1, 0], lam())     # left wall
    B.add_quad([1, 0, 0], [0, 1, 0], [0, 0, 1], lam())     # right wall
    mirror = B.add_material(material(KIND_MIRROR, f0=rng.uniform(0.6, 0.95, 3)))
    B.add_quad([0.55, 0.1, 0.001], [0, 0.6, 0], [0.35, 0, 0], mirror)   # panel on the back wall, facing +z
    metal = B.add_material(material(KIND_MIRROR, f0=rng.uniform(0.6, 0.95, 3)))
    for q in _box_faces((0.72, 0.25, 0.35), (0.2, 0.5, 0.2), 20.0):
        B.add_mesh(np.stack(q), [[0, 1, 2], [0, 2, 3]], metal)
    glass = B.add_material(material(KIND_GLASS, eta=1.5))
    V, F = icosphere(subdiv)
    B.add_mesh(V * 0.17 + np.array([0.33, 0.17, 0.6]), F, glass)
    B.add_light([0.4, 0.999, 0.4], [0.2, 0, 0], [0, 0, 0.2], (15.0, 15.0, 15.0))
    cam = [0.5, 0.5, 2.2, 0.5, 0.5, 0.0, 0.0, 1.0, 0.0, 40.0]
    return B.finish(cam, width, height, "specular_box")


def mirror_plane(f0=(0.9, 0.6, 0.3), Le=(4.0, 3.0, 2.0), width: int = 16, height: int = 16) -> dict:
    """A smooth-conductor square in the plane z = -1 (side 4, centred) facing
    +z; a quad light in the plane z = 1 facing -z (towards the mirror); the
    camera at the origin looking down -z.  The light is seen only through the
    mirror (used to pin the delta lobes)."""
    B = _Builder()
    m = B.add_material(material(KIND_MIRROR, f0=f0))
    B.add_quad([-2, -2, -1], [4, 0, 0], [0, 4, 0], m)               # e1 x e2 = +z
    B.add_light([-0.3, -0.2, 1.0], [0, 0.5, 0], [0.7, 0, 0], Le)    # e1 x e2 = -z
    cam = [0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0.0, 1.0, 0.0, 60.0]
    return B.finish(cam, width, height, "mirror_plane")


def glass_slab(eta: float = 1.5, Le=(4.0, 3.0, 2.0), thickness: float = 0.5, width: int = 16,
               height: int = 16, eye_z: float = 0.0) -> dict:
    """A closed smooth-dielectric slab between the planes z = -1 and
    z = -1 - thickness (side 4, outward winding: two faces and four thin
    sides), a quad light in the plane z = -3 facing +z, the camera at
    (0, 0, eye_z) looking down -z (above the slab by default; inside it for
    eye_z in (-1 - thickness, -1)).  Rays reach the light only through the
    slab's lower face."""
    B = _Builder()
    g = B.add_material(material(KIND_GLASS, eta=eta))
    z0, z1, h = -1.0, -1.0 - thickness, 2.0
    B.add_quad([-h, -h, z0], [2 * h, 0, 0], [0, 2 * h, 0], g)             # top face, normal +z
    B.add_quad([-h, -h, z1], [0, 2 * h, 0], [2 * h, 0, 0], g)             # bottom face, normal -z
    B.add_quad([-h, -h, z1], [2 * h, 0, 0], [0, 0, thickness], g)         # y = -h, normal -y
    B.add_quad([-h, h, z1], [0, 0, thickness], [2 * h, 0, 0], g)          # y = +h, normal +y
    B.add_quad([-h, -h, z1], [0, 0, thickness], [0, 2 * h, 0], g)         # x = -h, normal -x
    B.add_quad([h, -h, z1], [0, 2 * h, 0], [0, 0, thickness], g)          # x = +h, normal +x
    B.add_light([-1.5, -1.5, -3.0], [3.0, 0, 0], [0, 3.0, 0], Le)         # e1 x e2 = +z
    cam = [0.0, 0.0, eye_z, 0.0, 0.0, eye_z - 1.0, 0.0, 1.0, 0.0, 60.0]
    return B.finish(cam, width, height, "glass_slab")


def white_furnace(albedo: float = 0.5, Le: float = 1.0, width: int = 8, height: int = 8) -> dict:
    """Closed cube whose six faces are inward-emitting quad lights with a
    Lambertian albedo; the camera sits inside.  Every pixel's expected value is
    Le (1 - a^L) / (1 - a) for path length L."""
    B = _Builder()
    s = 2.0
    # (p0, e1, e2) with e1 x e2 pointing into the cube
    faces = [
        ([-1, -1, -1], [0, 0, s], [s, 0, 0]),   # y = -1, normal +y
        ([-1, 1, -1], [s, 0, 0], [0, 0, s]),    # y = +1, normal -y
        ([-1, -1, -1], [s, 0, 0], [0, s, 0]),   # z = -1, normal +z
        ([-1, -1, 1], [0, s, 0], [s, 0, 0]),    # z = +1, normal -z
        ([-1, -1, -1], [0, s, 0], [0, 0, s]),   # x = -1, normal +x
        ([1, -1, -1], [0, 0, s], [0, s, 0]),    # x = +1, normal -x
    ]
    for p0, e1, e2 in faces:
        B.add_light(p0, e1, e2, (Le, Le, Le), albedo=(albedo, albedo, albedo))
    cam = [0.1, 0.2, 0.3, 0.1, 0.2, -1.0, 0.0, 1.0, 0.0, 60.0]
    return B.finish(cam, width, height, "white_furnace")


def one_bounce_plane(albedo=(0.6, 0.5, 0.4), Le=(4.0, 3.0, 2.0), width: int = 16, height: int = 16) -> dict:
    """Lambertian square z = 0 (side 4, centred), one downward quad light at
    z = 1.5, camera above looking down.  With path length 2 the contribution
    has a closed form (used to pin f and its gradient)."""
    B = _Builder()
    m = B.add_material(material(KIND_LAMBERT, albedo=albedo))
    B.add_quad([-2, -2, 0], [4, 0, 0], [0, 4, 0], m)
    B.add_light([-0.25, -0.5, 1.5], [0, 0.6, 0], [0.8, 0, 0], Le)   # e1 x e2 = -z
    cam = [0.3, -0.2, 3.0, 0.1, 0.05, 0.0, 0.0, 1.0, 0.0, 35.0]
    return B.finish(cam, width, height, "one_bounce_plane")


# ---------------------------------------------------------------------------
# Procedural meshes
# ---------------------------------------------------------------------------
def icosphere(subdiv: int):
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, np.float64) / np.linalg.norm(v) for v in V]
    for _ in range(subdiv):
        cache: dict = {}

        def mid(a, b):
            k = (a, b) if a < b else (b, a)
            if k not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[k] = len(V) - 1
            return cache[k]

        nF = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nF += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nF
    return np.array(V), np.array(F, np.int64)


def _value_noise(P, rng_seed: int, res: int = 16):
    """Trilinear value noise with smoothstep on a seeded periodic lattice."""
    lat = np.random.default_rng(rng_seed).uniform(-1, 1, (res, res, res))
    q = P * res
    i0 = np.floor(q).astype(np.int64)
    f = q - i0
    f = f * f * (3 - 2 * f)
    out = 0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                w = (f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) * (f[:, 2] if dz else 1 - f[:, 2])
                out = out + w * lat[(i0[:, 0] + dx) % res, (i0[:, 1] + dy) % res, (i0[:, 2] + dz) % res]
    return out


def displaced(V, seed: int, amp: float = 0.15, octaves: int = 4):
    """Radial displacement 1 + amp * fbm(value noise) of unit-sphere vertices."""
    fbm = 0
    for o in range(octaves):
        fbm = fbm + 0.5 ** o * _value_noise((V * 0.5 + 0.5) * 2 ** o * 0.5, seed * 131 + o)
    return V * (1.0 + amp * fbm)[:, None]


def _rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _plane(B, size, n, z0, mat):
    xs = np.linspace(-size, size, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    V = np.stack([X.ravel(), np.full(X.size, z0), Y.ravel()], 1)
    I = []
    for i in range(n):
        for j in range(n):
            a = i * (n + 1) + j
            b, c, d = a + (n + 1), a + (n + 1) + 1, a + 1
            I += [(a, b, c), (a, c, d)]
    B.add_mesh(V, I, mat)


def procedural_spheres(seed: int = 1, width: int = 512, height: int = 512, n_spheres: int = 10, subdiv: int = 4,
                       specular: bool = False) -> dict:
    """Noise-displaced icospheres (subdivision 4, 5,120 triangles each) on a
    tessellated ground plane; GGX conductors with roughness U[0.1, 0.5] and F0
    U[0.5, 0.95] per object; Lambertian 0.5 ground; two quad lights, each
    partly occluded by a seeded blocker quad.  About 53k triangles.  With
    `specular`, every third sphere (k = 1 mod 3) is a smooth dielectric
    (eta 1.5) and the next (k = 2 mod 3) a smooth conductor with the drawn
    F0; the seeded draws, hence the geometry, are those of the default."""
    rng = np.random.default_rng(seed)
    B = _Builder()
    Vs, Fs = icosphere(subdiv)
    ground = B.add_material(material(KIND_LAMBERT, albedo=(0.5, 0.5, 0.5)))
    _plane(B, 6.0, 32, 0.0, ground)
    placed = []
    for k in range(n_spheres):
        for _ in range(100):
            r = rng.uniform(0.45, 0.9)
            c = np.array([rng.uniform(-3.5, 3.5), r * 1.05, rng.uniform(-3.5, 3.5)])
            if all(np.linalg.norm(c[[0, 2]] - q[[0, 2]]) > (r + rq) * 1.2 for q, rq in placed):
                break
        placed.append((c, r))
        rough, f0 = rng.uniform(0.1, 0.5), rng.uniform(0.5, 0.95, 3)
        if specular and k % 3 == 1:
            m = B.add_material(material(KIND_GLASS, eta=1.5))
        elif specular and k % 3 == 2:
            m = B.add_material(material(KIND_MIRROR, f0=f0))
        else:
            m = B.add_material(material(KIND_GGX, rough=rough, f0=f0))
        V = displaced(Vs, seed * 1000 + k) @ _rot(rng).T * r + c
        B.add_mesh(V, Fs, m)
    blocker = B.add_material(material(KIND_LAMBERT, albedo=(0.3, 0.3, 0.3)))
    for lc in ([-2.0, 5.0, -1.0], [2.5, 4.5, 1.5]):
        lc = np.array(lc)
        # light facing down: e1 x e2 = -y
        B.add_light(lc - [0.75, 0, 0.75], [1.5, 0, 0], [0, 0, 1.5], (12.0, 11.0, 10.0))
        off = rng.uniform(-0.4, 0.4, 2)
        B.add_quad(lc + [off[0] - 0.5, -0.6, off[1] - 0.5], [1.0, 0, 0], [0, 0, 1.0], blocker)
    cam = [0.0, 4.5, 8.5, 0.0, 0.6, 0.0, 0.0, 1.0, 0.0, 45.0]
    return B.finish(cam, width, height, "procedural_spheres")


def procedural_instances(seed: int = 3, width: int = 1280, height: int = 720, n_inst: int = 200,
                         subdiv: int = 4) -> dict:
    """About 1M triangles: n_inst instances (random rotation, scale and
    position) of 5 displaced icosphere meshes, flattened to world space, over a
    ground plane, open to the sky (paths end by escaping), two quad lights."""
    rng = np.random.default_rng(seed)
    B = _Builder()
    Vs, Fs = icosphere(subdiv)
    protos = [displaced(Vs, seed * 77 + k, amp=0.25) for k in range(5)]
    ground = B.add_material(material(KIND_LAMBERT, albedo=(0.45, 0.45, 0.45)))
    _plane(B, 20.0, 16, 0.0, ground)
    mats = [B.add_material(material(KIND_GGX, rough=rng.uniform(0.1, 0.5), f0=rng.uniform(0.5, 0.95, 3)))
            for _ in range(3)]
    mats += [B.add_material(material(KIND_LAMBERT, albedo=rng.uniform(0.3, 0.8, 3))) for _ in range(3)]
    for k in range(n_inst):
        s = rng.uniform(0.3, 1.0)
        c = np.array([rng.uniform(-15, 15), s * rng.uniform(0.8, 3.0), rng.uniform(-15, 15)])
        V = protos[k % 5] @ _rot(rng).T * s + c
        B.add_mesh(V, Fs, mats[k % len(mats)])
    B.add_light([-6, 12, -6], [4, 0, 0], [0, 0, 4], (20.0, 19.0, 17.0))
    B.add_light([5, 9, 3], [3, 0, 0], [0, 0, 3], (12.0, 14.0, 18.0))
    cam = [0.0, 9.0, 24.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 50.0]
    return B.finish(cam, width, height, "procedural_instances")


def procedural_interior(seed: int = 5, width: int = 1920, height: int = 1080, n_inst: int = 400,
                        subdiv: int = 4) -> dict:
    """About 2M triangles: a closed room with instanced displaced
    furniture-like meshes, two ceiling quad lights and one partly occluded
    light."""
    rng = np.random.default_rng(seed)
    B = _Builder()
    Vs, Fs = icosphere(subdiv)
    protos = [displaced(Vs, seed * 91 + k, amp=0.2) * np.array([1.6, 0.6, 1.0]) for k in range(5)]
    wall = B.add_material(material(KIND_LAMBERT, albedo=(0.7, 0.68, 0.65)))
    floor = B.add_material(material(KIND_LAMBERT, albedo=(0.4, 0.35, 0.3)))
    X, Y, Z = 10.0, 4.0, 8.0
    B.add_quad([-X, 0, -Z], [2 * X, 0, 0], [0, 0, 2 * Z], floor)
    B.add_quad([-X, Y, -Z], [0, 0, 2 * Z], [2 * X, 0, 0], wall)
    B.add_quad([-X, 0, -Z], [0, Y, 0], [2 * X, 0, 0], wall)
    B.add_quad([-X, 0, Z], [2 * X, 0, 0], [0, Y, 0], wall)
    B.add_quad([-X, 0, -Z], [0, 0, 2 * Z], [0, Y, 0], wall)
    B.add_quad([X, 0, -Z], [0, Y, 0], [0, 0, 2 * Z], wall)
    mats = [B.add_material(material(KIND_GGX, rough=rng.uniform(0.1, 0.5), f0=rng.uniform(0.5, 0.95, 3)))
            for _ in range(3)]
    mats += [B.add_material(material(KIND_LAMBERT, albedo=rng.uniform(0.3, 0.8, 3))) for _ in range(4)]
    for k in range(n_inst):
        s = rng.uniform(0.15, 0.45)
        c = np.array([rng.uniform(-X + 1, X - 1), rng.uniform(0.2, Y - 1.0), rng.uniform(-Z + 1, Z - 1)])
        V = protos[k % 5] @ _rot(rng).T * s + c
        B.add_mesh(V, Fs, mats[k % len(mats)])
    B.add_light([-5, Y - 0.01, -1.5], [3, 0, 0], [0, 0, 3], (14.0, 13.0, 12.0))
    B.add_light([3, Y - 0.01, -2.0], [3, 0, 0], [0, 0, 3], (14.0, 13.0, 12.0))
    B.add_light([7.5, 2.5, 6.0], [1.2, 0, 0], [0, -1.2, 0], (25.0, 20.0, 15.0))   # faces -z
    blocker = B.add_material(material(KIND_LAMBERT, albedo=(0.2, 0.2, 0.2)))
    B.add_quad([7.3, 1.1, 5.5], [0.9, 0, 0], [0, 0.9, 0], blocker)
    cam = [-7.0, 2.2, 6.5, 2.0, 1.2, -2.0, 0.0, 1.0, 0.0, 60.0]
    return B.finish(cam, width, height, "procedural_interior")


def camera_path(sc: dict, frame: int, n_frames: int = 60) -> np.ndarray:
    """Camera of frame `frame` on a constant-speed arc through the room."""
    a = 2 * math.pi * 0.25 * frame / max(n_frames, 1)
    eye = np.array([-7.0 + 3.0 * math.sin(a), 2.2, 6.5 - 2.0 * (1 - math.cos(a))])
    at = np.array([2.0, 1.2, -2.0])
    return np.array([*eye, *at, 0.0, 1.0, 0.0, float(sc["camera"][9])], np.float32)


# ---------------------------------------------------------------------------
# Chain states and per-chain diffusion scales
# ---------------------------------------------------------------------------
def random_state(d: int, n: int, seed: int, killed_frac: float = 0.1, score_scale: float = 30.0) -> dict:
    """A seeded chain state: x ~ U[0,1)^d (24-bit, so exact in FP32), scores
    ~ N(0, score_scale^2), a fraction of chains flagged killed.  Planar d x n."""
    rng = np.random.default_rng(seed)
    x = (rng.integers(0, 1 << 24, (d, n)) / float(1 << 24)).astype(np.float32)
    score = (rng.normal(size=(d, n)) * score_scale).astype(np.float32)
    killed = (rng.uniform(size=n) < killed_frac).astype(np.uint32)
    return dict(x=x, score=score, killed=killed)


def random_points(d: int, n: int, seed: int) -> np.ndarray:
    """n points on the torus (n x d), 24-bit grid so they are exact in FP32."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 1 << 24, (n, d)) / float(1 << 24)).astype(np.float32)


def per_chain_sigma(d: int, n: int, seed: int, stddev: float = 5e-3) -> np.ndarray:
    """Per-chain diagonal step scale stddev * 2^U[-1,1] (d x n, float32)."""
    rng = np.random.default_rng(seed)
    return (stddev * 2.0 ** rng.uniform(-1, 1, (d, n))).astype(np.float32)


def mixture_target(d: int = 8, seed: int = 11):
    """Wrapped Gaussian mixture on T^d: 4 modes, weights 0.4/0.3/0.2/0.1, std
    0.03 or 0.05, means at least 0.3 apart on the torus (seeded)."""
    rng = np.random.default_rng(seed)
    means = []
    while len(means) < 4:
        m = rng.uniform(0, 1, d)
        ok = True
        for q in means:
            dd = np.abs(m - q)
            dd = np.minimum(dd, 1 - dd)
            if np.linalg.norm(dd) < 0.3:
                ok = False
        if ok:
            means.append(m)
    return dict(weights=np.array([0.4, 0.3, 0.2, 0.1]), means=np.array(means), stds=np.array([0.03, 0.05, 0.03, 0.05]))


CONFIGS = {
    # name: (scene factory, path length L, chains)
    "tiny": (cornell_tiny, 4, 256),
    "spheres": (procedural_spheres, 8, 65536),
    "instances": (procedural_instances, 12, 1 << 20),
    "spheres_1080p_L16": (lambda seed=1: procedural_spheres(seed, 1920, 1080), 16, 1 << 21),
    "spheres_specular": (lambda seed=1: procedural_spheres(seed, specular=True), 8, 65536),
    "interior": (procedural_interior, 8, 1 << 22),
}
