"""Triangle meshes for the mixed mesh + Gaussian workloads: a subdivided plane,
an icosphere and a box (outward winding: e1 x e2 points out of closed
shapes). Pure geometry generation (float32 vertices, int32 indices)."""

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    verts: np.ndarray   # [V, 3] float32
    tris: np.ndarray    # [T, 3] int32
    mirror: np.ndarray  # [T] int32 material code: 0 diffuse, 1 mirror, 2 glass

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


def subdivided_plane(cells, half, z=0.0):
    xs = np.linspace(-half, half, cells + 1)
    X, Y = np.meshgrid(xs, xs)
    verts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)
    tris = []
    for j in range(cells):
        for i in range(cells):
            a = j * (cells + 1) + i
            b = a + 1
            c = a + (cells + 1)
            d = c + 1
            tris.append((a, b, d))
            tris.append((a, d, c))
    return verts, np.asarray(tris, dtype=np.int64)


def icosphere(subdiv, radius, centre):
    t = (1.0 + np.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    verts = np.asarray(verts) * radius + np.asarray(centre, np.float64)
    return verts, np.asarray(faces, dtype=np.int64)


def mirror_mesh(plane_cells=50, plane_half=3.0, sphere_subdiv=4, sphere_radius=0.6,
                sphere_centre=(0.0, 0.0, 0.8)):
    """Mirror plane (2*cells^2 triangles at z = 0) plus a diffuse icosphere."""
    pv, pt = subdivided_plane(plane_cells, plane_half)
    sv, st = icosphere(sphere_subdiv, sphere_radius, sphere_centre)
    verts = np.concatenate([pv, sv])
    tris = np.concatenate([pt, st + pv.shape[0]])
    mirror = np.concatenate([np.ones(len(pt), np.int32), np.zeros(len(st), np.int32)])
    return Mesh(np.ascontiguousarray(verts.astype(np.float32)), np.ascontiguousarray(tris.astype(np.int32)),
                np.ascontiguousarray(mirror))


def box(lo, hi):
    """Axis-aligned box as 12 triangles, normals pointing out."""
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    c = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], np.float64)
    verts = lo + c * (hi - lo)
    # quads (a, b, c, d) counter-clockwise seen from outside
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    tris = []
    for a, b, cc, d in quads:
        tris += [(a, b, cc), (a, cc, d)]
    return verts, np.asarray(tris, dtype=np.int64)


def glass_mesh(plane_cells=50, plane_half=3.0, sphere_subdiv=4, sphere_radius=0.6, sphere_centre=(0.0, 0.0, 0.8),
               box_lo=(0.9, -1.6, 0.05), box_hi=(1.7, -0.8, 0.85)):
    """Mirror plane at z = 0, a glass icosphere and a glass box."""
    pv, pt = subdivided_plane(plane_cells, plane_half)
    sv, st = icosphere(sphere_subdiv, sphere_radius, sphere_centre)
    bv, bt = box(box_lo, box_hi)
    verts = np.concatenate([pv, sv, bv])
    tris = np.concatenate([pt, st + len(pv), bt + len(pv) + len(sv)])
    mat = np.concatenate([np.ones(len(pt), np.int32), np.full(len(st), 2, np.int32), np.full(len(bt), 2, np.int32)])
    return Mesh(np.ascontiguousarray(verts.astype(np.float32)), np.ascontiguousarray(tris.astype(np.int32)),
                np.ascontiguousarray(mat))
