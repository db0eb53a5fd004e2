"""Closed, outward-oriented flat-triangle surface meshes.

Vertices are float64 (M, 3); triangles are int32 (E, 3), counter-clockwise when seen
from outside, so the right-hand normal points out of the enclosed volume.
"""
import numpy as np


def _orient_outward(xyz, tri, centre_of):
    """Flip every triangle whose right-hand normal points towards centre_of(centroid)."""
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    c = (p0 + p1 + p2) / 3.0
    out = c - centre_of(c)
    flip = np.einsum("ij,ij->i", nrm, out) < 0
    tri = tri.copy()
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def icosphere(level):
    """Unit sphere: regular icosahedron, `level` times 4-way midpoint subdivision with
    projection of the new vertices onto the sphere.  level 2 -> 320/162, level 4 -> 5120/2562."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    # faces: triples of mutually adjacent vertices (edge length 2 before normalisation)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    e = d.min(where=d > 1e-9, initial=10.0)
    adj = np.abs(d - e) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    tri = np.array(faces, dtype=np.int64)
    xyz = v
    for _ in range(level):
        mid = {}
        pts = list(xyz)
        newtri = []

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = 0.5 * (pts[a] + pts[b])
                m = m / np.linalg.norm(m)
                mid[key] = len(pts)
                pts.append(m)
            return mid[key]

        for a, b, c in tri:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            newtri += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        xyz = np.array(pts)
        tri = np.array(newtri, dtype=np.int64)
    tri = _orient_outward(xyz, tri, lambda c: np.zeros_like(c))
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32)


def geodesic_sphere(nu):
    """Unit sphere, class I geodesic of frequency nu: every face of the regular icosahedron split
    into nu^2 triangles on its barycentric grid, vertices projected onto the sphere (20 nu^2
    triangles, 10 nu^2 + 2 vertices).  nu = 4 gives the 320 triangles of icosphere(2)."""
    ico, faces = icosphere(0)
    pts, index = [], {}

    def vertex(key, p):
        if key not in index:
            index[key] = len(pts)
            pts.append(p / np.linalg.norm(p))
        return index[key]

    tri = []
    for f in faces:
        A, B, C = ico[f[0]], ico[f[1]], ico[f[2]]
        ids = {}
        for a in range(nu + 1):
            for b in range(nu + 1 - a):
                c = nu - a - b
                # a grid point on a shared edge or corner gets the same key from both faces
                w = {int(f[0]): a, int(f[1]): b, int(f[2]): c}
                key = tuple(sorted((v, x) for v, x in w.items() if x > 0))
                ids[(a, b)] = vertex(key, (a * A + b * B + c * C) / nu)
        for a in range(nu):
            for b in range(nu - a):
                tri.append((ids[(a, b)], ids[(a + 1, b)], ids[(a, b + 1)]))
                if a + b + 1 < nu:
                    tri.append((ids[(a + 1, b)], ids[(a + 1, b + 1)], ids[(a, b + 1)]))
    xyz = np.array(pts)
    tri = _orient_outward(xyz, np.array(tri, dtype=np.int64), lambda c: np.zeros_like(c))
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32)


def torus(nu, nv, R=1.0, r=0.35):
    """Structured torus: nu x nv quads on the (u, v) parameter grid, each quad
    (i,j),(i+1,j),(i+1,j+1),(i,j+1) split along the (i,j)-(i+1,j+1) diagonal."""
    i = np.arange(nu)
    j = np.arange(nv)
    U, V = np.meshgrid(2 * np.pi * i / nu, 2 * np.pi * j / nv, indexing="ij")
    xyz = np.stack([(R + r * np.cos(V)) * np.cos(U), (R + r * np.cos(V)) * np.sin(U), r * np.sin(V)], -1)
    xyz = xyz.reshape(-1, 3)
    idx = lambda a, b: (a % nu) * nv + (b % nv)
    tri = []
    for a in range(nu):
        for b in range(nv):
            p, q, s, t = idx(a, b), idx(a + 1, b), idx(a + 1, b + 1), idx(a, b + 1)
            tri += [(p, q, s), (p, s, t)]
    tri = np.array(tri, dtype=np.int64)

    def tube_centre(c):
        ang = np.arctan2(c[:, 1], c[:, 0])
        return np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros_like(ang)], -1)

    tri = _orient_outward(xyz, tri, tube_centre)
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32)


def mesh_diameter(xyz):
    """Largest vertex-to-vertex distance (equals the diameter of a flat-triangle mesh)."""
    from scipy.spatial.distance import pdist
    return float(pdist(xyz).max())
