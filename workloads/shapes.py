"""Surface meshes and quadrature points for the synthetic workloads.

Geometry only: vertices, triangle centroids, outward normals and areas. The
paper's electrostatic example puts one quadrature point at each element
centroid, weighted by the element area, with the exact spherical area on
spheres (Sec. III); these helpers produce exactly those inputs. Its
magnetostatic example also integrates with a fifth-order rule on each
triangle, so that sources far outnumber the mesh nodes (Sec. IV.A):
triangle_rule_deg5 and mesh_quadrature.
"""

from __future__ import annotations

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
], dtype=np.float64)
_ICO_V /= np.linalg.norm(_ICO_V, axis=1, keepdims=True)
_ICO_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
], dtype=np.int64)


def _face_grid(freq):
    """Barycentric integer grid of one icosahedron face and its freq^2 triangles."""
    ij = [(i, j) for i in range(freq + 1) for j in range(freq + 1 - i)]
    index = {t: n for n, t in enumerate(ij)}
    tris = []
    for i in range(freq):
        for j in range(freq - i):
            tris.append((index[(i, j)], index[(i + 1, j)], index[(i, j + 1)]))
            if i + j <= freq - 2:
                tris.append((index[(i + 1, j)], index[(i + 1, j + 1)], index[(i, j + 1)]))
    return np.array(ij, dtype=np.int64), np.array(tris, dtype=np.int64)


def icosphere(freq):
    """Class-I geodesic icosphere of frequency `freq` on the unit sphere.

    Returns (vertices [V,3], triangles [20*freq^2, 3]) with shared vertices
    de-duplicated (V = 10*freq^2 + 2) and triangles oriented outward.
    """
    ij, tris = _face_grid(freq)
    key_to_vid = {}
    verts = []
    faces = []
    for f in _ICO_F:
        a, b, c = f
        local = np.empty(len(ij), dtype=np.int64)
        for n, (i, j) in enumerate(ij):
            k = freq - i - j
            key = tuple(sorted(t for t in ((a, i), (b, j), (c, k)) if t[1] > 0))
            vid = key_to_vid.get(key)
            if vid is None:
                vid = len(verts)
                key_to_vid[key] = vid
                verts.append((i * _ICO_V[a] + j * _ICO_V[b] + k * _ICO_V[c]) / freq)
            local[n] = vid
        faces.append(local[tris])
    v = np.array(verts)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t = np.concatenate(faces)
    # orient outward: (b-a) x (c-a) must point away from the origin
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    t[flip] = t[flip][:, [0, 2, 1]]
    return v, t


def spherical_triangle_area(a, b, c):
    """Exact area of unit-sphere triangles (rows of a, b, c are unit vectors).

    Uses tan(E/2) = |a.(b x c)| / (1 + a.b + b.c + c.a) (Van Oosterom-Strackee).
    """
    num = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c)))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def sphere_quadrature(freq, centre, radius):
    """Centroid quadrature on an icosphere of radius `radius` at `centre`.

    Point = normalised triangle centroid (on the sphere), normal = the same
    unit vector, weight = exact spherical-triangle area * radius^2.
    """
    v, t = icosphere(freq)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    n = a + b + c
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    w = spherical_triangle_area(a, b, c) * radius * radius
    return np.asarray(centre) + radius * n, n, w


def triangle_rule_deg5():
    """Radon's seven-point rule on a triangle, exact for polynomials of degree 5.

    Returns (bary [7, 3], weights [7]) with the weights summing to 1 (multiply
    by the triangle's area): the centroid and two orbits of three points
    (a, a, 1 - 2a) with a = (6 -+ sqrt(15)) / 21. Stroud's T2:5-1; the paper's
    magnetostatic example integrates with a fifth-order rule (Sec. IV.A).
    """
    s15 = np.sqrt(15.0)
    bary = [[1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0]]
    weights = [9.0 / 40.0]
    for a, wa in (((6.0 - s15) / 21.0, (155.0 - s15) / 1200.0), ((6.0 + s15) / 21.0, (155.0 + s15) / 1200.0)):
        b = 1.0 - 2.0 * a
        bary += [[a, a, b], [a, b, a], [b, a, a]]
        weights += [wa] * 3
    return np.array(bary), np.array(weights)


def mesh_quadrature(verts, tris, bary, weights):
    """Quadrature points of a rule on every flat triangle of a mesh.

    Returns (points [T*Q, 3], normals [T*Q, 3], weights [T*Q]), triangle-major:
    point q of triangle t is sum_k bary[q, k] verts[tris[t, k]], its normal the
    triangle's unit normal (orientation of tris) and its weight
    weights[q] * area(t). A field linear on each triangle with vertex values f
    is, at the points, (f[tris] @ bary.T).reshape(-1).
    """
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    pts = np.einsum("qk,tkc->tqc", bary, np.stack([a, b, c], axis=1)).reshape(-1, 3)
    nq = len(weights)
    return pts, np.repeat(nrm, nq, axis=0), (area[:, None] * weights[None, :]).reshape(-1)


def cube_surface(side, n_nodes_target):
    """Structured triangulation of a cube surface centred at the origin.

    k nodes per edge with 6(k-1)^2+2 ~= n_nodes_target unique nodes; every
    grid square is split into two triangles. Returns (nodes, centroids,
    normals, areas, solid_angle_at_nodes). The interior solid angle is 2*pi
    on faces, pi on edges and pi/2 at corners.
    """
    k = max(2, int(round(((n_nodes_target - 2) / 6.0) ** 0.5)) + 1)
    h = side / (k - 1)
    g = np.arange(k)
    # unique nodes: integer grid points with at least one coordinate on the boundary
    ii, jj, kk = np.meshgrid(g, g, g, indexing="ij")
    on = (ii == 0) | (ii == k - 1) | (jj == 0) | (jj == k - 1) | (kk == 0) | (kk == k - 1)
    idx = np.stack([ii[on], jj[on], kk[on]], axis=1)
    nodes = idx * h - side / 2.0
    nb = ((idx == 0) | (idx == k - 1)).sum(axis=1)
    solid = np.where(nb == 1, 2 * np.pi, np.where(nb == 2, np.pi, np.pi / 2))
    cents, norms, areas = [], [], []
    u = np.arange(k - 1)
    uu, vv = np.meshgrid(u, u, indexing="ij")
    uu = uu.ravel().astype(np.float64)
    vv = vv.ravel().astype(np.float64)
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            o1, o2 = [a for a in range(3) if a != axis]
            for (du0, dv0), (du1, dv1), (du2, dv2) in (
                ((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))):
                c = np.zeros((len(uu), 3))
                c[:, axis] = sgn * side / 2.0
                c[:, o1] = (uu + (du0 + du1 + du2) / 3.0) * h - side / 2.0
                c[:, o2] = (vv + (dv0 + dv1 + dv2) / 3.0) * h - side / 2.0
                nvec = np.zeros((len(uu), 3))
                nvec[:, axis] = sgn
                cents.append(c)
                norms.append(nvec)
                areas.append(np.full(len(uu), 0.5 * h * h))
    return nodes, np.concatenate(cents), np.concatenate(norms), np.concatenate(areas), solid


def ellipsoid_surface(axes, n_nodes_target):
    """Ellipsoid with semi-axes `axes`, meshed as a scaled icosphere.

    Nodes are the scaled icosphere vertices (10 f^2 + 2 ~= n_nodes_target);
    sources are flat-triangle centroids with flat areas and outward normals.
    The surface is smooth, so the solid angle is 2*pi at every node.
    """
    f = max(1, int(round(((n_nodes_target - 2) / 10.0) ** 0.5)))
    v, t = icosphere(f)
    v = v * np.asarray(axes)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    cen = (a + b + c) / 3.0
    return v, cen, nrm, area, np.full(len(v), 2 * np.pi)


def random_rotation(rng):
    """Uniformly random proper rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q
