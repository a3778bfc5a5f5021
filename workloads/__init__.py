"""Seeded synthetic inputs shaped like the paper's boundary-integral workloads.

This module only makes inputs: point clouds, surface quadrature points with
normals and weights, densities, and the physical parameters of each problem.
It holds none of the fast-multipole arithmetic and none of the operator
arithmetic; both the GPU library and the CPU oracle read what it returns.

Every array is returned as float32 (the precision the GPU path consumes); the
oracle upcasts these exact float32 values to float64.

Workloads (all sizes as the paper's problems are scaled here, Sec. IV):
  cube_uniform   N points uniform in [0,1)^3 with densities U[-1,1]
  spheres_8      8 unit spheres on a 2x2x2 lattice (spacing 2.5), icosphere
                 centroid quadrature (one-point rule, Sec. III), double layer
  dielectric     non-overlapping spheres of random radius in a box with
                 random inner permittivities and a uniform external field
  clustered      clustered point cloud (Gaussian blobs + uniform background)
"""

from __future__ import annotations

import math

import numpy as np

from .shapes import (icosphere, sphere_quadrature, cube_surface, ellipsoid_surface, random_rotation,
                     triangle_rule_deg5, mesh_quadrature)

__all__ = [
    "cube_uniform",
    "spheres_8",
    "dielectric",
    "clustered",
    "ferro_batch",
    "icosphere",
    "sphere_quadrature",
    "cube_surface",
    "ellipsoid_surface",
    "triangle_rule_deg5",
    "mesh_quadrature",
    "SINGULAR_RADIUS",
    "float32_bits",
]

# Pairs closer than this are excluded from every sum (Sec. III.A.1).
SINGULAR_RADIUS = 1.0e-5


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def float32_bits(n, seed, lo=-30, hi=30, ties=0):
    """float32 values with random signs, binary exponents in [lo, hi) and
    uniformly random 23-bit fractions, so that every rounding position of a
    narrower format is exercised; the last `ties` values have their low 16
    bits set to 0x8000 (exactly halfway between two bfloat16 values)."""
    rng = np.random.default_rng(seed)
    frac = rng.integers(0, 1 << 23, n, dtype=np.uint32)
    exp = rng.integers(lo + 127, hi + 127, n).astype(np.uint32)
    sign = rng.integers(0, 2, n).astype(np.uint32)
    bits = (sign << 31) | (exp << 23) | frac
    if ties:
        bits[n - ties:] = (bits[n - ties:] & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    return bits.view(np.float32)


def cube_uniform(n=4096, seed=0):
    """N points uniform in [0,1)^3, densities uniform in [-1,1].

    Densities are drawn in float64 and rounded to float32.
    """
    rng = np.random.default_rng(seed)
    xyz = _f32(rng.random((n, 3)))
    q = _f32(rng.uniform(-1.0, 1.0, n))
    return {"name": f"cube_uniform_n{n}", "xyz": xyz, "q": q,
            "root": (0.0, 0.0, 0.0, 1.0)}


def spheres_8(freq=35, seed=2, spacing=2.5, radius=1.0):
    """Eight spheres on a 2x2x2 lattice, each a class-I geodesic icosphere.

    One quadrature point per triangle: the normalised centroid, with the
    outward normal and the exact spherical-triangle area as weight.
    freq=35 gives 20*35^2 = 24,500 points per sphere (196,000 total).
    Also returns a double-layer density mu ~ N(0,1) and the boundary data
    g = 1/|r - r0| with r0 the lattice centre (outside all spheres).
    """
    rng = np.random.default_rng(seed)
    centres = np.array([[i, j, k] for i in (0.0, spacing) for j in (0.0, spacing)
                        for k in (0.0, spacing)], dtype=np.float64)
    pts, nrm, wts, body = [], [], [], []
    for b, c in enumerate(centres):
        p, n, w = sphere_quadrature(freq, c, radius)
        pts.append(p)
        nrm.append(n)
        wts.append(w)
        body.append(np.full(len(w), b, dtype=np.int32))
    xyz = np.concatenate(pts)
    nrm = np.concatenate(nrm)
    w = np.concatenate(wts)
    mu = rng.standard_normal(len(w))
    r0 = np.full(3, spacing / 2.0)
    xyz32 = _f32(xyz)
    g = 1.0 / np.linalg.norm(xyz32.astype(np.float64) - r0, axis=1)
    return {"name": f"spheres_8_f{freq}", "xyz": xyz32, "normals": _f32(nrm),
            "weights": _f32(w), "mu": _f32(mu), "body": np.concatenate(body),
            "centres": centres, "radius": radius, "g": g, "r0": r0}


def dielectric(n_spheres=1000, freq=7, box=40.0, seed=3, gap=0.1,
               rmin=0.5, rmax=1.5, eps_lo=2.0, eps_hi=10.0, eps_m=1.0,
               e0=(0.0, 0.0, 1.0)):
    """Non-overlapping dielectric spheres by random sequential addition.

    Radii ~ U[rmin, rmax], centres in [r, box - r]^3, surface gap >= `gap`.
    Each sphere is an icosphere of frequency `freq` (20*freq^2 points).
    Returns per-point geometry (xyz, outward normals, areas, curvature 1/r),
    per-point inner permittivity eps_i, the medium permittivity and E0.
    """
    rng = np.random.default_rng(seed)
    centres = np.zeros((n_spheres, 3))
    radii = np.zeros(n_spheres)
    k = 0
    tries = 0
    while k < n_spheres:
        tries += 1
        if tries > 200 * n_spheres:
            raise RuntimeError("random sequential addition did not finish")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r, box - r, 3)
        if k:
            d = np.linalg.norm(centres[:k] - c, axis=1)
            if np.any(d < radii[:k] + r + gap):
                continue
        centres[k] = c
        radii[k] = r
        k += 1
    eps_i = rng.uniform(eps_lo, eps_hi, n_spheres)
    pts, nrm, wts, curv, epsp, body = [], [], [], [], [], []
    for b in range(n_spheres):
        p, n, w = sphere_quadrature(freq, centres[b], radii[b])
        pts.append(p)
        nrm.append(n)
        wts.append(w)
        curv.append(np.full(len(w), 1.0 / radii[b]))
        epsp.append(np.full(len(w), eps_i[b]))
        body.append(np.full(len(w), b, dtype=np.int32))
    return {"name": f"dielectric_{n_spheres}x{20 * freq * freq}",
            "xyz": _f32(np.concatenate(pts)), "normals": _f32(np.concatenate(nrm)),
            "areas": _f32(np.concatenate(wts)), "curvature": _f32(np.concatenate(curv)),
            "eps_i": _f32(np.concatenate(epsp)), "eps_m": float(eps_m),
            "e0": np.asarray(e0, dtype=np.float64), "centres": centres, "radii": radii,
            "eps_body": eps_i, "body": np.concatenate(body)}


def _reject_close(xyz, rng, sampler, min_dist):
    """Re-draw points that sit within `min_dist` of another (non-identical) point."""
    from scipy.spatial import cKDTree

    for _ in range(50):
        pts32 = xyz.astype(np.float32).astype(np.float64)
        tree = cKDTree(pts32)
        pairs = tree.query_pairs(min_dist, output_type="ndarray")
        if len(pairs) == 0:
            return xyz
        bad = np.unique(pairs[:, 1])
        xyz[bad] = sampler(len(bad), bad)
    raise RuntimeError("could not separate close pairs")


def clustered(n=4_000_000, seed=4, n_blobs=64, frac_blob=0.7, sigma=0.02,
              min_dist=2.0 * SINGULAR_RADIUS):
    """Clustered cloud in [0,1)^3: 70% in 64 Gaussian blobs, 30% uniform.

    Blob centres ~ U[0.1,0.9]^3, sigma 0.02; blob points falling outside
    [0,1)^3 are re-drawn. No two points are closer than `min_dist`, so the
    singular-exclusion test never sits at its threshold. Normals are
    isotropic unit vectors; q and mu ~ N(0,1).
    """
    rng = np.random.default_rng(seed)
    n_blob = int(round(n * frac_blob))
    per = np.full(n_blobs, n_blob // n_blobs)
    per[: n_blob - per.sum()] += 1
    centres = rng.uniform(0.1, 0.9, (n_blobs, 3))
    owner = np.repeat(np.arange(n_blobs), per)

    def draw_blob(idx_owner):
        out = centres[idx_owner] + sigma * rng.standard_normal((len(idx_owner), 3))
        bad = np.any((out < 0.0) | (out >= 1.0), axis=1)
        while np.any(bad):
            out[bad] = centres[idx_owner[bad]] + sigma * rng.standard_normal((bad.sum(), 3))
            bad = np.any((out < 0.0) | (out >= 1.0), axis=1)
        return out

    xyz = np.empty((n, 3))
    xyz[:n_blob] = draw_blob(owner)
    xyz[n_blob:] = rng.random((n - n_blob, 3))
    all_owner = np.concatenate([owner, np.full(n - n_blob, -1)])

    def sampler(k, idx):
        out = np.empty((k, 3))
        ob = all_owner[idx]
        m = ob >= 0
        if m.any():
            out[m] = draw_blob(ob[m])
        if (~m).any():
            out[~m] = rng.random(((~m).sum(), 3))
        return out

    xyz = _reject_close(xyz, rng, sampler, min_dist)
    perm = rng.permutation(n)
    xyz = xyz[perm]
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    q = rng.standard_normal(n)
    mu = rng.standard_normal(n)
    return {"name": f"clustered_n{n}", "xyz": _f32(xyz), "normals": _f32(nrm),
            "q": _f32(q), "mu": _f32(mu), "root": (0.0, 0.0, 0.0, 1.0)}


def ferro_batch(n_inst=256, seed=5, nmin=2000, nmax=64000):
    """Batch of ferromagnet surface instances: cubes and ellipsoids.

    Instance sizes (target nodes) are log-uniform in [nmin, nmax]. Targets are
    surface nodes; sources are triangle centroids with flat-triangle area
    weights and outward normals. Each instance has a random rotation and
    offset; M is a random unit vector per instance. Returns a list of dicts.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        nt = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        rot = random_rotation(rng)
        centre = rng.uniform(-1.0, 1.0, 3)
        m = rng.standard_normal(3)
        m /= np.linalg.norm(m)
        if i % 2 == 0:
            side = rng.uniform(0.5, 2.0)
            nodes, cen, nrm, area, solid = cube_surface(side, nt)
            kind = "cube"
            dims = (side, side, side)
        else:
            axes = rng.uniform(0.5, 2.0, 3)
            nodes, cen, nrm, area, solid = ellipsoid_surface(axes, nt)
            kind = "ellipsoid"
            dims = tuple(axes)
        nodes = nodes @ rot.T + centre
        cen = cen @ rot.T + centre
        nrm = nrm @ rot.T
        out.append({"kind": kind, "dims": dims, "rot": rot, "centre": centre, "M": m,
                    "trg": _f32(nodes), "src": _f32(cen), "normals": _f32(nrm),
                    "weights": _f32(area), "solid_angle": solid})
    return out
