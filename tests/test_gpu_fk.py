"""Magnetostatics end to end on the GPU (Sec. II.B, Sec. IV.A): for a batch of
uniformly magnetised bodies, phi = phi_1 + phi_2 with phi_1 = 4 pi M.r and
phi_2 = D[phi_1 w] + (Omega/(4 pi) - 1) phi_1 (Eq. fk_integral_discrete),
three right-hand sides (M = e_x, e_y, e_z) in one batched plan; the
demagnetising tensor from the surface values against the oracle on the direct
sum and against the closed forms (cube: I/3; ellipsoid: Osborn's factors in
the body frame; trace 1 for every body)."""

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import operators as OP

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def _bodies():
    rng = np.random.default_rng(21)
    out = []
    for kind, dims in (("cube", (1.0,)), ("ellipsoid", (1.0, 0.7, 0.5)), ("cube", (1.6,)),
                       ("ellipsoid", (0.6, 1.2, 0.9))):
        rot = W.random_rotation(rng)
        if kind == "cube":
            _, cen, nrm, area, _ = W.cube_surface(dims[0], 6000)
            vol = dims[0] ** 3
        else:
            _, cen, nrm, area, _ = W.ellipsoid_surface(dims, 6000)
            vol = 4.0 / 3.0 * np.pi * np.prod(dims)
        shift = rng.uniform(-1, 1, 3)  # bodies overlap in space: instances must not interact
        out.append(dict(kind=kind, dims=dims, rot=rot, vol=vol, xyz=cen @ rot.T + shift, nrm=nrm @ rot.T,
                        w=area, shift=shift))
    return out


def test_demag_tensors_of_a_batch():
    import torch

    import paper_1605_01715_amd as F

    bodies = _bodies()
    off = np.concatenate([[0], np.cumsum([len(b["w"]) for b in bodies])])
    xyz = np.concatenate([b["xyz"] for b in bodies]).astype(np.float32)
    nrm = np.concatenate([b["nrm"] for b in bodies]).astype(np.float32)
    w = np.concatenate([b["w"] for b in bodies])
    # phi_1 = 4 pi M.(r - centre) per body; the double-layer density is phi_1 w
    phi1 = np.concatenate([np.stack([4 * np.pi * (b["xyz"][:, c] - b["shift"][c]) for c in range(3)], axis=1)
                           for b in bodies]).T  # [3][n]
    mu = (phi1 * w).astype(np.float32)
    say(f"test_demag_tensors_of_a_batch: {len(bodies)} bodies, {off[-1]} elements")
    opts = F.fmm_default_options(order=8, leaf_size=64, src_kernels=F.FMM_SRC_DOUBLE, outputs=F.FMM_OUT_POT, nrhs=3)
    plan = F.fmm_setup_batch(off, dev(xyz), dev(nrm), options=opts)
    pot = torch.empty(3 * int(off[-1]), device="cuda:0")
    F.fmm_apply(plan, mu=dev(np.ascontiguousarray(mu)), pot=pot)
    torch.cuda.synchronize()
    F.fmm_destroy(plan)
    dl = pot.cpu().numpy().astype(np.float64).reshape(3, -1)
    # elements are triangle centroids: solid angle 2 pi, Omega/(4 pi) - 1 = -1/2
    phi = phi1 + dl - 0.5 * phi1
    for i, b in enumerate(bodies):
        s = slice(off[i], off[i + 1])
        n_gpu = CF.demag_tensor_from_surface(phi[:, s], b["nrm"], b["w"], b["vol"])
        x64 = b["xyz"].astype(np.float32).astype(np.float64)
        n64 = b["nrm"].astype(np.float32).astype(np.float64)
        w64 = b["w"].astype(np.float32).astype(np.float64)
        a = np.full(len(w64), -0.5)
        ref = np.stack([phi1[c, s] + OP.fk_apply(phi1[c, s], x64, n64, w64, a) for c in range(3)])
        n_ref = CF.demag_tensor_from_surface(ref, b["nrm"], b["w"], b["vol"])
        if b["kind"] == "cube":
            exact = np.eye(3) / 3
        else:
            exact = b["rot"] @ np.diag(CF.ellipsoid_demag(b["dims"])) @ b["rot"].T
        e_or = np.abs(n_gpu - n_ref).max()
        e_cf = np.abs(n_gpu - exact).max()
        say(f"  body {i} ({b['kind']} {b['dims']}): trace {np.trace(n_gpu):.4f}, vs oracle {e_or:.1e}, "
            f"vs closed form {e_cf:.1e}")
        assert e_or < 1e-5
        assert abs(np.trace(n_gpu) - 1.0) < 1.5e-2
        assert e_cf < 1e-2
