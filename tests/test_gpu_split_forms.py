"""The M2L arithmetics side by side through the C ABI: float32, bf16x6 (three
bfloat16 parts, six products), bf16x4 and bf16x3 (two parts). On one plan
shape each is compared with the float64 direct sum and with the float32
form: bf16x6 is at float32 accuracy, the two-part forms add the error of
16-bit operands (about 2^-16 per product) to the far field only. Both far-field
forms, with tiles cut into pieces and sparse pair tiles exercised."""

import numpy as np
import pytest

import workloads as W
from oracle import direct as D

from gpu_common import errors, fmm_run, say

pytestmark = pytest.mark.gpu

PRECS = {"fp32": 0, "bf16x6": 1, "bf16x3": 2, "bf16x4": 3}


@pytest.mark.parametrize("basis,order,eps", [(0, 6, 1e-8), (1, 7, 1e-7)])
def test_m2l_arithmetics_against_direct_and_float32(basis, order, eps):
    d = W.clustered(40000, seed=17)
    x, nrm, q, mu = d["xyz"], d["normals"], d["q"], d["mu"]
    say(f"test_m2l_arithmetics_against_direct_and_float32: n=40000 basis {basis} order {order}")
    sample = np.sort(np.random.default_rng(3).choice(len(x), 3000, replace=False))
    ref, _ = D.direct_sum(x[sample], x, q, mu[:, None].astype(np.float64) * nrm)
    out = {}
    for name, prec in PRECS.items():
        r = fmm_run(x, q=q, mu=mu, nrm=nrm, order=order, leaf=48, root=d["root"], pinv_eps=eps, basis=basis,
                    precision=prec, m2l_pieces=2)
        out[name] = r["pot"][0]
        l2, worst = errors(out[name][sample], ref)
        say(f"  {name}: vs direct rel L2 {l2:.2e} (worst {worst:.1e}); vs float32 "
            f"{errors(out[name], out['fp32'])[0] if name != 'fp32' else 0.0:.2e}")
    e = {k: errors(v, out["fp32"])[0] for k, v in out.items() if k != "fp32"}
    d_ref = {k: errors(v[sample], ref)[0] for k, v in out.items()}
    assert e["bf16x6"] < 1e-6
    # the two-part forms: 16-bit operands in the far field only
    assert e["bf16x4"] < 3e-5 and e["bf16x3"] < 3e-5
    assert e["bf16x6"] < e["bf16x4"] and e["bf16x6"] < e["bf16x3"]
    assert d_ref["bf16x6"] < 1.5 * d_ref["fp32"] + 1e-7
    assert d_ref["bf16x3"] < d_ref["fp32"] + 3e-5
