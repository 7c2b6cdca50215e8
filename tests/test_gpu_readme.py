"""The Python example in README.md runs as written and computes what it says."""
import os
import re

import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded

pytestmark = pytest.mark.gpu

README = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "README.md")


def test_readme_python_example():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    code = re.search(r"```python\n(.*?)```", open(README).read(), re.S).group(1)
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    torch.cuda.synchronize()
    xh = ns["x"].cpu().numpy()
    so, co = oracle.sincos(xh, 0, 0, threads=oracle.default_threads())
    assert_bit_exact(ns["s"].cpu().numpy(), so, "README sin", xh)
    assert_bit_exact(ns["c"].cpu().numpy(), co, "README cos", xh)
    z = ns["z"].cpu().numpy()
    assert_bit_exact(z[0::2], co, "README complex cos", xh)
    assert_bit_exact(z[1::2], so, "README complex sin", xh)
    for (a, s, c) in ns["segs"]:
        ah = a.cpu().numpy()
        so2, co2 = oracle.sincos(ah, 0, 0)
        assert_bit_exact(s.cpu().numpy(), so2, "README ragged sin", ah)
        assert_bit_exact(c.cpu().numpy(), co2, "README ragged cos", ah)
    g = ns["theta"].grad.cpu().numpy()
    want = (co.astype(np.float32) - so.astype(np.float32)).astype(np.float32)
    assert np.array_equal(g.view(np.uint32), want.view(np.uint32))
    # the fit step: the loss of the oracle's forward model, the same gradients as autograd
    from paper_cs_0406049_amd.autograd import sinusoid
    th, Ah, wh, ph = (ns[k].cpu().numpy() for k in ("t", "A", "w", "phi"))
    y_obs = ns["torch"].sin(3 * ns["t"])
    r = oracle.sinusoid_forward(th, Ah, wh, ph).astype(np.float64) - y_obs.cpu().numpy()
    assert abs(float(ns["loss"]) - 0.5 * float((r * r).sum())) <= 1e-5 * 0.5 * float((r * r).sum())
    Ap, wp, pp = (ns[k].clone().requires_grad_(True) for k in ("A", "w", "phi"))
    (0.5 * ((sinusoid(ns["t"], Ap, wp, pp) - y_obs) ** 2).sum()).backward()
    for got, ref in ((ns["gA"], Ap.grad), (ns["gw"], wp.grad), (ns["gphi"], pp.grad)):
        assert torch.equal(got, ref)
    # the served request: the same bits as the plain call
    assert_bit_exact(ns["s_req"].cpu().numpy(), so, "README served sin", xh)
    assert_bit_exact(ns["c_req"].cpu().numpy(), co, "README served cos", xh)
