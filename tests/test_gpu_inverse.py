"""Inverse loop: multi-start Adam fit of the velocity scale and root onsets to an
ECG that the FP64 oracle computed from hidden parameters.  The misfit must fall
substantially and the captured iterations must stay within their budgets."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from test_gpu_parity import _dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("warm", [True, False])
def test_multistart_fit_reduces_misfit(warm):
    _dev()
    from paper_2308_08410_amd.inverse import MultiStartFit
    p = gi.shell_problem(8_000, seed=13, n_roots=4, n_leads=12)
    vs_true = gi.smooth_field(p.xyz, 0.7, 1.3, seed=23)
    ap = dict(p.ap, n_steps=200)
    To, _ = O.solve(p.xyz, p.tets, p.D, vs_true, p.root_node, p.root_t)
    target = O.ecg_forward(To, p.W, ap)
    rng = np.random.Generator(np.random.PCG64(3))
    starts = 3
    vs0 = [np.ones(p.n_v, np.float32) for _ in range(starts)]
    rt0 = [(p.root_t + rng.uniform(-6, 6, size=len(p.root_t))).astype(np.float32) for _ in range(starts)]
    fit = MultiStartFit(p.xyz, p.tets, p.D, p.W, p.root_node, target, ap, vs0, rt0, warm=warm)
    out = fit.run(120, log_every=10, check_every=10)
    first, last = out["history"][0][1], out["history"][-1][1]
    assert np.all(np.isfinite(last))
    assert np.all(last < 0.3 * first), (first, last)
    # the fitted onsets moved towards the hidden ones for the best start
    best = int(np.argmin(last))
    _, rt_b, _ = fit.instance(best)
    err0 = np.abs(rt0[best] - p.root_t).mean()
    err1 = np.abs(rt_b.cpu().numpy() - p.root_t).mean()
    assert err1 < err0
