"""Lead weights B = K Z assembled on the GPU (Sec. 2.4) against the oracle's
`lead_field`.  Both sides read the same float32 coordinates and electrodes and
work in FP64; the GPU rounds its result to float32 once, so the bar is float32
rounding of each weight (rtol 1e-6, plus 1e-7 of the largest weight for the
entries that nearly cancel).  The ECG computed from the GPU's weights is held
to the ECG bar (1e-3)."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from test_gpu_parity import B, _dev, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _check(W, Wo):
    W = np.asarray(W, np.float64)
    np.testing.assert_allclose(W, Wo, rtol=1e-6, atol=1e-7 * np.abs(Wo).max())


def test_lead_field_cube_matches_oracle():
    dev = _dev()
    xyz, tets = gi.kuhn_cube(8)
    x = gi.jitter_nodes(xyz, 1.0 / 8, 0.15, 3)
    e = gi.sphere_electrodes(np.full(3, 0.5), 3.0, 8, seed=4).astype(np.float32)
    plan = B().Plan(x, tets)
    W = B().lead_field(plan, t32(e, dev)).cpu().numpy()
    Wo = O.lead_field(x.astype(np.float32), tets, e)
    _check(W, Wo)
    assert np.abs(W.astype(np.float64).sum(0)).max() <= 1e-6 * np.abs(W).sum(0).max()


def test_lead_field_shell_and_ecg():
    dev = _dev()
    p = gi.shell_problem(12_000, seed=91)
    e = p.extra.get("electrodes")
    if e is None:
        e = gi.sphere_electrodes(p.xyz.mean(0), 3 * np.abs(p.xyz - p.xyz.mean(0)).max(), 12, seed=5)
    e = np.asarray(e, np.float32)
    plan = B().Plan(p.xyz, p.tets)
    W = B().lead_field(plan, t32(e, dev))
    Wo = O.lead_field(p.xyz, p.tets, e)
    _check(W.cpu().numpy(), Wo)
    To, _ = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t)
    a = p.ap
    ap = B().make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
    ecg = B().ecg_forward(t32(To, dev), W, ap).cpu().numpy()
    eo = O.ecg_forward(To, Wo, p.ap)
    assert np.abs(ecg - eo).max() <= 1e-3 * np.abs(eo).max()


def test_lead_field_errors():
    dev = _dev()
    p = gi.cube_problem(3)
    plan = B().Plan(p.xyz, p.tets)
    with pytest.raises(B().GbpError):
        B().lead_field(plan, t32(np.zeros((0, 3)), dev))
    with pytest.raises(B().GbpError):
        B().lead_field(plan, t32(np.zeros((300, 3)), dev))


def test_lead_field_max_leads():
    """256 electrodes (the most one call takes: 32 chunks of 8) on a jittered cube."""
    dev = _dev()
    xyz, tets = gi.kuhn_cube(5)
    x = gi.jitter_nodes(xyz, 1.0 / 5, 0.15, 8)
    e = gi.sphere_electrodes(np.full(3, 0.5), 2.5, 256, seed=9).astype(np.float32)
    plan = B().Plan(x, tets)
    W = B().lead_field(plan, t32(e, dev)).cpu().numpy()
    assert W.shape == (len(x), 256)
    _check(W, O.lead_field(x.astype(np.float32), tets, e))
    with pytest.raises(B().GbpError):
        B().lead_field(plan, t32(np.zeros((257, 3)), dev))


def test_lead_field_full_size():
    """500k-vertex shell, 12 electrodes: element by element against the oracle."""
    dev = _dev()
    p = gi.shell_problem(500_000, seed=2)
    e = gi.sphere_electrodes(p.xyz.mean(0), 3 * np.abs(p.xyz - p.xyz.mean(0)).max(), 12, seed=6)
    e = np.asarray(e, np.float32)
    print(f"[case] lead field n_v={p.n_v} n_e={p.n_e} leads=12", flush=True)
    plan = B().Plan(p.xyz, p.tets)
    W = B().lead_field(plan, t32(e, dev)).cpu().numpy()
    _check(W, O.lead_field(p.xyz, p.tets, e))
