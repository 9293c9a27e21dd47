"""Pins of the oracle's ECG (Sec. 2.4): template shape as the paper states it,
lead-field invariances, exact time-shift equivariance, and FD of the backward."""
import json
import os

import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from conftest import rng

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def rabbit_ap(**kw):
    c = GOLD["rabbit_template"]
    ap = dict(K0=c["K0_mV"], K1=c["K1_mV"], tau=c["tau_ms"], t0=0.0, dt=1.0, n_steps=120)
    ap.update(kw)
    return ap


def test_template_range_is_K0_to_K1():
    """Sec. 2.4: K0 and K1 are the minimum and maximum transmembrane potential
    (this pins the reading U = K0 + (K1-K0)/2 (1 + tanh(2 xi/tau)))."""
    ap = rabbit_ap()
    xi = np.linspace(-50, 50, 10001)
    U = O.ap_template(xi, **ap)
    assert U.min() == pytest.approx(ap["K0"], abs=1e-9)
    assert U.max() == pytest.approx(ap["K1"], abs=1e-9)
    assert O.ap_template(0.0, **ap) == pytest.approx(0.5 * (ap["K0"] + ap["K1"]))
    assert np.all(np.diff(U) >= 0)
    # the cube workload's template 0.5 (1 + tanh((t - T)/0.5)) is K0=0, K1=1, tau=1
    cube = dict(gi.AP_CUBE)
    assert np.allclose(O.ap_template(xi, **cube), 0.5 * (1 + np.tanh(xi / 0.5)))


def test_template_derivative_fd():
    ap = rabbit_ap()
    xi = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (O.ap_template(xi + h, **ap) - O.ap_template(xi - h, **ap)) / (2 * h)
    assert np.allclose(O.ap_template_deriv(xi, **ap), fd, rtol=1e-6, atol=1e-6)


@pytest.fixture(scope="module")
def small_cube():
    p = gi.cube_problem(6, jitter=0.1)
    T, _ = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t)
    return p, T


def test_lead_weights_sum_to_zero(small_cube):
    p, _ = small_cube
    W = p.W.astype(np.float64)
    assert np.abs(W.sum(0)).max() < 1e-6 * np.abs(W).sum(0).max()


def test_ecg_offset_and_uniform_invariance(small_cube):
    p, T = small_cube
    ap = dict(p.ap)
    e0 = O.ecg_forward(T, p.W, ap)
    ap2 = dict(ap, K0=-85.0, K1=-84.0)          # same amplitude, offset K0
    e1 = O.ecg_forward(T, p.W, ap2)
    scale = np.abs(e0).max()
    assert np.abs(e1 - e0).max() < 1e-5 * scale + 85 * np.abs(p.W.astype(np.float64).sum(0)).max()
    eu = O.ecg_forward(np.full_like(T, 0.7), p.W, ap)
    assert np.abs(eu).max() < 1e-5 * scale
    # silent before the earliest activation, silent long after the latest
    ap3 = dict(ap, t0=-5.0, n_steps=10)
    assert np.abs(O.ecg_forward(T, p.W, ap3)).max() < 1e-9 * scale + 1e-12
    ap4 = dict(ap, t0=T.max() + 20.0, n_steps=10)
    assert np.abs(O.ecg_forward(T, p.W, ap4)).max() < 1e-5 * scale


def test_ecg_time_shift_is_exact(small_cube):
    p, T = small_cube
    ap = dict(p.ap)
    k = 7
    e0 = O.ecg_forward(T, p.W, ap)
    e1 = O.ecg_forward(T + k * ap["dt"], p.W, ap)
    assert np.allclose(e1[k:], e0[:-k], rtol=1e-12, atol=1e-12 * np.abs(e0).max())


def test_ecg_linear_in_W(small_cube):
    p, T = small_cube
    r = rng(3)
    W2 = r.normal(size=p.W.shape)
    a, b = 0.7, -1.3
    lhs = O.ecg_forward(T, a * p.W.astype(np.float64) + b * W2, p.ap)
    rhs = a * O.ecg_forward(T, p.W, p.ap) + b * O.ecg_forward(T, W2, p.ap)
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12)


def test_ecg_backward_fd(small_cube):
    p, T = small_cube
    r = rng(4)
    ap = dict(p.ap)
    G = r.normal(size=(ap["n_steps"], p.W.shape[1]))
    dT = O.ecg_backward(T, p.W, ap, G)
    h = 1e-5
    for n in r.choice(len(T), size=12, replace=False):
        e = np.zeros_like(T)
        e[n] = h
        fp = (G * O.ecg_forward(T + e, p.W, ap)).sum()
        fm = (G * O.ecg_forward(T - e, p.W, ap)).sum()
        assert (fp - fm) / (2 * h) == pytest.approx(dT[n], rel=1e-5, abs=1e-9)


def test_unreached_nodes_rest(small_cube):
    p, T = small_cube
    T2 = T.copy()
    T2[:5] = np.inf
    ap = dict(p.ap)
    e = O.ecg_forward(T2, p.W, ap)
    W = p.W.astype(np.float64)
    ref = O.ecg_forward(T2[5:], W[5:], ap) + ap["K0"] * W[:5].sum(0)[None, :]
    assert np.allclose(e, ref, rtol=1e-12, atol=1e-14)
    assert np.all(O.ecg_backward(T2, p.W, ap, np.ones((ap["n_steps"], W.shape[1])))[:5] == 0)


def test_loss_and_gradient():
    r = rng(5)
    a = r.normal(size=(50, 12))
    b = r.normal(size=(50, 12))
    L, G = O.ecg_loss(a, b)
    assert L == pytest.approx(((a - b) ** 2).mean())
    h = 1e-6
    e = np.zeros_like(a)
    e[3, 4] = h
    assert (O.ecg_loss(a + e, b)[0] - O.ecg_loss(a - e, b)[0]) / (2 * h) == pytest.approx(G[3, 4], rel=1e-6)
