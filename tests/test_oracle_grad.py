"""Pins of the oracle's adjoint (Sec. 2.3): exact homogeneity identities of the
discrete scheme, central finite differences, and back-propagation through the
unrolled global iteration (the paper's own strategy)."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import rng
from test_oracle_fim import jittered_problem


def loss_T(x, tets, D6, vs, roots, rt, g):
    T, st = O.solve(x, tets, D6, vs, roots, rt, eps_abs=0.0, eps_rel=1e-15)
    return float(g @ T)


@pytest.mark.parametrize("seed", range(4))
def test_gradient_identities(seed):
    """For L = g.T:
       shift:        sum_r dL/dt_r = sum_i g_i
       velocity:     sum_n s_n dL/ds_n - sum_r t_r dL/dt_r = -g.T   (T(cs, t/c) = T/c)
       tensor:       sum_j <D_j, dL/dD_j> - 1/2 sum_r t_r dL/dt_r = -1/2 g.T
                                                              (T(cD, t/sqrt c) = T/sqrt c)"""
    x, tets, D6, vs, roots, rt = jittered_problem(50 + seed)
    T, _ = O.solve(x, tets, D6, vs, roots, rt)
    g = rng(seed).normal(size=len(T))
    res = O.adjoint(x, tets, D6, vs, roots, rt, T, g)
    gT = g @ T
    assert res["droot_t"].sum() == pytest.approx(g.sum(), rel=1e-10)
    lhs_v = vs @ res["dvscale"] - rt @ res["droot_t"]
    assert lhs_v == pytest.approx(-gT, rel=1e-9)
    lhs_d = (D6 * res["dD"]).sum() - 0.5 * rt @ res["droot_t"]
    assert lhs_d == pytest.approx(-0.5 * gT, rel=1e-9)


@pytest.mark.parametrize("seed", range(2))
def test_gradient_central_fd(seed):
    x, tets, D6, vs, roots, rt = jittered_problem(60 + seed, n=3)
    T, _ = O.solve(x, tets, D6, vs, roots, rt, eps_abs=0.0, eps_rel=1e-15)
    r = rng(seed)
    g = r.normal(size=len(T))
    res = O.adjoint(x, tets, D6, vs, roots, rt, T, g)
    h = 1e-6
    # onsets
    for k in range(len(rt)):
        e = np.zeros_like(rt)
        e[k] = h
        fd = (loss_T(x, tets, D6, vs, roots, rt + e, g) - loss_T(x, tets, D6, vs, roots, rt - e, g)) / (2 * h)
        assert fd == pytest.approx(res["droot_t"][k], rel=1e-4, abs=1e-6)
    # nodal velocity scales
    for n in r.choice(len(x), size=6, replace=False):
        e = np.zeros_like(vs)
        e[n] = h
        fd = (loss_T(x, tets, D6, vs + e, roots, rt, g) - loss_T(x, tets, D6, vs - e, roots, rt, g)) / (2 * h)
        assert fd == pytest.approx(res["dvscale"][n], rel=1e-4, abs=1e-6)
    # element tensors (all 6 packed components of a few elements)
    for j in r.choice(len(tets), size=4, replace=False):
        for c in range(6):
            e = np.zeros_like(D6)
            e[j, c] = h
            fd = (loss_T(x, tets, D6 + e, vs, roots, rt, g) - loss_T(x, tets, D6 - e, vs, roots, rt, g)) / (2 * h)
            assert fd == pytest.approx(res["dD"][j, c], rel=1e-4, abs=1e-6)


@pytest.mark.parametrize("seed", range(3))
def test_backprop_through_iteration_equals_adjoint(seed):
    """Sec. 2.3: back-propagating through Alg. 2 equals the frozen-parent adjoint."""
    from oracle.alg2_autograd import solve_autograd
    x, tets, D6, vs, roots, rt = jittered_problem(70 + seed, n=2)
    D6_t = torch.tensor(D6, requires_grad=True)
    vs_t = torch.tensor(vs, requires_grad=True)
    rt_t = torch.tensor(rt, requires_grad=True)
    T_t = solve_autograd(x, tets, D6_t, vs_t, roots, rt_t)
    T, _ = O.solve(x, tets, D6, vs, roots, rt)
    assert np.abs(T_t.detach().numpy() - T).max() < 1e-11
    g = rng(seed).normal(size=len(T))
    (torch.tensor(g) * T_t).sum().backward()
    res = O.adjoint(x, tets, D6, vs, roots, rt, T, g)
    assert np.allclose(rt_t.grad.numpy(), res["droot_t"], rtol=1e-8, atol=1e-10)
    assert np.allclose(vs_t.grad.numpy(), res["dvscale"], rtol=1e-8, atol=1e-10)
    assert np.allclose(D6_t.grad.numpy(), res["dD"], rtol=1e-8, atol=1e-10)


def test_overshadowed_root_has_zero_gradient():
    """Sec. 2.5: a root reached earlier by another activation gets no gradient."""
    x, tets, D6, vs, roots, rt = jittered_problem(80, n=3)
    roots = np.array([0, len(x) - 1], np.int32)
    rt = np.array([0.0, 100.0])                    # second root overshadowed
    T, _ = O.solve(x, tets, D6, vs, roots, rt)
    g = np.ones(len(T))
    res = O.adjoint(x, tets, D6, vs, roots, rt, T, g)
    assert res["droot_t"][1] == 0.0
    assert res["droot_t"][0] == pytest.approx(len(T))
