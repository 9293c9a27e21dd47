"""Pins of the oracle's Alg. 1 (FISTA on the local problem, Sec. 2.2):
simplex projection, the Lipschitz bound Eq. (lipschitz_est), the FISTA rate
Eq. (fista_convergence), and convergence to the exact minimum."""
import numpy as np
import pytest
import scipy.optimize as so

import oracle as O
from conftest import rng
from test_oracle_local import random_face


@pytest.mark.parametrize("seed", range(10))
def test_simplex_projection_vs_qp(seed):
    r = rng(seed)
    y = r.normal(size=3) * 2
    p = O.simplex_projection(y)
    res = so.minimize(lambda a: ((a - y) ** 2).sum(), np.full(3, 1 / 3), method="SLSQP",
                      bounds=[(0, None)] * 3, constraints=[{"type": "eq", "fun": lambda a: a.sum() - 1}],
                      options=dict(ftol=1e-15))
    assert np.allclose(p, res.x, atol=1e-6)
    assert p.min() >= 0 and p.sum() == pytest.approx(1.0)


@pytest.mark.parametrize("seed", range(8))
def test_lipschitz_bound_holds(seed):
    """Eq. (lipschitz_est) bounds the Lipschitz constant of grad h on the simplex."""
    r = rng(20 + seed)
    Q = random_face(r)
    L = O.lipschitz_bound(Q)
    a = r.dirichlet(np.ones(3), size=2000)
    b = r.dirichlet(np.ones(3), size=2000)
    ga = (a @ Q) / np.sqrt(np.einsum("ni,ij,nj->n", a, Q, a))[:, None]
    gb = (b @ Q) / np.sqrt(np.einsum("ni,ij,nj->n", b, Q, b))[:, None]
    ratio = np.linalg.norm(ga - gb, axis=1) / np.linalg.norm(a - b, axis=1)
    assert ratio.max() <= L


@pytest.mark.parametrize("seed", range(8))
def test_fista_rate_bound(seed):
    """Eq. (fista_convergence): phi^k - phi* <= 2 L ||alpha_0 - alpha*||^2 / (k+1)^2."""
    r = rng(40 + seed)
    Q = random_face(r)
    Phi = r.uniform(-0.5, 0.5, size=3) * np.sqrt(np.trace(Q) / 3)
    L = O.lipschitz_bound(Q)
    val, astar, _ = O.local_solve(Q, Phi)
    n_f = 200
    _, _, hist = O.fista_local(Q, Phi, L, n_f)
    a0 = np.full(3, 1 / 3)
    k = np.arange(1, n_f + 1)
    bound = 2 * L * ((a0 - astar) ** 2).sum() / (k + 1) ** 2
    assert np.all(hist - val <= bound + 1e-12)
    assert np.all(hist >= val - 1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_fista_tight_converges_to_exact(seed):
    r = rng(60 + seed)
    Q = random_face(r)
    Phi = r.uniform(-0.5, 0.5, size=3) * np.sqrt(np.trace(Q) / 3)
    val, _, _ = O.local_solve(Q, Phi)
    Lt = O.lipschitz_tight(Q)
    assert Lt <= O.lipschitz_bound(Q)
    a, v, _ = O.fista_local(Q, Phi, Lt, 3000)
    assert v == pytest.approx(val, rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("seed", range(8))
def test_fista_iterations_meet_tolerance(seed):
    """Per-face counts from Eq. (fista_convergence): with the Lipschitz bound of
    Eq. (lipschitz_est) the value after that many iterations is within tau of the
    exact minimum, for tolerances from loose to tight; one iteration fewer is not
    always enough for the bound (the count is the smallest the bound allows)."""
    r = rng(80 + seed)
    Q = random_face(r)
    Phi = r.uniform(-0.5, 0.5, size=3) * np.sqrt(np.trace(Q) / 3)
    val, astar, _ = O.local_solve(Q, Phi)
    L = O.lipschitz_bound(Q)
    for tau in (1e-1, 1e-2, 1e-3, 1e-4):
        n = int(O.fista_iterations(L, tau, 10 ** 6))
        _, v, _ = O.fista_local(Q, Phi, L, n)
        assert v - val <= tau * (1 + 1e-9)
        # the count is the least k with 2 L (2/3) / (k+1)^2 <= tau (float64 rounding only)
        assert 2 * L * (2 / 3) / (n + 1) ** 2 <= tau * (1 + 1e-12)
        if n > 1:
            assert 2 * L * (2 / 3) / n ** 2 > tau * (1 - 1e-12)


def test_fista_iterations_limits():
    L = np.array([1.0, 3.0, 1e8, np.inf, np.nan, 0.0], np.float32)
    assert list(O.fista_iterations(L, 0.0, 50)) == [50] * 6
    n = O.fista_iterations(L, 1.0, 50)
    # sqrt(4/3) = 1.15 -> 1 iteration; sqrt(4) = 2 -> 1; capped; non-finite -> cap; L = 0 -> 1
    assert list(n) == [1, 1, 50, 50, 50, 1]
    assert list(O.fista_iterations(np.float32(300.0), 1e-2, 10 ** 6)[None]) == [199]
    # counts never grow as the tolerance loosens
    taus = np.logspace(-6, 1, 40)
    c = [int(O.fista_iterations(np.float32(123.4), t, 10 ** 7)) for t in taus]
    assert all(a >= b for a, b in zip(c, c[1:]))
