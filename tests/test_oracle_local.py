"""Pins of the oracle's local solver (Sec. 2.2, Eq. (upwind_eq_lsqr)) against
things other than itself: a barycentric brute force, scipy's constrained
minimiser, the textbook edge cost, shift equivariance and Danskin's theorem."""
import numpy as np
import pytest
import scipy.optimize as so

import oracle as O
from conftest import rng, random_spd


def random_face(r, aniso=6.0):
    """Random non-degenerate tet + SPD metric -> Q = E^T Minv E for vertex 0."""
    while True:
        v = r.normal(size=(4, 3))
        E = (v[1:] - v[0]).T
        if abs(np.linalg.det(E)) > 0.2:
            break
    Minv = random_spd(r, 3, aniso)
    return E.T @ Minv @ E


def objective(Q, Phi, a):
    return a @ Phi + np.sqrt(np.einsum("...i,ij,...j->...", a, Q, a))


def brute(Q, Phi, N=300):
    i, j = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="ij")
    m = (i + j) <= N
    a = np.stack([i[m] / N, j[m] / N, (N - i[m] - j[m]) / N], axis=1)
    fin = np.isfinite(Phi)
    P = np.where(fin, Phi, 0.0)
    f = a @ P + np.sqrt(np.einsum("ni,ij,nj->n", a, Q, a))
    # alpha must vanish on infinite vertices
    bad = (a[:, ~fin] > 0).any(axis=1) if (~fin).any() else np.zeros(len(a), bool)
    f[bad] = np.inf
    k = np.argmin(f)
    return f[k], a[k]


@pytest.mark.parametrize("seed", range(40))
def test_local_vs_bruteforce(seed):
    r = rng(seed)
    Q = random_face(r)
    scale = np.sqrt(np.trace(Q) / 3)
    Phi = r.uniform(-1.5, 1.5, size=3) * scale
    val, alpha, mask = O.local_solve(Q, Phi)
    bval, _ = brute(Q, Phi)
    # the exact value is a feasible objective value, and never above the grid minimum
    assert abs(objective(Q, Phi, alpha) - val) < 1e-12 * max(1, abs(val))
    assert np.all(alpha >= 0) and abs(alpha.sum() - 1) < 1e-12
    assert val <= bval + 1e-12
    lip = np.abs(Phi).max() + np.sqrt(np.linalg.eigvalsh(Q)[-1])
    assert bval - val <= 2.0 * lip / 300


@pytest.mark.parametrize("seed", range(20))
def test_local_vs_scipy(seed):
    r = rng(100 + seed)
    Q = random_face(r)
    scale = np.sqrt(np.trace(Q) / 3)
    Phi = r.uniform(-1.0, 1.0, size=3) * scale
    val, alpha, _ = O.local_solve(Q, Phi)
    best = np.inf
    for start in ([1 / 3] * 3, [0.8, 0.1, 0.1], [0.1, 0.8, 0.1], [0.1, 0.1, 0.8]):
        res = so.minimize(lambda a: objective(Q, Phi, a), np.array(start), method="SLSQP",
                          bounds=[(0, 1)] * 3,
                          constraints=[{"type": "eq", "fun": lambda a: a.sum() - 1}],
                          options=dict(ftol=1e-14, maxiter=500))
        best = min(best, res.fun)
    assert val <= best + 1e-9
    assert best - val < 1e-6 * max(1.0, abs(val))


def test_edge_path_textbook():
    """When one vertex is far earlier than the others the minimiser is that
    vertex: the value is the edge cost ||v_n - v_i||_{D^-1}."""
    r = rng(7)
    for _ in range(10):
        Q = random_face(r)
        big = 100.0 * np.sqrt(np.trace(Q))
        for n in range(3):
            Phi = np.full(3, big)
            Phi[n] = 0.25
            val, alpha, mask = O.local_solve(Q, Phi)
            assert mask == (1 << n)
            assert val == pytest.approx(0.25 + np.sqrt(Q[n, n]), rel=1e-14)


def test_equal_values_isotropic_regular():
    """Regular tet, unit metric, equal face values: the minimiser is the face
    centroid and the value is Phi + the height of the regular tet."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    E = (v[1:] - v[0]).T
    Q = E.T @ E
    val, alpha, mask = O.local_solve(Q, np.zeros(3))
    edge = np.sqrt(8.0)
    height = edge * np.sqrt(2.0 / 3.0)
    assert mask == 7
    assert np.allclose(alpha, 1 / 3, atol=1e-14)
    assert val == pytest.approx(height, rel=1e-14)


@pytest.mark.parametrize("seed", range(10))
def test_shift_equivariance(seed):
    r = rng(200 + seed)
    Q = random_face(r)
    Phi = r.uniform(-1, 1, size=3)
    v0, a0, _ = O.local_solve(Q, Phi)
    for c in (-3.7, 0.5, 125.0):
        v1, a1, _ = O.local_solve(Q, Phi + c)
        assert v1 == pytest.approx(v0 + c, rel=1e-12, abs=1e-12)
        assert np.allclose(a1, a0, atol=1e-9)


@pytest.mark.parametrize("seed", range(15))
def test_danskin_gradient(seed):
    """d value / d Phi = alpha* (envelope theorem), checked by central FD."""
    r = rng(300 + seed)
    Q = random_face(r)
    Phi = r.uniform(-0.7, 0.7, size=3) * np.sqrt(np.trace(Q) / 3)
    val, alpha, _ = O.local_solve(Q, Phi)
    h = 1e-6
    fd = np.zeros(3)
    for n in range(3):
        e = np.zeros(3)
        e[n] = h
        fd[n] = (O.local_solve(Q, Phi + e)[0] - O.local_solve(Q, Phi - e)[0]) / (2 * h)
    assert np.allclose(fd, alpha, atol=1e-6)


@pytest.mark.parametrize("seed", range(10))
def test_metric_gradient_danskin(seed):
    """d value / dQ = alpha alpha^T / (2 h) (envelope theorem), central FD on Q."""
    r = rng(400 + seed)
    Q = random_face(r)
    Phi = r.uniform(-0.5, 0.5, size=3) * np.sqrt(np.trace(Q) / 3)
    val, alpha, _ = O.local_solve(Q, Phi)
    hh = np.sqrt(alpha @ Q @ alpha)
    G = np.outer(alpha, alpha) / (2 * hh)
    dQ = random_spd(r)
    eps = 1e-6
    fd = (O.local_solve(Q + eps * dQ, Phi)[0] - O.local_solve(Q - eps * dQ, Phi)[0]) / (2 * eps)
    assert fd == pytest.approx((G * dQ).sum(), rel=1e-5, abs=1e-8)


def test_infinite_vertices():
    """Faces with unreached vertices: minimise over the finite ones only."""
    r = rng(11)
    for _ in range(10):
        Q = random_face(r)
        v, a, m = O.local_solve(Q, np.array([0.3, np.inf, np.inf]))
        assert m == 1 and v == pytest.approx(0.3 + np.sqrt(Q[0, 0]), rel=1e-14)
        Phi = np.array([0.0, 0.2, np.inf])
        v, a, m = O.local_solve(Q, Phi)
        bval, _ = brute(Q, Phi, N=600)
        assert a[2] == 0.0 and v <= bval + 1e-12 and bval - v < 1e-2
        v, a, m = O.local_solve(Q, np.full(3, np.inf))
        assert m == 0 and v == np.inf
