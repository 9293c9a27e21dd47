"""Pins of the FP64 warm-start network reference against library routines
(torch.nn layers, autograd), central differences and hand-computed feature
rows."""
import numpy as np
import pytest

import gbp_inputs as gi
from oracle import mlp as M

torch = pytest.importorskip("torch")


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(11))


def _torch_net(params):
    P = M.unpack(params)
    layers = []
    for l in range(1, 5):
        lin = torch.nn.Linear(P[f"W{l}"].shape[1], 256).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(P[f"W{l}"]))
            lin.bias.copy_(torch.from_numpy(P[f"b{l}"]))
        layers += [lin, torch.nn.ReLU()]
    head = torch.nn.Linear(256, 1).double()
    with torch.no_grad():
        head.weight.copy_(torch.from_numpy(P["w5"][None, :]))
        head.bias.copy_(torch.from_numpy(P["b5"]))
    return torch.nn.Sequential(*layers, head)


def test_layout_matches_generator():
    assert M.N_PARAMS == sum(int(np.prod(s)) for _, s in gi.MLP_SIZES)
    assert M.N_PARAMS == 256 * 16 + 3 * 256 * 256 + 4 * 256 + 256 + 1


def test_forward_equals_torch_layers(rng):
    p = gi.mlp_params(3)
    X = rng.normal(size=(300, 16))
    y = M.forward(p, X)
    with torch.no_grad():
        yt = _torch_net(p)(torch.from_numpy(X)).numpy()[:, 0]
    np.testing.assert_allclose(y, yt, rtol=1e-12, atol=1e-12)


def test_gradient_equals_autograd(rng):
    p = gi.mlp_params(4)
    X = rng.normal(size=(200, 16))
    t = rng.normal(size=200)
    loss, g = M.loss_and_gradient(p, X, t)
    net = _torch_net(p)
    lt = ((net(torch.from_numpy(X))[:, 0] - torch.from_numpy(t)) ** 2).mean()
    lt.backward()
    P = {}
    for l, k in zip(range(1, 5), (0, 2, 4, 6)):
        P[f"W{l}"] = net[k].weight.grad.numpy()
        P[f"b{l}"] = net[k].bias.grad.numpy()
    P["w5"] = net[8].weight.grad.numpy()[0]
    P["b5"] = net[8].bias.grad.numpy()
    assert loss == pytest.approx(float(lt.detach()), rel=1e-12)
    np.testing.assert_allclose(g, M.pack(P), rtol=1e-10, atol=1e-13)


def test_gradient_central_differences(rng):
    p = gi.mlp_params(5).astype(np.float64)
    X = rng.normal(size=(64, 16))
    t = rng.normal(size=64)
    _, g = M.loss_and_gradient(p, X, t)
    idx = rng.choice(M.N_PARAMS, size=40, replace=False)
    idx = np.concatenate([idx, [0, 256 * 16, M.N_PARAMS - 1, M.N_PARAMS - 2]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss_and_gradient(p + e, X, t)[0]
              - M.loss_and_gradient(p - e, X, t)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i


def test_features_by_hand():
    xyz = np.array([[1.0, 2.0, 2.0], [0.0, 0.0, 0.0], [4.0, 0.0, 0.0]])
    fib = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    vs = np.array([1.5, 0.5, 2.0])
    root_xyz = np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0]])
    root_t = np.array([0.0, 2.0])
    norm = (1.0, 0.0, 0.0, 2.0, 4.0)        # centre (1,0,0), len 2, time 4
    T = np.array([8.0, 0.0, 2.0])
    X, tgt = M.features(xyz, fib, vs, None, root_xyz, root_t, norm, T=T)
    # vertex 0: |x - r0| = 3, |x - r1| = sqrt(9+4+4) = sqrt(17)
    a0, a1 = 3 / 2 + 0 / 4, np.sqrt(17) / 2 + 2 / 4
    np.testing.assert_allclose(X[0, 0:3], [0.0, 1.0, 1.0])
    np.testing.assert_allclose(X[0, 3:6], [1.0, 0.0, 0.0])
    np.testing.assert_allclose(X[0, 6:14], sorted([a0, a1] + [a0] * 6))
    assert X[0, 14] == 1.5 and X[0, 15] == 0.0
    # vertex 1 sits on root 0: feature 0 (t=0), root 1 at distance 4 -> 2 + 0.5
    np.testing.assert_allclose(X[1, 6:14], [0.0] * 7 + [2.5])
    np.testing.assert_allclose(tgt, T / 4.0)
    # the root order does not matter
    X2 = M.features(xyz, fib, vs, None, root_xyz[::-1], root_t[::-1], norm)
    X3 = M.features(xyz, fib, vs, None, np.repeat(root_xyz, [7, 1], axis=0),
                    np.repeat(root_t, [7, 1]), norm)
    assert not np.array_equal(X2, X)        # padding repeats a different root 0
    np.testing.assert_allclose(X3, X)
