"""Learned warm start: the bf16 matrix-core network kernels (features, forward,
gradient, Adam step) against the FP64 reference that rounds to bf16 at the same
points, and the warm-started solve against the oracle's cold solution.

Tolerances.  Both sides round the same quantities to bf16, but the library
accumulates in fp32 (relative error about 1e-6) and the reference in fp64, so a
value that lies within that distance of a bf16 rounding boundary can round to
neighbouring bf16 numbers on the two sides (probability ~1e-6 / 2^-8 per
element).  A flip moves one hidden activation by one bf16 ulp (2^-8 relative),
which moves the output by about 2^-8 / 16 of its size; features may differ by
one bf16 ulp.  Bars: features within one bf16 ulp elementwise, outputs 1e-3
(relative L2) and 5e-3 (max, relative to max |y|), gradients 5e-3 (relative L2
per parameter block)."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from oracle import mlp as M
from test_gpu_parity import B, _dev, i32, rel_l2, rel_max, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def bits_to_f64(X):
    b = X.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def blocks(v):
    out, o = {}, 0
    for name, shape in M.SIZES:
        n = int(np.prod(shape))
        out[name] = v[o:o + n]
        o += n
    return out


@pytest.fixture(scope="module")
def shell():
    return gi.shell_problem(6_000, seed=41, n_roots=5, vscale_range=(0.6, 1.4))


def _norm(p):
    c = 0.5 * (p.xyz.min(0) + p.xyz.max(0))
    L = float(np.linalg.norm(p.xyz - c, axis=1).max())
    return (float(c[0]), float(c[1]), float(c[2]), L, L / 0.6)


def test_features_match_oracle(shell):
    dev = _dev()
    p = shell
    norm = _norm(p)
    nf = p.extra["node_fibre"]
    r = np.random.Generator(np.random.PCG64(5))
    rows = r.integers(0, p.n_v, size=3001).astype(np.int32)
    rows[-1] = p.n_v                          # an invalid id: zero row, NaN target
    T = r.uniform(0, 100, size=p.n_v).astype(np.float32)
    rx = p.xyz[p.root_node]
    X, tg = B().mlp_features(t32(p.xyz, dev), t32(nf, dev), t32(rx, dev), t32(p.root_t, dev), norm,
                             vscale=t32(p.vscale, dev), rows=i32(rows, dev), T=t32(T, dev))
    Xo, to = M.features(p.xyz, nf, p.vscale, rows[:-1], rx, p.root_t, norm, T=T)
    Xg = bits_to_f64(X)
    assert np.all(Xg[-1] == 0) and np.isnan(tg[-1].item())
    assert np.all(np.abs(Xg[:-1] - Xo) <= 2.0 ** -7 * np.abs(Xo))
    np.testing.assert_allclose(tg[:-1].cpu().numpy(), to, rtol=1e-6)
    # all rows, no vscale (ones), a single root
    X1 = B().mlp_features(t32(p.xyz, dev), t32(nf, dev), t32(rx[:1], dev), t32(p.root_t[:1], dev), norm)
    Xo1 = M.features(p.xyz, nf, None, None, rx[:1], p.root_t[:1], norm)
    assert np.all(np.abs(bits_to_f64(X1) - Xo1) <= 2.0 ** -7 * np.abs(Xo1))


@pytest.mark.parametrize("m", [1, 63, 3000])
def test_forward_matches_oracle(m):
    _dev()
    params = gi.mlp_params(7)
    bits, vals = gi.mlp_rows(m, seed=m)
    net = B().MLP(4096, seed=0)
    net.set_params(params)
    Xd = torch.as_tensor(bits, device="cuda")
    y = net.forward(Xd).cpu().numpy()
    yo = M.forward(params, vals)
    assert rel_l2(y, yo) <= 1e-3
    assert np.abs(y - yo).max() <= 5e-3 * np.abs(yo).max()
    y2 = net.forward(Xd, out_scale=2.5).cpu().numpy()
    np.testing.assert_allclose(y2, 2.5 * y, rtol=1e-6)
    assert np.array_equal(net.get_params(), params)


@pytest.mark.parametrize("m", [700, 5000])
def test_gradient_matches_oracle(m):
    _dev()
    params = gi.mlp_params(8)
    bits, vals = gi.mlp_rows(m, seed=100 + m)
    r = np.random.Generator(np.random.PCG64(m))
    t = r.normal(size=m).astype(np.float32)
    net = B().MLP(8192, seed=0)
    net.set_params(params)
    loss = net.gradient(torch.as_tensor(bits, device="cuda"), t32(t, "cuda"))
    _, g = net.get_params(grads=True)
    lo, go = M.loss_and_gradient(params, vals, t)
    assert float(loss) == pytest.approx(lo, rel=1e-4)
    gb, gob = blocks(g), blocks(go)
    for name, _ in M.SIZES:
        assert rel_l2(gb[name], gob[name]) <= 5e-3, name
    assert np.all(gb["W1"].reshape(256, 16)[:, 15] == 0)


def test_train_step_is_adam_on_the_gradient():
    _dev()
    params = gi.mlp_params(9)
    bits, vals = gi.mlp_rows(2000, seed=9)
    t = np.random.Generator(np.random.PCG64(9)).normal(size=2000).astype(np.float32)
    net = B().MLP(2048, seed=0)
    net.set_params(params)
    lr = 1e-3
    loss = torch.empty(1, device="cuda")
    net.train_step(torch.as_tensor(bits, device="cuda"), t32(t, "cuda"), lr, loss=loss)
    p1 = net.get_params()
    _, go = M.loss_and_gradient(params, vals, t)
    dp = p1.astype(np.float64) - params.astype(np.float64)
    # first Adam step: m_hat = g, v_hat = g^2, so the update is -lr g / (|g| + 1e-8)
    for name, sl in blocks(np.arange(M.N_PARAMS)).items():
        g = go[sl]
        big = np.abs(g) > max(1e-2 * np.sqrt(np.mean(g * g)), 1e-6)
        assert big.sum() > 0.5 * len(g) or name == "W1", name
        np.testing.assert_allclose(dp[sl][big], -lr * np.sign(g[big]), atol=0.02 * lr, err_msg=name)
    assert np.all(dp[:4096].reshape(256, 16)[:, 15] == 0)
    assert float(loss) == pytest.approx(M.loss_and_gradient(params, vals, t)[0], rel=1e-4)


def test_bad_sizes_rejected():
    _dev()
    net = B().MLP(100, seed=0)
    bits, _ = gi.mlp_rows(101, seed=1)
    with pytest.raises(B().GbpError):
        net.forward(torch.as_tensor(bits, device="cuda"))


def test_training_reduces_loss_and_warm_start_equals_cold():
    dev = _dev()
    from paper_2308_08410_amd import warmstart as WS
    p = gi.shell_problem(12_000, seed=43)
    plan = B().Plan(p.xyz, p.tets)
    D = t32(p.D, dev)
    data = WS.make_dataset(plan, p.xyz, D, p.extra["endo"], 24, seed=17)
    ws = WS.WarmStart(p.xyz, p.extra["node_fibre"], max_rows=8192, seed=1)
    hist = WS.train(ws, data, 400, batch=4096, lr=2e-3, log_every=50)
    first = np.mean([h[1] for h in hist[:1]])
    last = np.mean([h[1] for h in hist[-2:]])
    assert np.isfinite(last) and last < 0.25 * first, hist
    # held-out case: the warm solve from the network's guess is the cold solution
    rn, rt, vs = WS.random_case(p.xyz, p.extra["endo"], seed=999_001)
    To, _ = O.solve(p.xyz, p.tets, p.D, vs, rn, rt)
    case = dict(root_node=i32(rn, dev), root_t=t32(rt, dev), vscale=t32(vs, dev))
    T, st = ws.forward(plan, D, case["vscale"], case["root_node"], case["root_t"])
    assert rel_max(T.cpu().numpy(), To) <= 1e-4
    guess = ws.predict(case["root_node"], case["root_t"], case["vscale"]).cpu().numpy()
    fin = np.isfinite(To)
    err_mlp = np.linalg.norm(guess[fin] - To[fin]) / np.linalg.norm(To[fin])
    assert err_mlp < 0.5, err_mlp
    rows = WS.evaluate(ws, plan, D, [dict(case, T=None)], repeats=1)
    print("warm start:", rows[0])
    assert rows[0]["warm_vs_cold_rel_max"]["mlp"] <= 1e-4
    assert rows[0]["warm_vs_cold_rel_max"]["geo"] <= 1e-4
