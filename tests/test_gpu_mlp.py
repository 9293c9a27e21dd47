"""Learned warm start: the bf16 matrix-core network kernels (features, forward,
gradient, Adam step) against the exact FP64 network of ``oracle/mlp.py``, and the
warm-started solve against the oracle's cold solution.

Bounds, from the rounding unit of bf16 (8 significant bits, u = 2^-8: a rounded
value is x (1 + delta) with |delta| <= u).  The library stores the features, the
hidden weights, the hidden activations and the back-propagated dZ in bf16 and
accumulates in fp32 (2^-24, negligible beside u).
* Features: one rounding of a value computed in fp32, so |X - X64| <= u |X64|
  plus fp32 error (1e-6 absolute for the centred coordinates).
* Forward: the standard probabilistic model of rounding error (independent,
  mean-zero delta; variance at most u^2 for any distribution on [-u, u]) and a
  first-order expansion give, per output, Var(y - y64) <= u^2 sum over rounding
  events of (dy/d(value) * value)^2, with the sensitivities dy/dZ_l, dy/dH_l of
  the FP64 network itself.  Each output must lie within 6 such standard
  deviations.
* Gradients: the same model sampled (16 draws of delta ~ U[-u, u] at every
  rounding point of the FP64 network, ``oracle.mlp``'s ``perturb``) gives the
  spread of the gradient under bf16 storage; each parameter block's relative L2
  error must stay within 3 times the sampled root-mean-square error (the
  uniform draws have twice the variance of round-to-nearest errors)."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from oracle import mlp as M
from test_gpu_parity import B, _dev, i32, rel_l2, rel_max, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


U_BF16 = 2.0 ** -8


def forward_sigma(params, X):
    """Per-row standard deviation bound of the bf16 forward's error (first order,
    independent rounding errors of variance <= u^2): weight rounding of W_l
    (each product W_jk H_k), activation rounding of H_1..H_4."""
    y, zs, hs = M.forward(params, X, cache=True)
    P = M.unpack(params)
    var = ((P["w5"][None, :] * hs[4]) ** 2).sum(1)          # rounding of H4
    s = P["w5"][None, :] * (zs[3] > 0)                        # dy/dZ4
    for l in range(4, 0, -1):
        W = P[f"W{l}"]
        var += (s ** 2 * ((hs[l - 1] ** 2) @ (W ** 2).T)).sum(1)   # rounding of W_l
        if l > 1:
            g = s @ W                                        # dy/dH_{l-1}
            var += ((g * hs[l - 1]) ** 2).sum(1)              # rounding of H_{l-1}
            s = g * (zs[l - 2] > 0)
    return y, U_BF16 * np.sqrt(var)


def gradient_spread(params, X, t, draws=16, seed=0):
    """Root-mean-square error of the FP64 gradient under the rounding model
    (delta ~ U[-u, u] wherever the library stores bf16), per element."""
    r = np.random.Generator(np.random.PCG64(seed))
    _, g64 = M.loss_and_gradient(params, X, t)
    acc = np.zeros_like(g64)

    def perturb(name, a):
        return a * (1.0 + r.uniform(-U_BF16, U_BF16, size=a.shape))

    for _ in range(draws):
        _, gk = M.loss_and_gradient(params, X, t, perturb=perturb)
        acc += (gk - g64) ** 2
    return g64, np.sqrt(acc / draws)


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
    assert np.all(np.abs(Xg[:-1] - Xo) <= U_BF16 * np.abs(Xo) + 1e-6)
    np.testing.assert_allclose(tg[:-1].cpu().numpy(), to, rtol=1e-6)
    # all rows, no vscale (ones), a single root
    X1 = B().mlp_features(t32(p.xyz, dev), t32(nf, dev), t32(rx[:1], dev), t32(p.root_t[:1], dev), norm)
    Xo1 = M.features(p.xyz, nf, None, None, rx[:1], p.root_t[:1], norm)
    assert np.all(np.abs(bits_to_f64(X1) - Xo1) <= U_BF16 * np.abs(Xo1) + 1e-6)


@pytest.mark.parametrize("m", [1, 63, 3000, 4096, 40_000, 70_000])
def test_forward_matches_oracle(m):
    """Every row tiling of the inference kernel (32 rows per block below 16384 rows,
    64 below 65536, 128 above), ragged tails included."""
    _dev()
    params = gi.mlp_params(7)
    bits, vals = gi.mlp_rows(m, seed=m)
    net = B().MLP(max(m, 4096), seed=0)
    net.set_params(params)
    Xd = torch.as_tensor(bits, device="cuda")
    y = net.forward(Xd).cpu().numpy()
    yo, sig = forward_sigma(params, vals)
    ratio = np.abs(y - yo) / (sig + 1e-6 * np.abs(yo))
    print(f"[mlp forward] m={m} rel L2 err {rel_l2(y, yo):.2e}, max |err|/sigma {ratio.max():.2f}",
          flush=True)
    assert ratio.max() <= 6.0
    y2 = net.forward(Xd, out_scale=2.5).cpu().numpy()
    np.testing.assert_allclose(y2, 2.5 * y, rtol=1e-6)
    assert np.array_equal(net.get_params(), params)


@pytest.mark.parametrize("m", [700, 40_000, 66_000])
def test_gradient_matches_oracle(m):
    """Every row tiling of the fused forward and backward (32, 64 and 128 rows per
    block), ragged tails, one to many weight-gradient splits; the gradient is
    bitwise repeatable."""
    _dev()
    params = gi.mlp_params(8)
    bits, vals = gi.mlp_rows(m, seed=100 + m)
    r = np.random.Generator(np.random.PCG64(m))
    t = r.normal(size=m).astype(np.float32)
    net = B().MLP(max(m, 8192), seed=0)
    net.set_params(params)
    Xd, td = torch.as_tensor(bits, device="cuda"), t32(t, "cuda")
    loss = net.gradient(Xd, td)
    _, g = net.get_params(grads=True)
    loss2 = net.gradient(Xd, td)
    _, g2 = net.get_params(grads=True)
    assert np.array_equal(g, g2) and float(loss) == float(loss2)
    lo, _, c = M.loss_and_gradient(params, vals, t, cache=True)
    _, sig = forward_sigma(params, vals)
    # loss = mean (y - t)^2 moves by at most 2 rms(y - t) rms(dy) (Cauchy-Schwarz)
    dl = 2.0 * np.sqrt(lo) * np.sqrt(np.mean((6.0 * sig) ** 2))
    assert abs(float(loss) - lo) <= dl + 1e-6 * lo
    go, spread = gradient_spread(params, vals, t)
    gb, gob, sb = blocks(g), blocks(go), blocks(spread)
    for name, _ in M.SIZES:
        err = rel_l2(gb[name], gob[name])
        bar = 3.0 * np.linalg.norm(sb[name]) / np.linalg.norm(gob[name])
        print(f"[mlp gradient] m={m} {name}: rel L2 err {err:.2e}, bar {bar:.2e}", flush=True)
        assert err <= bar + 1e-6, name
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
    go, spread = gradient_spread(params, vals, t)
    dp = p1.astype(np.float64) - params.astype(np.float64)
    # first Adam step: m_hat = g, v_hat = g^2, so the update is -lr g / (|g| + 1e-8); the
    # device's gradient has the FP64 sign wherever |g| is far outside its rounding spread
    # (per element, and at least the block's RMS spread, since 16 draws estimate a single
    # element's spread loosely).  A ReLU mask that flips where a pre-activation lies within
    # rounding of zero moves a row's contribution discretely, so a few elements in 10^4
    # may still differ.
    for name, sl in blocks(np.arange(M.N_PARAMS)).items():
        g = go[sl]
        sp = np.maximum(spread[sl], np.sqrt(np.mean(spread[sl] ** 2)))
        big = (np.abs(g) > 12.0 * sp) & (np.abs(g) > 1e-6)
        assert big.sum() > 0.25 * len(g) or name == "W1", (name, big.sum())
        ok = np.abs(dp[sl][big] + lr * np.sign(g[big])) <= 0.02 * lr
        assert np.sum(~ok) <= max(1, 1e-4 * big.sum()), (name, int(np.sum(~ok)), int(big.sum()))
    assert np.all(dp[:4096].reshape(256, 16)[:, 15] == 0)
    lo = M.loss_and_gradient(params, vals, t)[0]
    _, sig = forward_sigma(params, vals)
    assert abs(float(loss) - lo) <= 2.0 * np.sqrt(lo) * np.sqrt(np.mean((6.0 * sig) ** 2)) + 1e-6 * lo


def test_bad_sizes_rejected():
    """Training batches are bounded by max_rows; inference, which keeps nothing per
    row on the device, is not."""
    _dev()
    net = B().MLP(100, seed=0)
    bits, _ = gi.mlp_rows(101, seed=1)
    Xd = torch.as_tensor(bits, device="cuda")
    with pytest.raises(B().GbpError):
        net.gradient(Xd, torch.zeros(101, device="cuda"))
    y = net.forward(Xd)
    assert torch.equal(y[:100], net.forward(Xd[:100].contiguous()))
    # the inference kernel reads feature rows in 16-byte pieces: a misaligned X is refused
    flat = torch.as_tensor(bits, device="cuda").reshape(-1)
    shifted = torch.empty(flat.numel() + 8, dtype=flat.dtype, device="cuda")
    view = shifted[1:1 + 50 * 16].view(50, 16)
    view.copy_(flat[:50 * 16].view(50, 16))
    with pytest.raises(B().GbpError, match="aligned"):
        net.forward(view)


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


def test_training_resumes_from_checkpoint(tmp_path):
    """Training stopped half-way through its schedule (checkpoint written) and
    resumed by a new network object follows the uninterrupted run exactly: the
    same row batches from the restored generator, the same Adam state, and
    deterministic kernels, so the parameters and moments are bitwise equal."""
    _dev()
    from paper_2308_08410_amd import warmstart as WS
    p = gi.shell_problem(6_000, seed=11)
    plan = B().Plan(p.xyz, p.tets)
    D = torch.as_tensor(p.D, device="cuda")
    data = WS.make_dataset(plan, p.xyz, D, p.extra["endo"], 3, seed=77)
    ck = str(tmp_path / "train.npz")
    net = lambda seed: WS.WarmStart(p.xyz, p.extra["node_fibre"], max_rows=4096, seed=seed)
    full = net(4)
    h_full = WS.train(full, data, 24, batch=2048, log_every=4, seed=9)
    part = net(4)
    WS.train(part, data, 24, batch=2048, log_every=4, seed=9, checkpoint=ck, stop=12)
    assert part.mlp.get_state()["step"] == 12
    resumed = net(123)                      # initial weights replaced by the checkpoint's
    h_res = WS.train(resumed, data, 24, batch=2048, log_every=4, seed=9, checkpoint=ck, resume=True)
    assert np.array_equal(resumed.mlp.get_params(), full.mlp.get_params())
    a, b = resumed.mlp.get_state(), full.mlp.get_state()
    assert a["step"] == b["step"] == 24
    assert np.array_equal(a["m"], b["m"]) and np.array_equal(a["v"], b["v"])
    assert h_res == h_full
