"""The ECG forward that allocates nothing (gbp_ecg_forward_noalloc) against the
ordinary one (gbp_ecg_forward) and the oracle, on two calls in a row (the second
smaller, so the first call's leftovers in the library's fixed scratch must not
leak into it).  Bar: ECG 1e-3 relative (max norm), as for gbp_ecg_forward; the
two entry points run the same kernels, so they agree to FP32 reassociation of
the window sums."""
import numpy as np
import pytest

import oracle as O
from test_gpu_parity import B, _dev, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_ecg_matches_ecg_forward():
    dev = _dev()
    r = np.random.Generator(np.random.PCG64(77))
    cases = ((20_000, 31, 1500, 0.09), (3_000, 5, 77, 0.7))   # the second call is smaller
    for n_v, L, S, dt in cases:
        print(f"[case] noalloc ECG n_v={n_v} L={L} S={S}", flush=True)
        T = r.uniform(0.0, 120.0, size=n_v)
        T[::53] = np.inf
        W = r.normal(size=(n_v, L)).astype(np.float32)
        ap = dict(K0=-85.0, K1=30.0, tau=1.0, t0=-3.0, dt=dt, n_steps=S)
        Td, Wd, apd = t32(T, dev), t32(W, dev), B().make_ap(**ap)
        out = torch.full((S, L), float("nan"), dtype=torch.float32, device=dev)
        e_na = B().ecg_forward_noalloc(Td, Wd, apd, out).cpu().numpy()
        e = B().ecg_forward(Td, Wd, apd).cpu().numpy()
        eo = O.ecg_forward(T.astype(np.float32), W, ap)
        scale = np.abs(eo).max()
        assert np.all(np.isfinite(e_na))
        assert np.abs(e_na - e).max() <= 1e-5 * np.abs(e).max(), (n_v, L, S)
        assert np.abs(e_na - eo).max() <= 1e-3 * scale, (n_v, L, S)
    with pytest.raises(B().GbpError):
        B().ecg_forward_noalloc(Td, t32(np.zeros((3_000, 257)), dev), apd,
                                torch.empty((77, 257), device=dev))
