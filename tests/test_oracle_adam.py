"""The oracle's Adam step against torch.optim.Adam (an independent implementation)."""
import numpy as np
import torch

import oracle as O
from conftest import rng


def test_adam_matches_torch():
    r = rng(0)
    p0 = r.normal(size=20)
    p = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.5, betas=(0.9, 0.999), eps=1e-8)
    q, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for step in range(1, 8):
        g = r.normal(size=20)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        q, m, v = O.adam_step(q, g, m, v, step)
        assert np.allclose(p.detach().numpy(), q, rtol=1e-12, atol=1e-12)
