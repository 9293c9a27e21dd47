"""Pins of the oracle's lead weights B = K Z (Sec. 2.4): the stiffness of the
reference element in closed form, symmetry and vanishing row sums, exactness on
linear functions at interior vertices, the Dirichlet energy of a linear
function, and the vanishing lead sums of the ECG (P9)."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from conftest import rng


def test_reference_element_closed_form():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    K = O.p1_stiffness(xyz, np.array([[0, 1, 2, 3]])).toarray()
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    assert np.allclose(K, ref, atol=1e-15)
    # scaling the element by s scales K by s (|E| s^3, gradients 1/s each)
    assert np.allclose(O.p1_stiffness(2.5 * xyz, np.array([[0, 1, 2, 3]])).toarray(), 2.5 * ref)


@pytest.mark.parametrize("seed", range(2))
def test_stiffness_structure_and_linear_exactness(seed):
    xyz, tets = gi.kuhn_cube(5)
    x = gi.jitter_nodes(xyz, 0.2, 0.15, seed).astype(np.float64)
    K = O.p1_stiffness(x, tets)
    assert abs(K - K.T).max() < 1e-14
    assert np.abs(K @ np.ones(len(x))).max() < 1e-13
    c = rng(seed).normal(size=3)
    f = x @ c + 0.7
    interior = np.all((xyz > 1e-9) & (xyz < 1 - 1e-9), axis=1)
    assert np.abs((K @ f)[interior]).max() < 1e-12
    # Dirichlet energy of a linear function over the unit cube's volume
    vol = np.abs(np.linalg.det(x[tets[:, 1:]] - x[tets[:, :1]])).sum() / 6.0
    assert f @ (K @ f) == pytest.approx(c @ c * vol, rel=1e-12)


def test_lead_field_sums_and_limits():
    p = gi.cube_problem(6)
    e = gi.sphere_electrodes(np.full(3, 0.5), 3.0, 5, seed=3)
    B = O.lead_field(p.xyz, p.tets, e)
    assert np.abs(B.sum(axis=0)).max() < 1e-12 * np.abs(B).max() * len(B)
    # one electrode far away: Z is nearly constant over the mesh, B -> 0
    far = O.lead_field(p.xyz, p.tets, [[1e6, 0, 0]])
    assert np.abs(far).max() < 1e-9
