"""Pins for the oracle's immersed-boundary pieces: the four-point kernel of Eq. 18,
the interpolation of Eq. 17, and the BCE correction of Eqs. 20-24."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import grid, ib


def test_kernel_special_values_and_moments():
    assert ib.delta4(0.0) == pytest.approx(0.5, abs=1e-16)
    assert ib.delta4(1.0) == pytest.approx(0.25, abs=1e-16)
    assert ib.delta4(2.0) == 0.0
    assert ib.delta4(2.5) == 0.0
    # continuity at |r| = 1 from both branches
    assert ib.delta4(1.0 - 1e-12) == pytest.approx(ib.delta4(1.0 + 1e-12), abs=1e-11)
    rng = np.random.default_rng(0)
    for r in rng.random(50) * 4 - 2:
        j = np.arange(-4, 5)
        d = ib.delta4(r - j)
        assert d.sum() == pytest.approx(1.0, abs=1e-14)                   # partition of unity
        assert d[j % 2 == 0].sum() == pytest.approx(0.5, abs=1e-14)       # even/odd halves
        assert ((r - j) * d).sum() == pytest.approx(0.0, abs=1e-14)       # first moment
        assert (d ** 2).sum() == pytest.approx(3.0 / 8.0, abs=1e-14)      # sum of squares
        assert ib.delta4(-r) == pytest.approx(ib.delta4(r), abs=1e-16)    # even


def test_interpolation_reproduces_linear_fields():
    nx, ny, nz, h = 9, 8, 10, 0.2
    origin = np.array([0.1, -0.3, 0.25])
    rng = np.random.default_rng(1)
    X = origin + h * (2.0 + rng.random((20, 3)) * (np.array([nx, ny, nz]) - 4.0))
    I = ib.interpolation_matrix(X, nx, ny, nz, h, origin)
    i, j, k = grid.node_index_arrays(nx, ny, nz)
    xyz = origin[:, None] + h * np.stack([i, j, k]).astype(np.float64)
    assert np.allclose(I @ np.ones(i.size), 1.0, atol=1e-14)
    coef = np.array([0.4, -1.7, 2.2])
    np.testing.assert_allclose(I @ (coef @ xyz), X @ coef, atol=1e-12)
    assert np.all(np.diff(I.indptr) <= 64)


def _tiny_problem(seed=2):
    c = synth.random_blob_case(seed=seed)
    s = grid.derive_sets(c.nx, c.ny, c.nz, c.node_mask, None)
    I = ib.interpolation_matrix(c.X, c.nx, c.ny, c.nz, c.h, c.origin)
    return c, s, I


def test_bce_constraint_and_minimum_norm():
    c, s, I = _tiny_problem()
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3, c.N)) * s.in_P
    u_ib, lam, _ = ib.bce_correction(I, s.in_F, c.U_B, u)
    # the constraint of Eq. 15/20 holds for the corrected field
    for d in range(3):
        assert np.abs(I @ u_ib[d] - c.U_B[:, d]).max() < 1e-12
    # only free nodes move
    assert np.abs((u_ib - u)[:, ~s.in_F]).max() == 0.0
    # the correction is the minimum-norm one (brute force with a pseudo-inverse)
    IF = (I @ sp.diags(s.in_F.astype(float))).toarray()
    for d in range(3):
        b = c.U_B[:, d] - I @ u[d]
        du = np.linalg.pinv(IF) @ b
        np.testing.assert_allclose(u_ib[d] - u[d], du, atol=1e-11)


def test_bce_iterative_path_matches_direct():
    c, s, I = _tiny_problem(seed=4)
    rng = np.random.default_rng(6)
    u = rng.standard_normal((3, c.N)) * s.in_P
    a, _, _ = ib.bce_correction(I, s.in_F, c.U_B, u, direct_max=2000)
    b, _, info = ib.bce_correction(I, s.in_F, c.U_B, u, direct_max=0)
    assert info["method"] == "cg"
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_singular_point_detected():
    c, s, I = _tiny_problem()
    none_free = np.zeros_like(s.in_F)
    with pytest.raises(ib.SingularIB):
        ib.bce_correction(I, none_free, c.U_B, np.zeros((3, c.N)))
