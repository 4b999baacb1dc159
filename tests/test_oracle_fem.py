"""Pins for the oracle's Q1 forms: closed-form tensor products, the interior
assembled stencils, and invariants that any correct assembly satisfies."""
import numpy as np
import pytest

import synth
from oracle import fem, grid

H = 0.37


def _kron3(z, y, x):
    # local corner a = ax + 2 ay + 4 az  ->  z slowest
    return np.kron(z, np.kron(y, x))


def _one_d(h):
    M1 = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    K1 = 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])
    D1 = 0.5 * np.array([[-1.0, 1.0], [-1.0, 1.0]])          # int phi_i phi_j'
    return M1, K1, D1


def test_element_matrices_match_tensor_products():
    Me, Ke, Ge, Ce = fem.element_matrices(H)
    M1, K1, D1 = _one_d(H)
    np.testing.assert_allclose(Me, _kron3(M1, M1, M1), rtol=1e-13, atol=1e-16)
    Kc = _kron3(M1, M1, K1) + _kron3(M1, K1, M1) + _kron3(K1, M1, M1)
    np.testing.assert_allclose(Ke, Kc, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Ge[0], _kron3(M1, M1, D1), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(Ge[1], _kron3(M1, D1, M1), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(Ge[2], _kron3(D1, M1, M1), rtol=1e-13, atol=1e-16)
    # advection with a constant field a reduces to sum_d a_d G_d
    a = np.array([0.3, -1.1, 0.7])
    Ca = np.einsum("cd,icdb->ib", np.tile(a, (8, 1)), Ce)
    np.testing.assert_allclose(Ca, a[0] * Ge[0] + a[1] * Ge[1] + a[2] * Ge[2], atol=1e-15)


def _full_box(n=4, h=H):
    mask = np.ones((n + 1) ** 3, np.uint8)
    sets = grid.derive_sets(n, n, n, mask, None)
    return sets, fem.Operators(sets, h)


def test_interior_stencils():
    n = 4
    sets, ops = _full_box(n)
    c = 2 + (n + 1) * (2 + (n + 1) * 2)        # centre node (2,2,2)
    h = H
    Kexp = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}
    Mexp = {0: 8 * h ** 3 / 27, 1: 2 * h ** 3 / 27, 2: h ** 3 / 54, 3: h ** 3 / 216}
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                j = c + dx + (n + 1) * (dy + (n + 1) * dz)
                kind = abs(dx) + abs(dy) + abs(dz)
                assert ops.K[c, j] == pytest.approx(Kexp[kind], abs=1e-14)
                assert ops.M[c, j] == pytest.approx(Mexp[kind], rel=1e-13)
    assert ops.K[c].nnz <= 27


def test_invariants_on_masked_grid():
    case = synth.small_cylinder(8, 16)
    sets = grid.derive_sets(case.nx, case.ny, case.nz, case.node_mask, None)
    ops = fem.Operators(sets, case.h)
    one = sets.in_P.astype(np.float64)
    # symmetry and Neumann null space of the stiffness
    assert abs(ops.K - ops.K.T).max() < 1e-15
    assert np.abs(ops.K @ one).max() < 1e-14
    # total mass = kept volume
    assert one @ (ops.M @ one) == pytest.approx(sets.corners.shape[0] * case.h ** 3, rel=1e-13)
    # gradients annihilate constants; advection annihilates constants
    for d in range(3):
        assert np.abs(ops.G[d] @ one).max() < 1e-15
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, one.size)) * one
    C = ops.advection(a)
    assert np.abs(C @ one).max() < 1e-14


def test_linear_fields_give_mass_weighted_constants():
    """G_d x = (d_d x) M 1 and C(a) x = (a . grad x) M 1 for a constant a and a
    linear x (exact on every row, boundary rows included)."""
    n = 4
    sets, ops = _full_box(n)
    i, j, k = grid.node_index_arrays(n, n, n)
    xyz = np.stack([i, j, k]).astype(np.float64) * H
    slope = np.array([0.7, -0.2, 1.3])
    x = slope @ xyz
    M1 = ops.M @ np.ones(x.size)
    for d in range(3):
        np.testing.assert_allclose(ops.G[d] @ x, slope[d] * M1, atol=1e-14)
    a = np.array([1.5, 0.25, -0.5])
    C = ops.advection(np.tile(a[:, None], (1, x.size)))
    np.testing.assert_allclose(C @ x, (a @ slope) * M1, atol=1e-14)


def test_stiffness_annihilates_trilinear_on_interior_rows():
    n = 5
    sets, ops = _full_box(n)
    i, j, k = grid.node_index_arrays(n, n, n)
    x, y, z = i * H, j * H, k * H
    f = 0.3 + x - 2 * y + 0.5 * z + x * y - 3 * y * z + 2 * x * z + 4 * x * y * z
    interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
    assert np.abs((ops.K @ f)[interior]).max() < 1e-12


def test_divergence_theorem_on_box():
    """1^T B u = boundary flux of the Q1 interpolant (bilinear face quadrature)."""
    n = 3
    sets, ops = _full_box(n)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3, (n + 1) ** 3))
    total = np.sum(ops.divergence(u))
    U = u.reshape(3, n + 1, n + 1, n + 1)       # [comp, k, j, i]

    def face_integral(f2d):                       # bilinear on an (n+1)x(n+1) face grid
        return H * H / 4.0 * (f2d[:-1, :-1] + f2d[1:, :-1] + f2d[:-1, 1:] + f2d[1:, 1:]).sum()

    flux = (face_integral(U[0, :, :, -1]) - face_integral(U[0, :, :, 0])
            + face_integral(U[1, :, -1, :]) - face_integral(U[1, :, 0, :])
            + face_integral(U[2, -1, :, :]) - face_integral(U[2, 0, :, :]))
    assert total == pytest.approx(flux, rel=1e-12, abs=1e-13)


def test_default_tags_and_sets_small():
    """Hand-checked sets on a 2x1x2 grid with one in-vessel node."""
    nx, ny, nz = 2, 1, 2
    N = 3 * 2 * 3
    mask = np.zeros(N, np.uint8)
    centre = 1 + 3 * (0 + 2 * 1)               # node (1,0,1): on the y = 0 face
    mask[centre] = 1
    s = grid.derive_sets(nx, ny, nz, mask, None)
    assert s.kept_cells.sum() == 4              # every cell touches (1,0,1)
    assert s.P.size == N
    assert s.F.size == 0                        # the only m = 1 node lies on a wall face
    tag = grid.default_tags(nx, ny, nz)
    assert tag[1 + 3 * (0 + 2 * 0)] == grid.TAG_WALL   # edge node: wall wins
    assert (s.p_dir == (tag == grid.TAG_OUTLET)).all()
