"""CPU checks of the spectral interval behind the tensor-product preconditioner of
the consistent-mass correction (Sections 2.2 and 2.4: M_FF delta = (G Phi)_F).

P = D^-1/2 T D^-1/2, T the product over the axes of the stencil (-1/4, 1, -1/4)
among the free rows (on a refined lattice: at lattice spacing among the rows
with fine cells only, at twice that spacing among the rows with coarse cells or
hanging children), D the diagonal of M_FF.  On an unbounded grid the symbol of
P M per axis is (1 + cos/2)(1 - cos/2), so the spectrum is [27/64, 1]; the
Chebyshev iteration of the library takes [0.4, 1.6] and converges for every
eigenvalue in (0, 2).  These tests compute the generalized eigenvalues on small
masked grids with dense linear algebra."""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import synth
from oracle import fem, grid, ipcs

T1 = 0.25


def _tensor(i, j, k, lat, cls=None):
    """T among the rows at lattice coordinates (i, j, k); rows of class 1 couple
    at stride 2 among themselves, rows of class 0 at stride 1."""
    n = i.size
    cls = np.zeros(n, int) if cls is None else cls
    key = {(a, b, c): r for r, (a, b, c) in enumerate(zip(i, j, k))}
    rows, cols, vals = [], [], []
    for r in range(n):
        st = 2 if cls[r] == 1 else 1
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    q = key.get((i[r] + st * dx, j[r] + st * dy, k[r] + st * dz))
                    if q is None or cls[q] != cls[r]:
                        continue
                    rows.append(r)
                    cols.append(q)
                    vals.append((-T1) ** (abs(dx) + abs(dy) + abs(dz)))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n)).toarray()


def _spectrum(M, T):
    s = 1.0 / np.sqrt(np.diag(M))
    J = s[:, None] * M * s[None, :]
    # eigenvalues of T J: the symmetric pencil (J, T^-1)
    return sl.eigh(J, np.linalg.inv(T), eigvals_only=True)


def test_symbol_of_the_product_on_a_periodic_line():
    # one axis, periodic: Jacobi-scaled mass (1/4, 1, 1/4) times (-1/4, 1, -1/4)
    n = 64
    th = 2 * np.pi * np.arange(n) / n
    m = 1 + 0.5 * np.cos(th)
    t = 1 - 2 * T1 * np.cos(th)
    lam = m * t
    assert np.isclose(lam.min(), 0.75) and np.isclose(lam.max(), 1.0)
    assert np.isclose(lam.min() ** 3, 27 / 64)


@pytest.mark.parametrize("make", [lambda: synth.closed_box(6), lambda: synth.small_cylinder(10, 20),
                                  lambda: synth.random_blob_case((9, 8, 10), seed=3),
                                  lambda: synth.channel_case()])
def test_uniform_masks_inside_the_convergence_region(make):
    c = make()
    S = grid.derive_sets(c.nx, c.ny, c.nz, c.node_mask, c.bc_tag)
    F = S.F
    M = fem._assemble(S.corners, fem.element_matrices_all(c.h)[0], S.in_P.size).tocsr()[F][:, F].toarray()
    sy = c.nx + 1
    i, j, k = F % sy, (F // sy) % (c.ny + 1), F // (sy * (c.ny + 1))
    lam = _spectrum(M, _tensor(i, j, k, None))
    assert lam.min() > 0.25 and lam.max() < 1.65
    # the bulk of the spectrum lies in the interval the iteration is designed for
    inside = np.mean((lam >= 0.4 - 1e-9) & (lam <= 1.6))
    assert inside > 0.9


def test_refined_lattice_inside_the_interval():
    from synth.aneurysm import aneurysm_case
    c = aneurysm_case(base=(16, 16, 40), band=1.2)
    pb = ipcs.Problem.from_case(c)
    m = pb.mesh
    F = pb.sets.F
    M = pb.ops.M.tocsr()[F][:, F].toarray()
    coarse = np.zeros(m.N, bool)
    coarse[m.coarse.ravel()] = True
    for par in m.parents.values():
        coarse[par] = True
    sy, sz = m.lx + 1, (m.lx + 1) * (m.ly + 1)
    i, j, k = F % sy, (F % sz) // sy, F // sz
    lam = _spectrum(M, _tensor(i, j, k, None, coarse[F].astype(int)))
    assert lam.min() > 0.35 and lam.max() < 1.6
