"""The aorta-like input (arch tube with three branches, Womersley-type inlet) and
one oracle step on its quarter-resolution variant.

The Womersley shapes are inputs, not part of the method, but a wrong shape would
silently change the workload, so they are pinned to their defining ODE, the wall
value, the low-frequency (Poiseuille) limit and the plug core at large alpha."""
import math

import numpy as np
import pytest

import synth
from oracle import grid, ib, ipcs


def test_womersley_shapes_pins():
    R = 1.2
    r = np.linspace(0.0, R, 4001)
    # wall value and the defining ODE W'' + W'/r = i (a/R)^2 (W - 1), a = R sqrt(w rho / mu)
    for omega, mu in ((2 * math.pi, 0.01), (2 * math.pi, 0.3)):
        W = synth.womersley_shapes(r, R, omega, 1.0, mu, (1.0, 1.0))[1]
        a = R * math.sqrt(omega / mu)
        assert abs(W[-1]) < 1e-12
        dr = r[1] - r[0]
        i = np.arange(200, 3800)
        lap = (W[i + 1] - 2 * W[i] + W[i - 1]) / dr ** 2 + (W[i + 1] - W[i - 1]) / (2 * dr * r[i])
        rhs = 1j * (a / R) ** 2 * (W[i] - 1.0)
        assert np.max(np.abs(lap - rhs)) <= 1e-4 * np.max(np.abs(rhs)) + 1e-6
    # low frequency: the shape tends to the parabola 1 - r^2/R^2 (up to a factor)
    W = synth.womersley_shapes(r, R, 1e-6, 1.0, 1.0, (1.0, 1.0))[1]
    par = 1.0 - (r / R) ** 2
    assert np.max(np.abs(W / W[0] - par)) < 1e-6
    # high frequency (a ~ 30): a plug core with W = 1 in the centre
    W = synth.womersley_shapes(r, R, 2 * math.pi, 1.0, 0.01, (1.0, 1.0))[1]
    assert abs(W[0] - 1.0) < 1e-6
    # coefficients scale the shapes; the mean shape is the parabola
    s = synth.womersley_shapes(r, R, 2 * math.pi, 1.0, 0.01, (2.0, 0.5, 0.25j))
    assert np.allclose(s[0], 2.0 * par)
    assert np.allclose(s[2], 0.25j * synth.womersley_shapes(r, R, 4 * math.pi, 1.0, 0.01, (1.0, 1.0))[1])


@pytest.fixture(scope="module")
def quarter():
    return synth.aorta_case(scale=4, spacing=1.5, nsteps=1)


def test_aorta_geometry_and_tags(quarter):
    c = quarter
    assert (c.nx, c.ny, c.nz) == (64, 40, 96) and c.h == 0.25
    frac = c.node_mask.mean()
    assert 0.03 < frac < 0.08
    tag = c.bc_tag.reshape(c.nz + 1, c.ny + 1, c.nx + 1)
    # inlet and outlet disks share the z = 0 face; the branch outlets are on z = max
    assert (tag[0] == synth.TAG_INLET).any() and (tag[0] == synth.TAG_OUTLET).any()
    assert (tag[-1] == synth.TAG_OUTLET).sum() > 0 and not (tag[-1] == synth.TAG_INLET).any()
    assert not (tag[1:-1, 1:-1, 1:-1] != 0).any()
    assert np.all(c.bc_tag[c.inlet_ids] == synth.TAG_INLET) and np.all(c.node_mask[c.inlet_ids] == 1)
    assert c.inlet_K == 2 and c.inlet_shape.shape == (5, c.inlet_ids.size, 3)
    s = grid.derive_sets(c.nx, c.ny, c.nz, c.node_mask, c.bc_tag)
    assert s.in_Du[c.inlet_ids].all()
    out = np.nonzero(c.bc_tag == synth.TAG_OUTLET)[0]
    assert np.array_equal(np.nonzero(s.p_dir)[0], out[s.in_P[out]])
    # the three branches each reach an outlet: every outlet disk holds nodes of P
    top = (c.bc_tag == synth.TAG_OUTLET) & (np.arange(c.N) >= c.nz * (c.nx + 1) * (c.ny + 1))
    assert s.in_P[top].sum() >= 3


def test_aorta_oracle_step_invariants(quarter):
    c = quarter
    pr = ipcs.Problem.from_case(c)
    u, p = pr.initial_state(c.u0, c.p0)
    u1, p1, t1, info = pr.step(u, p, 0.0)
    I = ib.interpolation_matrix(c.X, c.nx, c.ny, c.nz, c.h, c.origin)
    for d in range(3):
        assert np.abs(I @ info.u_ib[d]).max() <= 1e-12
    # prescribed inlet values at t1: Re sum_k C_k W_k e^{i k w t}
    sh = c.inlet_shape[:, :, 2]
    W = [sh[0].astype(complex)] + [sh[2 * k - 1] + 1j * sh[2 * k] for k in range(1, c.inlet_K + 1)]
    val = sum(W[k] * np.exp(1j * k * c.inlet_omega * t1) for k in range(len(W))).real
    assert np.allclose(u1[2][c.inlet_ids], val, rtol=0, atol=1e-14)
    assert np.isfinite(u1).all() and np.isfinite(p1).all()
