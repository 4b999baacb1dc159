"""Pins of the oracle's density scaling and inlet time function from the mathematics
rather than from a restatement of its formulas.

Dynamic similarity: the incompressible momentum equation of Section 2.1,
rho (u_t + u . grad u) = -grad p + mu div grad u, is unchanged when rho, mu and p are
multiplied by the same factor alpha with u kept (the kinematic viscosity mu/rho stays
put).  Every discrete operator of the step is linear in rho, mu and p at a fixed
velocity, so the discrete step inherits this exactly: starting from (u, alpha p) with
(alpha rho, alpha mu), u after any number of steps is the same while the pressure and
every pressure increment scale by alpha.  A pressure increment with a missing, doubled
or misplaced density (Eq. 12 of Section 2.2 prints none) breaks one of the two.

Inlet time function: the prescribed inlet velocity is the real part of
sum_k W_k exp(i k omega t) (Sections 3.2 and 4); the pin evaluates it with complex
arithmetic, and for the pulsatile cylinder checks the centreline value
1 + 0.5 sin(2 pi t) that the workload's definition states.
"""
import copy
import math

import numpy as np
import pytest

import synth
from oracle import grid, ipcs


def _scaled(case, alpha):
    c = copy.deepcopy(case)
    c.rho = case.rho * alpha
    c.mu = case.mu * alpha
    c.p0 = case.p0 * alpha
    return c


def _run(case, nsteps, **kw):
    pr = ipcs.Problem.from_case(case, **kw)
    u, p = pr.initial_state(case.u0, case.p0)
    t = 0.05
    phis, uibs = [], []
    for _ in range(nsteps):
        u, p, t, info = pr.step(u, p, t)
        phis.append(info.phi)
        uibs.append(info.u_ib)
    return u, p, phis, uibs


def _similarity(case, alpha, nsteps=2, **kw):
    u1, p1, phi1, uib1 = _run(case, nsteps, **kw)
    u2, p2, phi2, uib2 = _run(_scaled(case, alpha), nsteps, **kw)
    us = np.abs(u1).max()
    assert us > 0
    # the velocity does not see the scaling
    assert np.abs(u2 - u1).max() <= 1e-12 * us
    for a, b in zip(uib1, uib2):
        assert np.abs(b - a).max() <= 1e-12 * us
    # the pressure increment of every step and the pressure scale by alpha
    for a, b in zip(phi1, phi2):
        assert np.abs(a).max() > 1e-6 * np.abs(p1).max()     # Phi is not trivially zero
        assert np.abs(b - alpha * a).max() <= 1e-11 * alpha * np.abs(a).max()
    assert np.abs(p2 - alpha * p1).max() <= 1e-11 * alpha * np.abs(p1).max()


@pytest.mark.parametrize("seed", [1, 3])
def test_dynamic_similarity_random_blob(seed):
    """Irregular mask, random wall velocity, two-harmonic inlet, rho = 1.3."""
    _similarity(synth.random_blob_case(seed=seed), alpha=3.7)


def test_dynamic_similarity_pulsatile_cylinder():
    """Pulsatile inlet from rest: Phi != 0 from the first step on."""
    c = synth.small_cylinder(8, 16, pulsatile=True, nsteps=2)
    c.p0 = 0.05 * (2.0 - c.node_coords()[:, 2])        # a nonzero initial pressure to scale
    _similarity(c, alpha=0.37, nsteps=3)


def test_dynamic_similarity_explicit_advection_and_strain_form():
    c = synth.random_blob_case(seed=2)
    _similarity(c, alpha=5.0, advection=1)
    _similarity(c, alpha=5.0, viscous=1)


def test_dynamic_similarity_closed_box():
    """Outlet-less domain: the mean-zero projection of the pressure increment."""
    c = synth.closed_box(cells=4, seed=1)
    c.p0 = np.random.default_rng(5).standard_normal(c.N) * 0.1
    _similarity(c, alpha=2.5)


def test_dynamic_similarity_refined_lattice():
    c = synth.refined_cylinder(8, 8, length=1.25, band=0.3, nsteps=2)
    c.p0 = 0.1 * (1.25 - c.node_coords()[:, 2])
    _similarity(c, alpha=4.0)


def test_ib_force_scales_with_density_over_dt():
    """The IB correction is the same for every rho: Lambda = c F with
    c = (dt/rho) dS/h^3 (Eqs. 20-22), so u_ib - u* does not depend on rho and the
    Eulerian force density (rho/dt)(u_ib - u*) scales with rho."""
    c = synth.random_blob_case(seed=4)
    pr1 = ipcs.Problem.from_case(c)
    pr2 = ipcs.Problem.from_case(_scaled(c, 2.0))
    u, p = pr1.initial_state(c.u0, c.p0)
    _, _, _, i1 = pr1.step(u, p, 0.0)
    _, _, _, i2 = pr2.step(u, 2.0 * p, 0.0)
    d1 = i1.u_ib - i1.u_star
    d2 = i2.u_ib - i2.u_star
    assert np.abs(d1).max() > 1e-6
    assert np.abs(d2 - d1).max() <= 1e-12 * np.abs(d1).max()


def test_inlet_values_are_real_part_of_complex_harmonics():
    c = synth.random_blob_case(seed=1)
    s = grid.derive_sets(c.nx, c.ny, c.nz, c.node_mask, c.bc_tag)
    W = [c.inlet_shape[0].astype(complex)]
    for k in range(1, c.inlet_K + 1):
        W.append(c.inlet_shape[2 * k - 1] + 1j * c.inlet_shape[2 * k])
    for t in (0.0, 0.13, 0.71, 2.9):
        z = sum(W[k] * np.exp(1j * k * c.inlet_omega * t) for k in range(len(W)))
        g = grid.dirichlet_values(s, c.node_mask, c.inlet_ids, c.inlet_shape, c.inlet_K,
                                  c.inlet_omega, t)
        np.testing.assert_allclose(g[:, c.inlet_ids].T, z.real, rtol=0, atol=1e-14)
        # every other node carries zero
        rest = np.ones(c.N, bool)
        rest[c.inlet_ids] = False
        assert not g[:, rest].any()


def test_pulsatile_centreline_value():
    """The pulsatile cylinder's inlet: u_max(t) = 1 + 0.5 sin(2 pi t) on the axis."""
    c = synth.small_cylinder(8, 16, pulsatile=True)
    s = grid.derive_sets(c.nx, c.ny, c.nz, c.node_mask, c.bc_tag)
    xyz = c.node_coords()
    axis = np.nonzero((xyz[:, 0] == 0.0) & (xyz[:, 1] == 0.0) & (xyz[:, 2] == 0.0))[0]
    assert axis.size == 1
    for t in (0.0, 0.1, 0.25, 0.6, 1.35):
        g = grid.dirichlet_values(s, c.node_mask, c.inlet_ids, c.inlet_shape, c.inlet_K,
                                  c.inlet_omega, t)
        assert g[2, axis[0]] == pytest.approx(1.0 + 0.5 * math.sin(2 * math.pi * t), abs=1e-14)
        assert g[0, axis[0]] == 0.0 and g[1, axis[0]] == 0.0
