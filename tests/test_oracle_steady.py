"""Pins of the steady-state test and the exact solution of the pressure-driven
Poiseuille experiment (Section 3.1) in the oracle, and of its inputs: the NRMSE
formula on hand-computed values and its invariances, the exact profile against the
momentum balance (finite differences of the returned field) and the paper's printed
U_max, the error norms on a hand example, the grids of Table 1 and the pressure
boundaries of the tube."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import ipcs, steady

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    with open(os.path.join(GOLDEN, "poiseuille_paper.json")) as f:
        return json.load(f)


def test_nrmse_hand_values():
    nodes = np.array([0, 2, 3, 5])
    old = np.zeros((3, 6))
    new = np.zeros((3, 6))
    old[0, nodes] = [0.0, 1.0, 2.0, 3.0]        # range 3
    new[0, nodes] = [1.0, 2.0, 3.0, 4.0]        # every difference 1: sqrt(4 / 16) = 1/2
    old[1, nodes] = 5.0                         # constant and unchanged: 0
    new[1, nodes] = 5.0
    old[2, nodes] = 5.0                         # constant but changed: +inf
    new[2, nodes] = [5.0, 5.0, 5.0, 6.0]
    old[:, 1] = 100.0                           # nodes outside the list do not count
    new[:, 4] = -100.0
    r = steady.nrmse(new, old, nodes)
    assert r[0] == pytest.approx(0.5 / 3.0, rel=1e-15)
    assert r[1] == 0.0
    assert np.isinf(r[2])


def test_nrmse_invariances():
    rng = np.random.default_rng(4)
    nodes = np.sort(rng.choice(200, 120, replace=False))
    old = rng.standard_normal((3, 200))
    new = old + 1e-3 * rng.standard_normal((3, 200))
    r = steady.nrmse(new, old, nodes)
    # the same affine map applied to both fields leaves it unchanged
    assert np.allclose(steady.nrmse(2.5 * new - 7.0, 2.5 * old - 7.0, nodes), r, rtol=1e-12)
    # a uniform change delta gives |delta| / (sqrt(N) range)
    shifted = old + 0.25
    rng_old = old[:, nodes].max(axis=1) - old[:, nodes].min(axis=1)
    assert np.allclose(steady.nrmse(shifted, old, nodes), 0.25 / (math.sqrt(nodes.size) * rng_old),
                       rtol=1e-12)


def test_poiseuille_profile_balances_the_pressure_drop():
    gold = _gold()
    R, L, mu = gold["R"], gold["L"], gold["mu"]
    for case in gold["cases"]:
        dp = case["p_inlet"]
        assert steady.poiseuille_u_max(dp, L, R, mu) == pytest.approx(case["U_max_exact"], rel=2e-3)
        # mu Laplacian(u_z) = dp/dz = -dp / L at interior points (second differences)
        e = 1e-5
        pts = np.array([[0.0, 0.0, 0.01], [0.002, -0.001, 0.02], [-0.003, 0.0025, 0.04]])
        lap = np.zeros(len(pts))
        for a in range(2):
            dv = np.zeros(3)
            dv[a] = e
            lap += (steady.poiseuille_velocity(pts + dv, dp, L, R, mu)[2]
                    - 2 * steady.poiseuille_velocity(pts, dp, L, R, mu)[2]
                    + steady.poiseuille_velocity(pts - dv, dp, L, R, mu)[2]) / (e * e)
        assert np.allclose(mu * lap, -dp / L, rtol=1e-5)
        # no-slip on the wall, zero outside
        wall = np.array([[R, 0.0, 0.01], [0.0, -R, 0.03], [0.004, 0.0045, 0.02]])
        v = steady.poiseuille_velocity(wall, dp, L, R, mu)
        assert np.all(np.abs(v) <= 1e-18)


def test_error_norms_hand_values():
    u = np.zeros((3, 4))
    ex = np.zeros((3, 4))
    u[2] = [1.0, 2.0, 3.0, 4.0]
    ex[2] = [1.0, 2.5, 3.0, 3.0]
    u[0, 1] = 0.5
    linf, l2 = steady.error_norms(u, ex)
    assert linf == 1.0
    assert l2 == pytest.approx(math.sqrt(0.25 + 1.0 + 0.25) / 4.0, rel=1e-15)


def test_e1_grids_and_pressure_boundaries():
    gold = _gold()
    for level, row in enumerate(gold["table1"]):
        c = synth.poiseuille_e1(level)
        assert c.N == row["nodes"] and c.h == pytest.approx(row["h"], rel=1e-12)
    c = synth.poiseuille_e1(0, p_in=1.0)
    pr = ipcs.Problem.from_case(c)
    s = pr.sets
    xyz = c.node_coords()
    disk = (c.node_mask == 1) & ((xyz[:, 2] == 0.0) | (np.abs(xyz[:, 2] - 0.05) < 1e-12))
    assert disk.sum() > 0
    # the pressure-Dirichlet nodes are exactly the two end disks, and their velocity is free
    pd = np.zeros(c.N, bool)
    pd[s.P] = True
    pd[s.Pp] = False
    assert np.array_equal(pd, disk)
    assert np.all(s.in_F[disk])
    # two steps: the flow goes from the high to the low pressure end, the disks keep
    # their pressures exactly
    u, p = pr.initial_state(c.u0, c.p0)
    t = 0.0
    for _ in range(2):
        u, p, t, _ = pr.step(u, p, t)
    inlet = disk & (xyz[:, 2] == 0.0)
    assert np.all(p[inlet] == 1.0) and np.all(p[disk & ~inlet] == 0.0)
    assert u[2][c.node_mask == 1].mean() > 0.0


def test_e1_wall_band_lattice():
    # the 2:1 wall band variant: arrays on the fine lattice, the split cells are those
    # whose centre lies within the band of the wall radius, the pressure disks and the
    # wall rings follow the fine spacing
    from synth import poiseuille as e1
    band = 2e-3
    c = synth.poiseuille_e1(0, p_in=1.0, domain="box", refine_band=band)
    assert c.refine_cell is not None and c.N == 25 * 25 * 101
    ci = (np.arange(12) + 0.5) * 1e-3 - e1.HALF_WIDTH
    _, cy, cx = np.meshgrid(np.arange(50), ci, ci, indexing="ij")
    expect = np.abs(np.hypot(cx, cy) - e1.R) <= band
    assert np.array_equal(c.refine_cell.astype(bool), expect.ravel())
    xyz = c.node_coords()
    disk = (xyz[:, 0] ** 2 + xyz[:, 1] ** 2 < e1.R ** 2) & ((xyz[:, 2] == 0.0) | (np.abs(xyz[:, 2] - e1.L) < 1e-12))
    assert np.array_equal(c.bc_tag == synth.TAG_OUTLET, disk)
    plain = synth.poiseuille_e1(0, p_in=1.0, domain="box")
    assert c.M > 3.5 * plain.M       # points at 1.5 fine spacings: about 4 times as many
    assert c.dS * c.M == pytest.approx(2.0 * np.pi * e1.R * e1.L)
