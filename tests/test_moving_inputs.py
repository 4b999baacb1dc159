"""Moving Lagrangian points on the CPU: the prescribed wall velocity is the time
derivative of the prescribed positions (central differences), and the oracle's
point update rebuilds I at the new positions, after which one step satisfies the
constraint I u_ib = U_B there."""
import numpy as np

import synth
from oracle import ib, ipcs


def test_pulsating_wall_velocity_is_the_position_derivative():
    _, wall = synth.pulsating_cylinder()
    e = 1e-6
    for t in (0.0, 0.037, 0.11):
        Xp, _ = wall.at(t + e)
        Xm, _ = wall.at(t - e)
        _, U = wall.at(t)
        assert np.allclose((Xp - Xm) / (2 * e), U, rtol=1e-7, atol=1e-8)
    # radial motion only: the heights do not change
    X0, _ = wall.at(0.0)
    X1, _ = wall.at(0.05)
    assert np.array_equal(X0[:, 2], X1[:, 2])


def test_oracle_set_points_rebuilds_the_interpolation():
    case, wall = synth.pulsating_cylinder()
    pr = ipcs.Problem.from_case(case)
    I0 = pr.I.copy()
    pr.set_points(case.X, case.U_B)
    assert abs(pr.I - I0).max() == 0.0
    X, U = wall.at(case.dt)
    pr.set_points(X, U)
    ref = ib.interpolation_matrix(X, case.nx, case.ny, case.nz, case.h, case.origin)
    assert abs(pr.I - ref).max() == 0.0
    assert abs(pr.I - I0).max() > 0.0
    u, p = pr.initial_state(case.u0, case.p0)
    _, _, _, info = pr.step(u, p, 0.0)
    Iu = np.stack([pr.I @ info.u_ib[d] for d in range(3)], axis=1)
    assert np.abs(Iu - U).max() <= 1e-10 * np.abs(U).max()
