"""Moving Lagrangian points: a vessel wall pulsating in the radial direction.

The wall points of a straight tube (rings at fixed heights, equal angles) move
with radius R(t) = R0 (1 + amp sin(2 pi t / period)); their prescribed velocity
is the time derivative of the position, R0 amp (2 pi / period) cos(2 pi t / period)
along the outward radial direction.  Inputs only: positions and velocities.
"""
from __future__ import annotations

import math

import numpy as np

from .cases import Case, refined_cylinder, small_cylinder


class PulsatingWall:
    """Positions and velocities of the ring points at time t."""

    def __init__(self, radius: float, z_levels: np.ndarray, per_ring: int, amp: float, period: float):
        self.r0 = float(radius)
        self.amp = float(amp)
        self.omega = 2.0 * math.pi / float(period)
        theta = 2.0 * math.pi * np.arange(per_ring, dtype=np.float64) / per_ring
        zz, tt = np.meshgrid(np.asarray(z_levels, np.float64), theta, indexing="ij")
        self.cos, self.sin, self.z = np.cos(tt).ravel(), np.sin(tt).ravel(), zz.ravel()

    def at(self, t: float):
        r = self.r0 * (1.0 + self.amp * math.sin(self.omega * t))
        v = self.r0 * self.amp * self.omega * math.cos(self.omega * t)
        X = np.stack([r * self.cos, r * self.sin, self.z], axis=1)
        U = np.stack([v * self.cos, v * self.sin, np.zeros_like(self.z)], axis=1)
        return X, U


def pulsating_cylinder(cells_xy: int = 8, cells_z: int = 16, length: float = 2.0, rings: int = 8,
                       per_ring: int = 12, amp: float = 0.04, period: float = 0.2,
                       nsteps: int = 3, dt: float = 0.02) -> tuple[Case, PulsatingWall]:
    """The reduced cylinder (R0 = 0.5, parabolic inlet) with its wall points moving
    radially; the case holds the positions at t = 0."""
    c = small_cylinder(cells_xy, cells_z, length=length, rings=rings, per_ring=per_ring,
                       nsteps=nsteps, dt=dt)
    z_levels = (np.arange(rings, dtype=np.float64) + 0.5) * (length / rings)
    wall = PulsatingWall(0.5, z_levels, per_ring, amp, period)
    c.X, c.U_B = wall.at(0.0)
    c.name = f"pulsating_wall_{cells_xy}x{cells_xy}x{cells_z}"
    return c, wall


def pulsating_refined_cylinder(amp: float = 0.03, period: float = 0.2, nsteps: int = 3) -> tuple[Case, PulsatingWall]:
    """The refined test cylinder (8 x 8 x 8 base cells of 1.25/8, 2:1 band of 0.3 around
    R0 = 0.5) with its wall rings moving radially; the supports stay in the band for
    amplitudes up to a few percent.  The case holds the positions at t = 0."""
    c = refined_cylinder(8, 8, length=1.25, band=0.3, nsteps=nsteps)
    z = np.unique(np.round(c.X[:, 2], 12))
    per_ring = c.M // z.size
    wall = PulsatingWall(0.5, z, per_ring, amp, period)
    X0, U0 = wall.at(0.0)
    if not np.allclose(np.sort(X0[:, 2]), np.sort(c.X[:, 2])):
        raise ValueError("ring layout differs from the refined cylinder's")
    c.X, c.U_B = X0, U0
    c.name = "pulsating_wall_refined_8x8x8"
    return c, wall
