"""One IPCS + BCE-IB time step (oracle; test infrastructure).

Order of Section 2.4 of the paper, with the readings listed in the design
notes (dynamic viscosity mu = rho nu, component-wise viscous form mu (grad u,
grad v), semi-implicit advection u^n . grad u*, minus sign in the velocity
correction, rho restored in the pressure equation, correction starting from
the IB-corrected velocity):

1. tentative velocity (Eq. 9, backward Euler):
   A = (rho/dt) M + rho C(u^n) + mu K,
   A_FF u*_F = (rho/dt)(M u^n)_F - (G_d p^n)_F - A_FD g(t^{n+1}),  u*_D = g(t^{n+1});
   with explicit advection (the fully explicit convection of Eq. 13, an option):
   A = (rho/dt) M + mu K (symmetric positive definite) and the right-hand side
   also carries - rho (C(u^n) u^n)_F;
   with the strain-rate viscous form 2 mu (eps(u), eps(v)) (an option) the three
   components couple: block (d, e) of the operator is A delta_de + mu X_de, and
   the three components are solved as one system;
2.-4. BCE-IB force and velocity correction (Eqs. 15-24): u_ib = u* + I_F^T Lambda with
   (I_F I_F^T) Lambda = U_B - I u*;
5. pressure increment (Eq. 12 with rho): K_{P'P'} Phi = -(rho/dt) (B u_ib)_{P'},
   Phi = 0 on outlet nodes, natural Neumann elsewhere; on a connected part of the
   domain without outlet the right-hand side is projected onto mean zero and the
   nodal mean of Phi is removed;
6. correction (L2 projection with the consistent mass):
   M_FF u^{n+1}_F = M_FF u_ib_F - (dt/rho)(G_d Phi)_F,  u^{n+1}_D = g(t^{n+1}),
   p^{n+1} = p^n + Phi.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

from . import fem, grid, ib, krylov, refine


@dataclasses.dataclass
class StepInfo:
    u_star: np.ndarray
    u_ib: np.ndarray
    phi: np.ndarray
    lam: np.ndarray
    iters: dict
    residuals: dict


class Problem:
    """Everything that depends only on the geometry and the parameters."""

    def __init__(self, nx, ny, nz, h, origin, node_mask, bc_tag, X, dS, U_B, rho, mu, dt,
                 inlet_K, inlet_omega, inlet_ids, inlet_shape, refine_cell=None, advection=0,
                 viscous=0):
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, float(h)
        if advection not in (0, 1):
            raise ValueError("advection must be 0 (semi-implicit) or 1 (explicit)")
        if viscous not in (0, 1):
            raise ValueError("viscous must be 0 (mu (grad u, grad v)) or 1 (2 mu (eps(u), eps(v)))")
        self.advection = int(advection)
        self.viscous = int(viscous)
        self.origin = np.asarray(origin, np.float64)
        self.mask = np.asarray(node_mask, np.uint8)
        self.rho, self.mu, self.dt = float(rho), float(mu), float(dt)
        self.mesh = None
        if refine_cell is not None:
            # 2:1 refined band: every array lives on the fine lattice (spacing h/2)
            self.mesh = refine.CompositeMesh(nx, ny, nz, h, self.mask, bc_tag, refine_cell)
            self.sets = self.mesh.derive_sets(bc_tag)
            self.ops = refine.CompositeOperators(self.mesh)
            lat, hk = (2 * nx, 2 * ny, 2 * nz), self.h / 2.0
        else:
            self.sets = grid.derive_sets(nx, ny, nz, self.mask, bc_tag)
            self.ops = fem.Operators(self.sets, self.h)
            lat, hk = (nx, ny, nz), self.h
        if self.sets.P.size == 0:
            raise ValueError("empty domain: no kept cell")
        self.inlet_K, self.inlet_omega = int(inlet_K), float(inlet_omega)
        self.inlet_ids = np.asarray(inlet_ids, np.int64)
        self.inlet_shape = np.asarray(inlet_shape, np.float64)
        grid.check_inlet_table(self.sets, self.mask, self.inlet_ids, skip_non_mesh=self.mesh is not None)
        self.X = np.asarray(X, np.float64).reshape(-1, 3)
        self.dS = float(dS)
        self.U_B = np.zeros_like(self.X) if U_B is None else np.asarray(U_B, np.float64)
        self.I = ib.interpolation_matrix(self.X, *lat, hk, self.origin)
        if self.mesh is not None:
            self._check_support_in_fine_band()
        self._pressure_setup()

    def set_points(self, X: np.ndarray, U_B: np.ndarray | None = None):
        """Move the Lagrangian points (same count): the interpolation matrix of Eq. 17
        is rebuilt at the new positions, U_B is their prescribed velocity (None = 0).
        The next step enforces I u = U_B at these positions."""
        X = np.asarray(X, np.float64).reshape(-1, 3)
        if X.shape != self.X.shape:
            raise ValueError("the number of Lagrangian points is fixed")
        self.X = X
        self.U_B = np.zeros_like(X) if U_B is None else np.asarray(U_B, np.float64).reshape(-1, 3)
        if self.mesh is not None:
            # the kernel on the fine lattice; the supports must stay in the band
            self.I = ib.interpolation_matrix(X, 2 * self.nx, 2 * self.ny, 2 * self.nz, self.h / 2.0, self.origin)
            self._check_support_in_fine_band()
        else:
            self.I = ib.interpolation_matrix(X, self.nx, self.ny, self.nz, self.h, self.origin)

    @classmethod
    def from_case(cls, c, advection=0, viscous=0):
        return cls(c.nx, c.ny, c.nz, c.h, c.origin, c.node_mask, c.bc_tag, c.X, c.dS, c.U_B,
                   c.rho, c.mu, c.dt, c.inlet_K, c.inlet_omega, c.inlet_ids, c.inlet_shape,
                   getattr(c, "refine_cell", None), advection, viscous)

    def _check_support_in_fine_band(self):
        """Reading of the refined band: the kernel support of every Lagrangian point
        lies in the closure of refined cells and holds no hanging node."""
        m = self.mesh
        ok = np.zeros(m.N, bool)
        bk, bj, bi = np.nonzero(m.refine)
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    ok[(2 * bi + dx) + m.sy * ((2 * bj + dy) + (m.ly + 1) * (2 * bk + dz))] = True
        ok &= ~m.is_hanging
        cols = self.I.indices
        if cols.size and not ok[cols].all():
            raise ValueError("a Lagrangian point's kernel support leaves the refined band")

    # -- step 5 helpers -------------------------------------------------------
    def _pressure_setup(self):
        s = self.sets
        Pp = s.Pp
        self.K_pp = self.ops.K[Pp][:, Pp].tocsr()
        # Connected parts of the kept region (through shared cells) without an outlet node.
        KP = self.ops.K[s.P][:, s.P]
        ncomp, label = csgraph.connected_components(KP, directed=False)
        has_outlet = np.zeros(ncomp, bool)
        has_outlet[label[s.p_dir[s.P]]] = True
        pos_in_P = -np.ones(s.in_P.size, np.int64)
        pos_in_P[s.P] = np.arange(s.P.size)
        lab_pp = label[pos_in_P[Pp]]
        self.floating = [np.nonzero(lab_pp == c)[0] for c in range(ncomp) if not has_outlet[c]]

    def g(self, t: float) -> np.ndarray:
        return grid.dirichlet_values(self.sets, self.mask, self.inlet_ids, self.inlet_shape,
                                     self.inlet_K, self.inlet_omega, t)

    # -- the time step -------------------------------------------------------
    def step(self, u: np.ndarray, p: np.ndarray, t: float):
        """Advance (u^n, p^n, t^n) -> (u^{n+1}, p^{n+1}, t^n + dt)."""
        s, ops = self.sets, self.ops
        rho, mu, dt = self.rho, self.mu, self.dt
        F, D = s.F, s.D
        t1 = t + dt
        g = self.g(t1)
        iters, resid = {}, {}

        # 1. tentative velocity
        C = ops.advection(u)
        if self.advection == 0:
            A = ((rho / dt) * ops.M + rho * C + mu * ops.K).tocsr()
        else:
            A = ((rho / dt) * ops.M + mu * ops.K).tocsr()
        A_FF = A[F][:, F].tocsr()
        diag = A_FF.diagonal()
        u_star = np.zeros_like(u)
        if self.viscous == 1:
            # coupled components: blocks A delta_de + mu X_de, one solve on all three
            # (BiCGStab; CG with explicit advection, where the blocks are symmetric)
            X = ops.strain_cross()
            full = [[(A if d == e else sp.csr_matrix(A.shape)) + mu * X[d][e] for e in range(3)]
                    for d in range(3)]
            rhs = []
            for d in range(3):
                r = (rho / dt) * (ops.M @ u[d]) - ops.G[d] @ p
                for e in range(3):
                    r = r - full[d][e] @ g[e]
                if self.advection == 1:
                    r = r - rho * (C @ u[d])
                rhs.append(r[F])
            AF = sp.bmat([[full[d][e][F][:, F] for e in range(3)] for d in range(3)]).tocsr()
            solve = krylov.bicgstab if self.advection == 0 else krylov.cg
            x, it, res = solve(AF, np.concatenate(rhs), x0=np.concatenate([u[d][F] for d in range(3)]),
                               diag=AF.diagonal())
            nf = F.size
            for d in range(3):
                u_star[d] = g[d]
                u_star[d][F] = x[d * nf:(d + 1) * nf]
                iters[f"s1_{d}"], resid[f"s1_{d}"] = it, res
        for d in range(3 if self.viscous == 0 else 0):
            rhs = (rho / dt) * (ops.M @ u[d]) - ops.G[d] @ p - A @ g[d]
            if self.advection == 0:
                x, it, res = krylov.bicgstab(A_FF, rhs[F], x0=u[d][F], diag=diag)
            else:
                rhs = rhs - rho * (C @ u[d])
                x, it, res = krylov.cg(A_FF, rhs[F], x0=u[d][F], diag=diag)
            u_star[d] = g[d]
            u_star[d][F] = x
            iters[f"s1_{d}"], resid[f"s1_{d}"] = it, res

        # 2.-4. BCE-IB correction
        u_ib, lam, info = ib.bce_correction(self.I, s.in_F, self.U_B, u_star)
        iters["ib"] = info.get("iters", info.get("method"))

        # 5. pressure increment
        rhs = -(rho / dt) * ops.divergence(u_ib)
        b = rhs[s.Pp]
        for comp in self.floating:
            b[comp] -= b[comp].mean()
        x, it, res = krylov.cg(self.K_pp, b, diag=self.K_pp.diagonal())
        for comp in self.floating:
            x[comp] -= x[comp].mean()
        phi = np.zeros(s.in_P.size)
        phi[s.Pp] = x
        iters["s3"], resid["s3"] = it, res

        # 6. correction
        M_FF = ops.M[F][:, F].tocsr()
        mdiag = M_FF.diagonal()
        u_new = np.zeros_like(u)
        for d in range(3):
            rhs = M_FF @ u_ib[d][F] - (dt / rho) * (ops.G[d] @ phi)[F]
            x, it, res = krylov.cg(M_FF, rhs, x0=u_ib[d][F], diag=mdiag)
            u_new[d] = g[d]
            u_new[d][F] = x
            iters[f"s4_{d}"], resid[f"s4_{d}"] = it, res
        p_new = np.where(s.in_P, p + phi, 0.0)
        return u_new, p_new, t1, StepInfo(u_star, u_ib, phi, lam, iters, resid)

    def initial_state(self, u0: np.ndarray, p0: np.ndarray):
        """Restrict an initial field to P (zero elsewhere)."""
        u = np.where(self.sets.in_P[None, :], u0, 0.0)
        p = np.where(self.sets.in_P, p0, 0.0)
        return u, p

    def run(self, u0, p0, nsteps: int, t0: float = 0.0):
        u, p = self.initial_state(u0, p0)
        t = t0
        infos = []
        for _ in range(nsteps):
            u, p, t, info = self.step(u, p, t)
            infos.append(info)
        return u, p, t, infos


def divergence_norm(problem: Problem, u: np.ndarray) -> float:
    """|(B u)_{P'}|_2, the discrete divergence on pressure-free nodes."""
    return float(np.linalg.norm(problem.ops.divergence(u)[problem.sets.Pp]))


def sparse_row(A: sp.csr_matrix, i: int):
    return A.indices[A.indptr[i]:A.indptr[i + 1]], A.data[A.indptr[i]:A.indptr[i + 1]]
