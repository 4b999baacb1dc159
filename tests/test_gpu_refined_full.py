"""GPU checks of the refined aneurysm at full size (128x128x320 base cells, a
257x257x641 lattice, 2.8 M nodes of P) in the configurations bench.py times.

The oracle cannot assemble the composite operators of the whole lattice, but an
operator row only depends on the mesh within two base cells of its node.  Each
check crops a window of base cells, builds the oracle's composite mesh and
operators on the window, and compares rows at nodes at least three base cells
inside it: the derived sets (bit for bit), every operator apply, and the
defining equation of every sub-step of a full-size step (tentative velocity,
pressure increment, mass correction) evaluated on the GPU's outputs; the IB
constraint I u_ib = U_B is checked on all points with the full interpolation
matrix."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import make_solver, say
from oracle import fem, grid, ib, refine

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

WIN = 10      # base cells per window side
MARGIN = 6    # lattice units (three base cells) kept away from the window faces


@pytest.fixture(scope="module")
def c3():
    c = synth.aneurysm_case((128, 128, 320), nsteps=1)
    say("case", c.name, "lattice nodes", c.N, "points", c.M)
    return c


@pytest.fixture(scope="module")
def plan_info(c3):
    pl = ibfe.Plan(**ibfe.inputs_from_case(c3, precision=1, precond=2))
    return pl.node_ids(), pl.node_flags()


def _window_origins(c, flags, rng):
    """Window corners (base cells): around seeded hanging nodes, at the inlet, at the outlet."""
    lx, ly = 2 * c.nx, 2 * c.ny
    sy, sz = lx + 1, (lx + 1) * (ly + 1)
    hang = np.nonzero(flags & ibfe.FLAG_HANG)[0]
    picks = list(rng.choice(hang, 3, replace=False))
    P = np.nonzero(flags & ibfe.FLAG_P)[0]
    picks.append(P[np.argmin(P // sz)])            # lowest plane (inlet)
    picks.append(P[np.argmax(P // sz)])            # highest plane (outlet)
    out = []
    for n in picks:
        i, j, k = n % sy, (n // sy) % (ly + 1), n // sz
        lo = np.array([i // 2, j // 2, k // 2]) - WIN // 2
        lo = np.clip(lo, 0, np.array([c.nx, c.ny, c.nz]) - WIN)
        out.append(tuple(int(v) for v in lo))
    return out


class Window:
    def __init__(self, c, lo, tags_full):
        bi, bj, bk = lo
        lx, ly = 2 * c.nx, 2 * c.ny
        sy, sz = lx + 1, (lx + 1) * (ly + 1)
        I = np.arange(2 * bi, 2 * (bi + WIN) + 1)
        J = np.arange(2 * bj, 2 * (bj + WIN) + 1)
        K = np.arange(2 * bk, 2 * (bk + WIN) + 1)
        self.ids = (I[None, None, :] + sy * J[None, :, None] + sz * K[:, None, None]).ravel()
        ref = c.refine_cell.reshape(c.nz, c.ny, c.nx)[bk:bk + WIN, bj:bj + WIN, bi:bi + WIN].ravel()
        tags = tags_full[self.ids]
        self.mesh = refine.CompositeMesh(WIN, WIN, WIN, c.h, c.node_mask[self.ids], tags, ref)
        self.ops = refine.CompositeOperators(self.mesh)
        self.sets = self.mesh.derive_sets(tags)
        L = 2 * WIN
        a = np.arange(L + 1)
        inner = (a >= MARGIN) & (a <= L - MARGIN)
        self.inner = (inner[None, None, :] & inner[None, :, None] & inner[:, None, None]).ravel()
        self.lo = lo

    def gather(self, vals_p, pos):
        """Full-P vector (canonical order) -> window lattice vector (0 off P)."""
        out = np.zeros(self.ids.size)
        ok = pos >= 0
        out[ok] = vals_p[pos[ok]]
        return out


def _positions(ids_p, win):
    pos = np.searchsorted(ids_p, win.ids)
    pos[pos >= ids_p.size] = 0
    return np.where(ids_p[pos] == win.ids, pos, -1)


@pytest.fixture(scope="module")
def windows(c3, plan_info):
    ids_p, flags = plan_info
    tags_full = grid.default_tags(2 * c3.nx, 2 * c3.ny, 2 * c3.nz)
    rng = np.random.default_rng(31)
    ws = [Window(c3, lo, tags_full) for lo in _window_origins(c3, flags, rng)]
    for w in ws:
        w.pos = _positions(ids_p, w)
        say("window", w.lo, "hanging", int(w.mesh.hanging.size), "inner P", int((w.sets.in_P & w.inner).sum()))
    return ws


def test_full_size_refined_sets_on_windows(c3, plan_info, windows):
    _, flags = plan_info
    for w in windows:
        f = flags[w.ids][w.inner]
        s = w.sets
        assert np.array_equal((f & ibfe.FLAG_P) > 0, s.in_P[w.inner])
        assert np.array_equal((f & ibfe.FLAG_F) > 0, s.in_F[w.inner])
        assert np.array_equal((f & ibfe.FLAG_DU) > 0, s.in_Du[w.inner])
        assert np.array_equal((f & ibfe.FLAG_PDIR) > 0, s.p_dir[w.inner])
        assert np.array_equal((f & ibfe.FLAG_HANG) > 0, w.mesh.is_hanging[w.inner])


def _rows(w, mask):
    return np.nonzero(w.inner & mask)[0]


def test_full_size_refined_applies(c3, windows):
    s = make_solver(c3, precision=1, precond=2)
    n = s.n_u
    rng = np.random.default_rng(32)
    x = rng.standard_normal(n)
    a = rng.standard_normal((3, n))
    s.set_state(a, np.zeros(n), 0.0)
    Mf, Kf, Gf, _ = fem.element_matrices(c3.h / 2)
    Mc, Kc, Gc, _ = fem.element_matrices(c3.h)
    out = {}
    for op, prec in ((ibfe.OP_MASS, 0), (ibfe.OP_MASS, 1), (ibfe.OP_STIFF, 0), (ibfe.OP_STIFF, 1),
                     (ibfe.OP_GRAD, 0)):
        out[(op, prec)] = s.apply(op, x, prec)
    u3 = rng.standard_normal((3, n))
    out[(ibfe.OP_DIV, 0)] = s.apply(ibfe.OP_DIV, u3.ravel())
    out[(ibfe.OP_ADVDIFF, 0)] = s.apply(ibfe.OP_ADVDIFF, u3.ravel(), 0)
    out[(ibfe.OP_ADVDIFF, 1)] = s.apply(ibfe.OP_ADVDIFF, u3.ravel(), 1)
    s.close()
    for w in windows:
        rows = _rows(w, w.sets.in_P)
        prow = w.pos[rows]
        xw = w.gather(x, w.pos)
        for op, A, lf, lc in ((ibfe.OP_MASS, w.ops.M, Mf, Mc), (ibfe.OP_STIFF, w.ops.K, Kf, Kc)):
            ref = (A @ xw)[rows]
            Af = refine._assemble(w.mesh.fine, np.abs(lf), w.mesh.N) + refine._assemble(w.mesh.coarse, np.abs(lc), w.mesh.N)
            C = abs(w.mesh.C)
            bound = (C.T @ (Af @ (C @ np.abs(xw))))[rows]
            for prec, tol in ((0, 1e-13), (1, 2e-6)):
                err = np.abs(out[(op, prec)][prow] - ref)
                say("window", w.lo, "op", op, "prec", prec, "max err/bound", float((err / bound).max()))
                assert np.all(err <= tol * bound)
        g = out[(ibfe.OP_GRAD, 0)].reshape(3, -1)
        for d in range(3):
            ref = (w.ops.G[d] @ xw)[rows]
            assert np.abs(g[d][prow] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        uw = np.stack([w.gather(u3[d], w.pos) for d in range(3)])
        ref = w.ops.divergence(uw)[rows]
        assert np.abs(out[(ibfe.OP_DIV, 0)][prow] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        aw = np.stack([w.gather(a[d], w.pos) for d in range(3)])
        A = (c3.rho / c3.dt) * w.ops.M + c3.rho * w.ops.advection(aw) + c3.mu * w.ops.K
        y64 = out[(ibfe.OP_ADVDIFF, 0)].reshape(3, -1)
        y32 = out[(ibfe.OP_ADVDIFF, 1)].reshape(3, -1)
        for d in range(3):
            ref = (A @ uw[d])[rows]
            scale = np.abs(ref).max()
            assert np.abs(y64[d][prow] - ref).max() <= 1e-12 * scale
            assert np.abs(y32[d][prow] - ref).max() <= 1e-5 * scale


def _smooth_field(c, ids_p, rng, k=3):
    lx, ly = 2 * c.nx, 2 * c.ny
    sy, sz = lx + 1, (lx + 1) * (ly + 1)
    i, j, kk = ids_p % sy, (ids_p // sy) % (ly + 1), ids_p // sz
    x = c.origin[0] + i * c.h / 2
    y = c.origin[1] + j * c.h / 2
    z = c.origin[2] + kk * c.h / 2
    f = np.zeros(ids_p.size)
    for _ in range(k):
        a, b, cc, ph = rng.uniform(0.2, 1.5, 3).tolist() + [rng.uniform(0, 6.28)]
        f += np.sin(a * x + b * y + cc * z + ph)
    return f


@pytest.mark.parametrize("precision,tol", [(1, 1e-6), (0, 1e-10)])
def test_full_size_refined_step_equations(c3, plan_info, windows, precision, tol):
    """One full-size step from a smooth non-trivial state: every sub-step's equation holds
    on the window rows (residual relative to the largest right-hand-side entry there), and
    I u_ib = U_B on all points."""
    ids_p, _ = plan_info
    rng = np.random.default_rng(33)
    u0 = np.stack([_smooth_field(c3, ids_p, rng) for _ in range(3)])
    p0 = _smooth_field(c3, ids_p, rng)
    s = make_solver(c3, precision=precision, precond=2)
    s.set_state(u0, p0, 0.0)
    s.step(1)
    st = s.stats()
    say("full-size refined step, precision", precision, {k: st[k] for k in ("s1_iters", "ib_iters", "s3_iters", "s4_iters")})
    ustar = s.field(ibfe.FIELD_USTAR).reshape(3, -1)
    uib = s.field(ibfe.FIELD_UIB).reshape(3, -1)
    phi = s.field(ibfe.FIELD_PHI)
    u1, p1, t1 = s.get_state()
    s.close()
    u1 = u1.reshape(3, -1)
    assert np.allclose(p1, p0 + phi, rtol=0, atol=1e-12 * np.abs(p1).max())
    # IB constraint on every point
    I = ib.interpolation_matrix(c3.X, 2 * c3.nx, 2 * c3.ny, 2 * c3.nz, c3.h / 2, c3.origin)
    for d in range(3):
        uf = np.zeros(c3.N)
        uf[ids_p] = uib[d]
        # the force solve stops at 1e-13 (FP64) or 1e-10 (mixed) relative residual
        assert np.abs(I @ uf).max() <= (1e-9 if precision == 0 else 1e-7) * np.abs(uib[d]).max()
    rho, mu, dt = c3.rho, c3.mu, c3.dt
    for w in windows:
        g = lambda v: w.gather(v, w.pos)
        a = np.stack([g(u0[d]) for d in range(3)])
        A = (rho / dt) * w.ops.M + rho * w.ops.advection(a) + mu * w.ops.K
        pw, phw = g(p0), g(phi)
        rowsF = _rows(w, w.sets.in_F)
        rowsPp = _rows(w, w.sets.in_P & ~w.sets.p_dir)
        worst = []
        for d in range(3):
            rhs = (rho / dt) * (w.ops.M @ a[d]) - w.ops.G[d] @ pw
            r1 = (A @ g(ustar[d]) - rhs)[rowsF]
            worst.append(("S1", np.abs(r1).max() / np.abs(rhs[rowsF]).max()))
            lhs4 = (rho / dt) * (w.ops.M @ (g(uib[d]) - g(u1[d])))
            rhs4 = w.ops.G[d] @ phw
            worst.append(("S4", np.abs((lhs4 - rhs4)[rowsF]).max() / np.abs(rhs4[rowsF]).max()))
        uibw = np.stack([g(uib[d]) for d in range(3)])
        rhs3 = -(rho / dt) * w.ops.divergence(uibw)
        r3 = (w.ops.K @ phw - rhs3)[rowsPp]
        worst.append(("S3", np.abs(r3).max() / np.abs(rhs3[rowsPp]).max()))
        say("window", w.lo, " ".join(f"{k}={v:.1e}" for k, v in worst))
        for k, v in worst:
            assert v <= tol, (w.lo, k, v)
