"""2:1 locally refined Q1 discretisation (oracle; test infrastructure).

The paper refines its tetrahedral mesh near and inside the immersed boundary
(Sections 3.2 and 4, Plaza-Carey bisection).  On the Cartesian Q1 grid the
refinement reads: base cells flagged by the input are split into 2x2x2 children
of side h/2; all nodes live on the fine lattice ((2nx+1)(2ny+1)(2nz+1) nodes,
spacing h/2, x fastest).  Active elements:

* fine elements: lattice cells inside refined base cells, kept when a corner
  has mask 1;
* coarse elements: unrefined base cells (corners at even lattice positions),
  kept when a corner has mask 1.

A fine node that lies strictly inside an edge of a kept coarse element (one odd
coordinate) or strictly inside a face (two odd coordinates) is hanging: its
value is the mean of the 2 edge end points or of the 4 face corners, so that the
space stays continuous.  With the constraint matrix C (identity on the other
nodes) every operator becomes C^T A C, assembled from the element matrices of
both sizes.  P (velocity/pressure nodes) = corners of kept elements minus the
hanging nodes; boundary tags, mask and Dirichlet sets follow the uniform rules
on the lattice.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem, grid


class CompositeMesh:
    def __init__(self, nx, ny, nz, h, node_mask, bc_tag, refine_cell):
        self.nx, self.ny, self.nz = nx, ny, nz           # base cells
        self.lx, self.ly, self.lz = 2 * nx, 2 * ny, 2 * nz   # lattice cells
        self.h, self.hf = float(h), float(h) / 2.0
        self.N = (self.lx + 1) * (self.ly + 1) * (self.lz + 1)
        self.mask = np.asarray(node_mask, np.uint8)
        if self.mask.shape != (self.N,):
            raise ValueError("node_mask must cover the fine lattice")
        ref = np.asarray(refine_cell, np.uint8).reshape(nz, ny, nx).astype(bool)
        self.refine = ref
        sy, sz = self.lx + 1, (self.lx + 1) * (self.ly + 1)
        self.sy, self.sz = sy, sz

        def nid(i, j, k):
            return i + sy * (j + (self.ly + 1) * k)

        # fine elements
        ci, cj, ck = np.meshgrid(np.arange(self.lx), np.arange(self.ly), np.arange(self.lz), indexing="ij")
        ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
        in_ref = ref[ck // 2, cj // 2, ci // 2]
        ci, cj, ck = ci[in_ref], cj[in_ref], ck[in_ref]
        fc = np.stack([nid(ci + (a & 1), cj + ((a >> 1) & 1), ck + ((a >> 2) & 1)) for a in range(8)], 1)
        fkept = (self.mask[fc] == 1).any(axis=1)
        self.fine = fc[fkept]
        # coarse elements
        bi, bj, bk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        bi, bj, bk = bi.ravel(), bj.ravel(), bk.ravel()
        unref = ~ref[bk, bj, bi]
        bi, bj, bk = bi[unref], bj[unref], bk[unref]
        cc = np.stack([nid(2 * (bi + (a & 1)), 2 * (bj + ((a >> 1) & 1)), 2 * (bk + ((a >> 2) & 1)))
                       for a in range(8)], 1)
        ckept = (self.mask[cc] == 1).any(axis=1)
        self.coarse = cc[ckept]
        self.coarse_lo = np.stack([2 * bi[ckept], 2 * bj[ckept], 2 * bk[ckept]], 1)

        # hanging nodes: fine-element corners strictly inside a kept coarse edge/face
        corner = np.zeros(self.N, bool)
        corner[self.fine.ravel()] = True
        corner[self.coarse.ravel()] = True
        parents = {}
        fine_nodes = np.unique(self.fine.ravel())
        fine_set = np.zeros(self.N, bool)
        fine_set[fine_nodes] = True
        for lo in self.coarse_lo:
            x0, y0, z0 = lo
            # points of the coarse cell's faces/edges at lattice resolution
            for dz in range(3):
                for dy in range(3):
                    for dx in range(3):
                        odd = (dx == 1) + (dy == 1) + (dz == 1)
                        if odd == 0 or odd == 3:
                            continue
                        n = nid(x0 + dx, y0 + dy, z0 + dz)
                        if not fine_set[n] or n in parents:
                            continue
                        par = []
                        for ax in ([0, 2] if dx == 1 else [dx]):
                            for ay in ([0, 2] if dy == 1 else [dy]):
                                for az in ([0, 2] if dz == 1 else [dz]):
                                    par.append(nid(x0 + ax, y0 + ay, z0 + az))
                        parents[n] = par
        self.hanging = np.array(sorted(parents), dtype=np.int64)
        self.parents = parents
        rows, cols, vals = [], [], []
        is_h = np.zeros(self.N, bool)
        is_h[self.hanging] = True
        self.is_hanging = is_h
        for n in range(self.N):
            if not is_h[n]:
                rows.append(n), cols.append(n), vals.append(1.0)
        for n, par in parents.items():
            for q in par:
                rows.append(n), cols.append(q), vals.append(1.0 / len(par))
        self.C = sp.coo_matrix((vals, (rows, cols)), shape=(self.N, self.N)).tocsr()
        self.corner = corner

    # -- sets on the lattice ---------------------------------------------------
    def derive_sets(self, bc_tag):
        lx, ly, lz = self.lx, self.ly, self.lz
        tag = grid.default_tags(lx, ly, lz) if bc_tag is None else np.asarray(bc_tag, np.uint8)
        in_P = self.corner & ~self.is_hanging
        in_Du = in_P & ((self.mask == 0) | (tag == grid.TAG_WALL) | (tag == grid.TAG_INLET))
        in_F = in_P & ~in_Du
        p_dir = in_P & (tag == grid.TAG_OUTLET)
        kept_cells = np.zeros(0, bool)
        return grid.Sets(nx=lx, ny=ly, nz=lz, kept_cells=kept_cells,
                         corners=np.concatenate([self.fine, self.coarse]), in_P=in_P, in_F=in_F,
                         in_Du=in_Du, p_dir=p_dir, tag=tag, P=np.nonzero(in_P)[0], F=np.nonzero(in_F)[0],
                         D=np.nonzero(in_Du)[0], Pp=np.nonzero(in_P & ~p_dir)[0])


def _assemble(corners, local, N):
    return fem._assemble(corners, local, N)


class CompositeOperators:
    """C^T A C for the forms of fem.Operators on the composite mesh (N x N over
    lattice nodes; hanging rows and columns are zero)."""

    def __init__(self, mesh: CompositeMesh):
        self.mesh = mesh
        self.N = mesh.N
        Mf, Kf, Gf, Cf, Xf = fem.element_matrices_all(mesh.hf)
        Mc, Kc, Gc, Cc, Xc = fem.element_matrices_all(mesh.h)
        self._Cf, self._Cc = Cf, Cc
        self._Xf, self._Xc = Xf, Xc
        self._X = None
        C = mesh.C

        def both(lf, lc):
            A = _assemble(mesh.fine, lf, self.N) + _assemble(mesh.coarse, lc, self.N)
            return (C.T @ A @ C).tocsr()

        self.M = both(Mf, Mc)
        self.K = both(Kf, Kc)
        self.G = [both(Gf[d], Gc[d]) for d in range(3)]

    def strain_cross(self):
        """C^T X_de C over the fine and coarse elements (3 x 3 list of N x N): the
        cross blocks of the strain-rate viscous form on the composite mesh."""
        if self._X is None:
            m = self.mesh
            self._X = [[(m.C.T @ (_assemble(m.fine, self._Xf[d, e], self.N) +
                                  _assemble(m.coarse, self._Xc[d, e], self.N)) @ m.C).tocsr()
                        for e in range(3)] for d in range(3)]
        return self._X

    def advection(self, a: np.ndarray) -> sp.csr_matrix:
        """C^T C(a_full) C with a_full = C a (hanging values from their parents)."""
        m = self.mesh
        af = np.stack([m.C @ a[d] for d in range(3)])
        A = sp.csr_matrix((self.N, self.N))
        for corners, Ce in ((m.fine, self._Cf), (m.coarse, self._Cc)):
            if corners.size == 0:
                continue
            aloc = np.stack([af[d][corners] for d in range(3)], axis=2)
            local = np.einsum("ecd,icdb->eib", aloc, Ce)
            A = A + _assemble(corners, local, self.N)
        return (m.C.T @ A @ m.C).tocsr()

    def divergence(self, u: np.ndarray) -> np.ndarray:
        return self.G[0] @ u[0] + self.G[1] @ u[1] + self.G[2] @ u[2]
