"""CPU-only checks of the C ABI library: it loads, exports every symbol that
include/ibfe.h declares, and its host set-up (derived sets, canonical order,
input validation) agrees bit for bit with the oracle."""
import os
import re

import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from oracle import grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "ibfe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibfe_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ibfe.load()
    names = _declared_symbols()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ibfe.SIGNATURES), "binding and header disagree"


CASES = [
    lambda: synth.random_blob_case(seed=1),
    lambda: synth.random_blob_case(cells=(7, 4, 5), seed=9),
    lambda: synth.poiseuille_c1(),
    lambda: synth.small_cylinder(8, 16),
    lambda: synth.closed_box(4),
    lambda: synth.channel_case(),
    lambda: synth.shear_advection_case(),
]


@pytest.mark.parametrize("make", CASES)
def test_plan_sets_match_oracle_bit_exactly(make):
    c = make()
    pl = ibfe.Plan(**ibfe.inputs_from_case(c))
    s = grid.derive_sets(c.nx, c.ny, c.nz, c.node_mask, c.bc_tag)
    np.testing.assert_array_equal(pl.node_ids(), s.P)
    f = pl.node_flags()
    np.testing.assert_array_equal((f & ibfe.FLAG_P) > 0, s.in_P)
    np.testing.assert_array_equal((f & ibfe.FLAG_F) > 0, s.in_F)
    np.testing.assert_array_equal((f & ibfe.FLAG_DU) > 0, s.in_Du)
    np.testing.assert_array_equal((f & ibfe.FLAG_PDIR) > 0, s.p_dir)
    sz = pl.sizes()
    assert sz["n_p"] == s.P.size and sz["n_free"] == s.F.size and sz["n_pfree"] == s.Pp.size
    assert sz["n_kept_cells"] == int(s.kept_cells.sum())


def test_c1_counts():
    c = synth.poiseuille_c1()
    sz = ibfe.Plan(**ibfe.inputs_from_case(c)).sizes()
    assert (sz["n_p"], sz["n_free"], sz["n_kept_cells"]) == (16705, 12352, 14336)


def test_floating_part_detected():
    assert ibfe.Plan(**ibfe.inputs_from_case(synth.closed_box(4))).sizes()["n_floating"] == 1
    assert ibfe.Plan(**ibfe.inputs_from_case(synth.shear_advection_case())).sizes()["n_floating"] == 1
    assert ibfe.Plan(**ibfe.inputs_from_case(synth.poiseuille_c1())).sizes()["n_floating"] == 0


def test_input_errors():
    c = synth.random_blob_case(seed=1)
    kw = ibfe.inputs_from_case(c)
    bad = dict(kw, node_mask=np.zeros_like(c.node_mask))
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    bad = dict(kw, node_mask=np.full_like(c.node_mask, 2))
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    bad = dict(kw, mu=-1.0)
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    # an inlet table node that is not an inlet-tagged node of P
    bad = dict(kw, inlet_ids=np.array([c.N - 1]), inlet_shape=np.zeros((5, 1, 3)))
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    bad = dict(kw, advection=2)
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    bad = dict(kw, precond=3)
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    ibfe.Plan(**dict(kw, advection=1, precond=1))
    # strain-rate viscous form: 0/1 only, uniform and refined, either advection
    ibfe.Plan(**dict(kw, viscous=1))
    ibfe.Plan(**dict(kw, viscous=1, advection=1))
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**dict(kw, viscous=2))
    # mass-correction preconditioner: 0 (Jacobi) or 1 (tensor product)
    ibfe.Plan(**dict(kw, mass_precond=0))
    with pytest.raises(ibfe.IbfeError, match="mass_precond"):
        ibfe.Plan(**dict(kw, mass_precond=2))
    rc = synth.refined_cylinder(8, 8, length=1.25, band=0.3)
    ibfe.Plan(**ibfe.inputs_from_case(rc, viscous=1))
    ibfe.Plan(**ibfe.inputs_from_case(rc, viscous=1, advection=1))
    # a Lagrangian point whose support holds no free node
    far = np.array([[100.0, 100.0, 100.0]])
    bad = dict(kw, X=far, U_B=None)
    with pytest.raises(ibfe.IbfeError, match="ESINGULAR"):
        ibfe.Plan(**bad)


def test_request_footprint_estimate_grows_with_size():
    small = ibfe.request_footprint(**ibfe.inputs_from_case(synth.small_cylinder(8, 16), precision=1, precond=2))
    big = ibfe.request_footprint(**ibfe.inputs_from_case(synth.small_cylinder(16, 32), precision=1, precond=2))
    fp64 = ibfe.request_footprint(**ibfe.inputs_from_case(synth.small_cylinder(16, 32), precision=0, precond=2))
    assert 0 < small < big
    assert fp64 < big          # the FP32 work space is extra
    c2 = ibfe.request_footprint(**ibfe.inputs_from_case(synth.pulsatile_c2(), precision=1, precond=2))
    assert 1e9 < c2 < 4e9      # 64x64x512: a few GB of the 288 GB


def test_serving_stream_is_seeded_and_sized():
    a = synth.request_stream(build=False)
    b = synth.request_stream(build=False)
    assert [(r.kind, r.radius, r.arrival) for r in a] == [(r.kind, r.radius, r.arrival) for r in b]
    assert len(a) == 64 and 8.0 < a[-1].arrival < 24.0   # Poisson arrivals at 4 per second
    assert {r.kind for r in a} == {"cylinder", "aneurysm", "branch"}


REFINED = [
    lambda: synth.refined_cylinder(8, 8, length=1.25, band=0.3),
    lambda: _no_points(synth.refined_cylinder(6, 4, length=1.25 * 4 / 6, band=0.25, mask_all=True)),
    lambda: synth.aneurysm_case((16, 16, 40), band=1.2, nsteps=2),
]


def _no_points(c):
    c.X = np.zeros((0, 3))
    return c


@pytest.mark.parametrize("make", REFINED)
def test_refined_plan_sets_match_oracle_bit_exactly(make):
    """2:1 refined lattice: P, F, D_u, outlet and hanging nodes, canonical order."""
    from oracle import refine

    c = make()
    pl = ibfe.Plan(**ibfe.inputs_from_case(c))
    mesh = refine.CompositeMesh(c.nx, c.ny, c.nz, c.h, c.node_mask, c.bc_tag, c.refine_cell)
    s = mesh.derive_sets(c.bc_tag)
    np.testing.assert_array_equal(pl.node_ids(), s.P)
    f = pl.node_flags()
    np.testing.assert_array_equal((f & ibfe.FLAG_P) > 0, s.in_P)
    np.testing.assert_array_equal((f & ibfe.FLAG_F) > 0, s.in_F)
    np.testing.assert_array_equal((f & ibfe.FLAG_DU) > 0, s.in_Du)
    np.testing.assert_array_equal((f & ibfe.FLAG_PDIR) > 0, s.p_dir)
    np.testing.assert_array_equal(np.nonzero(f & ibfe.FLAG_HANG)[0], mesh.hanging)
    sz = pl.sizes()
    assert sz["n_kept_cells"] == len(mesh.fine) + len(mesh.coarse)
    assert sz["n_p"] == s.P.size and sz["n_free"] == s.F.size and sz["n_pfree"] == s.Pp.size
    assert mesh.hanging.size > 0 or c.refine_cell.all()


def test_refined_input_errors():
    c = synth.refined_cylinder(8, 8, length=1.25, band=0.3)
    kw = ibfe.inputs_from_case(c)
    bad = dict(kw, refine_cell=np.full_like(c.refine_cell, 2))
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        ibfe.Plan(**bad)
    # a point whose kernel support leaves the refined band
    X = np.concatenate([c.X, [[0.0, 0.0, 0.6]]])
    with pytest.raises(ibfe.IbfeError, match="refined band"):
        ibfe.Plan(**dict(kw, X=X))
    # an inlet entry at a lattice point that is not a node of P is skipped, one at a
    # node of P that is not an inlet node is rejected
    from oracle import refine

    mesh = refine.CompositeMesh(c.nx, c.ny, c.nz, c.h, c.node_mask, c.bc_tag, c.refine_cell)
    s = mesh.derive_sets(c.bc_tag)
    assert not s.in_P[c.inlet_ids].all()
    ibfe.Plan(**kw)
    interior = s.P[(s.tag[s.P] == 0)][:1]
    with pytest.raises(ibfe.IbfeError, match="inlet"):
        ibfe.Plan(**dict(kw, inlet_ids=np.concatenate([c.inlet_ids, interior]),
                         inlet_shape=np.zeros((1, c.inlet_ids.size + 1, 3))))
