"""GPU parity of the Wilson-clover operator (the paper's ensembles, Sec. 4)
against the oracle's (oracle/clover.py), through the C ABI.

* The operator with the clover term in three forms, through the lattice's
  kernels (FP64 direction-split, FP32 site loop, FP16S generic) and through the
  hierarchy's block-staged fine operator (4^4 blocks): FP64 1e-12, FP32 2e-6
  and FP16S 4e-3 relative, the bounds of the plain operator's tests (the site
  blocks add six terms to each output component, the nine hop terms stay).
* gamma5-hermiticity of the GPU operator at 16^3x32 with the clover term.
* The FP64 setup with the clover term: smoothed vectors, singular values,
  prolongator columns and the Galerkin links (whose site term now carries the
  clover blocks) against the oracle, within the tolerances of the plain setup.
* The MG-GCR solve with the clover term: FP64 true residual 1e-10 in the FP32
  form and x against a dense LU solve within 2 kappa 1e-10.
"""
import numpy as np
import pytest

import synth
from oracle import lattice as olat, mg as omg
from oracle.gamma import gamma5_full
from oracle.stencil import StencilOp, as_columns, as_fields
from oracle.wilson import WilsonOp
from parity_bounds import compare_coarse_links, compare_prolongators, wilson_norm_bound

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-6, 2: 4e-3}
C_SW = 1.2


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("dims,xi,nrhs", [
    ([4, 4, 4, 4], 1.0, 1),
    ([4, 4, 6, 8], 3.5, 5),
    ([6, 2, 4, 10], 2.0, 3),
])
@pytest.mark.parametrize("form", [0, 1, 2])
def test_clover_operator_matches_oracle(crk, dims, xi, nrhs, form):
    print(f"clover dslash dims={dims} xi={xi} nrhs={nrhs} form={form}", flush=True)
    V = olat.volume(dims)
    U = synth.gauge_field(dims, 0.5, 1, config=111)
    psi = synth.gaussian_rhs(nrhs, V, config=111)
    lat = crk.Lattice(dims, -0.3, xi, c_sw=C_SW)
    lat.load_gauge(U)
    got = lat.dirac_apply(psi, form)
    op = WilsonOp(U, dims, -0.3, xi, c_sw=C_SW)
    ref = as_fields(op.apply(as_columns(psi)))
    err = float(_rel(got, ref))
    assert err <= TOL[form], err
    # the clover term is really applied: the plain operator differs by far more
    plain = as_fields(WilsonOp(U, dims, -0.3, xi).apply(as_columns(psi)))
    assert _rel(plain, ref) > 10 * TOL[form]
    lat.close()


def test_clover_set_before_and_after_gauge_load(crk):
    dims = [4, 4, 4, 8]
    U = synth.gauge_field(dims, 0.5, 1, config=112)
    psi = synth.gaussian_rhs(2, olat.volume(dims), config=112)
    a = crk.Lattice(dims, -0.2, 1.0, c_sw=0.9)
    a.load_gauge(U)
    b = crk.Lattice(dims, -0.2, 1.0)
    b.load_gauge(U)
    plain = b.dirac_apply(psi, 0)
    b.set_clover(0.9)
    assert np.array_equal(a.dirac_apply(psi, 0), b.dirac_apply(psi, 0))
    b.set_clover(0.0)
    assert np.array_equal(b.dirac_apply(psi, 0), plain)


@pytest.mark.parametrize("dims", [[8, 8, 8, 8], [4, 8, 4, 8]])
def test_clover_hierarchy_fine_operator(crk, dims):
    """The block-staged fine operator (4^4 blocks) with the clover blocks."""
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.3, 1, config=113)
    lat = crk.Lattice(dims, -0.2, 2.0, c_sw=C_SW)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[16], k=[8], block=[[4, 4, 4, 4]], n_smooth=[2], setup_form=crk.FORM_FP32)
    op = WilsonOp(U, dims, -0.2, 2.0, c_sw=C_SW)
    for nrhs in (1, 12):
        psi = synth.gaussian_vectors(nrhs, V, 12, config=114, level=nrhs)
        ref = as_fields(op.apply(as_columns(psi)))
        for form in (0, 1, 2):
            out = H.coarse_apply(0, psi, form=form)
            err = float(_rel(out, ref))
            print(dims, nrhs, form, err, flush=True)
            assert err <= TOL[form], (dims, nrhs, form, err)
    H.close()
    lat.close()


def test_clover_gamma5_hermiticity_full_size(crk):
    dims = [16, 16, 16, 32]
    V = olat.volume(dims)
    U = synth.gauge_field(dims, 0.2, 0, config=2)
    lat = crk.Lattice(dims, -0.1, 3.5, c_sw=1.5)
    lat.load_gauge(U)
    phi, chi = synth.gaussian_rhs(2, V, config=115)
    g5 = gamma5_full().diagonal()[None, :]
    Dphi, Dg5chi = lat.dirac_apply(np.stack([phi, g5 * chi]), 0)
    lhs = np.vdot(phi, g5 * Dg5chi)
    rhs = np.conj(np.vdot(chi, Dphi))
    assert abs(lhs - rhs) / abs(lhs) <= 1e-12


def test_clover_setup_fp64_matches_oracle(crk):
    dims, block, m, k, ns, m0 = [4, 4, 4, 8], [2, 2, 2, 2], 16, 8, 10, -0.4
    U = synth.gauge_field(dims, 0.3, 0, config=116)
    V = olat.volume(dims)
    v0 = synth.gaussian_vectors(m, V, 12, config=116, level=0)
    lat = crk.Lattice(dims, m0, 1.0, c_sw=C_SW)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[m], k=[k], block=[block], n_smooth=[ns], setup_form=crk.FORM_FP64,
                      init_vectors=[v0])
    try:
        op = WilsonOp(U, dims, m0, 1.0, c_sw=C_SW)
        ref = omg.mg_setup(op, [m], [k], [block], [ns], [as_columns(v0)], keep_vectors=True)
        vg, vo = H.vectors(0), as_fields(ref[0].vectors)
        assert (np.abs(vg - vo).max(axis=(1, 2)) / np.abs(vo).max(axis=(1, 2))).max() <= 1e-12
        Pg, Po = H.prolongator(0), ref[0].Pb
        dcol = compare_prolongators(Pg, Po, H.sigma(0), ref[0].sigma, k)
        L1 = ref[1].op
        # ||D|| with the clover term: the Wilson bound plus the largest site-block norm
        normD = wilson_norm_bound(m0, 1.0) + np.abs(np.linalg.eigvalsh(op.site - op.diag * np.eye(12))).max()
        compare_coarse_links(H.coarse_links(0), (L1.X, L1.Yp, L1.Ym), dcol, normD, L1.dims, Pg, Po)
    finally:
        H.close()
        lat.close()


def test_clover_solve_matches_dense_lu(crk):
    dims = [4, 4, 4, 4]
    U = synth.gauge_field(dims, 0.3, 0, config=117)
    v0 = synth.gaussian_vectors(16, 256, 12, config=117, level=0)
    lat = crk.Lattice(dims, -0.4, 1.0, c_sw=1.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[16], k=[8], block=[[2, 2, 2, 2]], n_smooth=[20], setup_form=crk.FORM_FP64,
                      init_vectors=[v0])
    try:
        b = synth.gaussian_rhs(2, 256, config=118)
        x, info = H.solve(b, form=crk.FORM_FP32)
        assert info["converged"] and info["true_rel_resid"] <= 1e-10, info
        D = WilsonOp(U, dims, -0.4, 1.0, c_sw=1.0).dense()
        kappa = np.linalg.cond(D)
        for r in range(2):
            xd = np.linalg.solve(D, b[r].reshape(-1))
            assert np.linalg.norm(x[r].reshape(-1) - xd) / np.linalg.norm(xd) <= 2 * kappa * 1e-10
    finally:
        H.close()
        lat.close()
