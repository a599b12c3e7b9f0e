"""GPU parity of the Wilson dslash (C ABI) against the FP64 oracle.

Tolerances: FP64 1e-12 relative (max-norm over the output); FP32 2e-6 and
FP16S 4e-3 relative, derived from the storage precision (2^-24, 2^-11) times the
~9 terms summed per output component.  Full-size (16^3x32, 48 RHS, the
smoother's launch shape) cases are checked on sampled sites and through the
closed-form free-field symbol and gamma5-hermiticity, which hold at any size.
"""
import numpy as np
import pytest

import synth
from oracle import lattice as olat
from oracle.gamma import gamma5_full
from oracle.stencil import as_columns, as_fields
from oracle.wilson import WilsonOp, free_field_symbol

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-6, 2: 4e-3}


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("dims,xi,nrhs", [
    ([4, 4, 4, 4], 1.0, 1),
    ([4, 4, 6, 8], 3.5, 5),      # ragged against 2 and 4 RHS per thread
    ([6, 2, 4, 10], 2.0, 3),     # volume not a multiple of the 256-site workgroup
])
@pytest.mark.parametrize("form", [0, 1, 2])
def test_dslash_matches_oracle(crk, dims, xi, nrhs, form):
    print(f"dslash parity dims={dims} xi={xi} nrhs={nrhs} form={form}", flush=True)
    V = olat.volume(dims)
    U = synth.gauge_field(dims, 0.5, 1, config=101)
    psi = synth.gaussian_rhs(nrhs, V, config=101)
    lat = crk.Lattice(dims, -0.3, xi)
    lat.load_gauge(U)
    got = lat.dirac_apply(psi, form)
    ref = as_fields(WilsonOp(U, dims, -0.3, xi).apply(as_columns(psi)))
    err = float(_rel(got, ref))
    assert err <= TOL[form], err


def test_neighbor_map_bit_exact(crk):
    dims = [4, 6, 2, 8]
    lat = crk.Lattice(dims, 0.0, 1.0)
    assert np.array_equal(lat.neighbor_map(), olat.neighbors(dims).astype(np.int32))


def test_free_field_plane_wave_full_size(crk):
    dims = [16, 16, 16, 32]
    V = olat.volume(dims)
    m0, xi = -0.2, 3.5
    lat = crk.Lattice(dims, m0, xi)
    lat.load_gauge(synth.unit_gauge(dims))
    crd = olat.coords(dims)
    rng = np.random.default_rng(9)
    vs, wants = [], []
    for n in ([1, 0, 0, 0], [3, 5, 7, 11]):
        p = 2 * np.pi * np.asarray(n) / np.asarray(dims)
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        ph = np.exp(1j * crd @ p)
        vs.append((ph[:, None, None] * chi[None]).reshape(V, 12))
        wants.append((ph[:, None, None] * (free_field_symbol(p, m0, xi) @ chi)[None]).reshape(V, 12))
    got = lat.dirac_apply(np.stack(vs), 0)
    err = float(_rel(got, np.stack(wants)))
    assert err <= 1e-13, err


def test_gamma5_hermiticity_full_size(crk):
    dims = [16, 16, 16, 32]
    V = olat.volume(dims)
    U = synth.gauge_field(dims, 0.2, 0, config=2)
    lat = crk.Lattice(dims, -0.1, 3.5)
    lat.load_gauge(U)
    phi, chi = synth.gaussian_rhs(2, V, config=102)
    g5 = gamma5_full().diagonal()[None, :]
    Dphi, Dg5chi = lat.dirac_apply(np.stack([phi, g5 * chi]), 0)
    lhs = np.vdot(phi, g5 * Dg5chi)
    rhs = np.conj(np.vdot(chi, Dphi))
    err = float(abs(lhs - rhs) / abs(lhs))
    assert err <= 1e-12, err


@pytest.mark.parametrize("form", [0, 1])
def test_dslash_full_size_sampled_sites(crk, form):
    """16^3x32, xi=3.5, 48 RHS: the setup smoother's launch shape."""
    import torch
    dims, nrhs = [16, 16, 16, 32], 48
    print(f"full-size dslash form={form}", flush=True)
    V = olat.volume(dims)
    U = synth.gauge_field(dims, 0.2, 1, config=2)
    psi = synth.gaussian_vectors(nrhs, V, 12, config=2, level=0)
    lat = crk.Lattice(dims, -0.05, 3.5)
    lat.load_gauge(U)
    dev = torch.device("cuda", 0)
    host_layout = torch.from_numpy(psi.view(np.float64)).to(dev)
    a = torch.empty(lat.field_bytes(form, nrhs), dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    lat.import_dev(host_layout, a, nrhs, form)
    lat.dirac_apply_dev(a, b, nrhs, form)
    out = torch.empty_like(host_layout)
    lat.export_dev(b, out, nrhs, form)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.complex128).reshape(nrhs, V, 12)
    op = WilsonOp(U, dims, -0.05, 3.5)
    sites = np.random.default_rng(4).choice(V, 64, replace=False)
    cols = as_columns(psi)
    ref = op.apply_at(cols, sites)  # [sites, 12, nrhs]
    err = float(_rel(got[:, sites].transpose(1, 2, 0), ref))
    assert err <= TOL[form], err


@pytest.mark.parametrize("dims", [[8, 8, 8, 8], [4, 8, 4, 8]])
def test_hierarchy_fine_operator_4x4_blocks(crk, dims):
    """The fine operator inside a hierarchy with 4^4 blocks (block-major site order,
    the kernels the smoother and K-cycle use) against the oracle.  Extent 4 puts a
    single block along that direction, so its neighbours wrap into the block."""
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.3, 1, config=12)
    lat = crk.Lattice(dims, -0.2, 2.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[16], k=[8], block=[[4, 4, 4, 4]], n_smooth=[2], setup_form=crk.FORM_FP32)
    op = WilsonOp(U, dims, -0.2, 2.0)
    for nrhs in (1, 12):
        psi = synth.gaussian_vectors(nrhs, V, 12, config=13, level=nrhs)
        ref = as_fields(op.apply(as_columns(psi)))
        for form, tol in ((crk.FORM_FP64, 1e-12), (crk.FORM_FP32, 2e-6), (crk.FORM_FP16S, TOL[2])):
            out = H.coarse_apply(0, psi, form=form)
            err = np.abs(out - ref).max() / np.abs(ref).max()
            print(dims, nrhs, form, err, flush=True)
            assert err <= tol, (dims, nrhs, form, err)
    H.close()
