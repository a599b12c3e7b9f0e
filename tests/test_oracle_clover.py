"""Pins of the oracle's clover term (Wilson-clover operator of the paper's
ensembles, Sec. 4) against facts that do not come from the oracle itself:

* the Dirac algebra of sigma_{mu nu} (Hermitian, square 1, odd under mu <-> nu,
  commuting with gamma5) and, derived by hand in the chiral basis,
  sigma_xy = i gamma_x gamma_y = -diag(sigma_3, sigma_3);
* a constant abelian field of quantised flux phi in one plane: every clover
  leaf is the plaquette diag(e^{i phi}, e^{-i phi}, 1), so
  F = diag(sin phi, -sin phi, 0) in that plane and 0 elsewhere, and the clover
  term's spectrum is +-(c_sw/2) w_mu w_nu sin(phi) (four each) and 0 (four);
* Hermiticity and exact chirality-block structure of C(x), gamma5-hermiticity
  of D with the clover term, gauge covariance, and the free field;
* the Galerkin stencil with the clover site term against the dense P^dag D P,
  and the MG solve against a dense LU solve.
"""
import numpy as np
import pytest

import synth
from oracle import chiral, clover, galerkin, lattice, mg as omg
from oracle.gamma import gamma, gamma5, gamma5_full
from oracle.stencil import as_columns
from oracle.wilson import WilsonOp


def test_sigma_algebra():
    for mu in range(4):
        for nu in range(4):
            s = clover.sigma_munu(mu, nu)
            assert np.allclose(s, s.conj().T, atol=0)
            assert np.allclose(s, -clover.sigma_munu(nu, mu), atol=0)
            assert np.allclose(s @ gamma5, gamma5 @ s, atol=0)
            if mu != nu:
                assert np.allclose(s @ s, np.eye(4), atol=1e-15)
                assert np.abs(s[:2, 2:]).max() == 0 and np.abs(s[2:, :2]).max() == 0
    # by hand: sigma_xy = i gamma_x gamma_y = i (-i s1)(i s2) (+) i (i s1)(-i s2) = i s1 s2 = -s3 in each block
    s3 = np.diag([1.0, -1.0])
    assert np.allclose(clover.sigma_munu(0, 1), -np.kron(np.eye(2), s3), atol=0)


def _abelian_flux(dims, mu, nu, n):
    """Constant flux phi = 2 pi n / (L_mu L_nu) in the (mu, nu) plane, in the U(1)
    subgroup diag(e^{i t}, e^{-i t}, 1): U_nu(x) = e^{i phi x_mu}; U_mu(x) = 1 except
    on the last mu-slice, where U_mu(x) = e^{-i phi L_mu x_nu} closes the torus."""
    V = lattice.volume(dims)
    c = lattice.coords(dims)
    phi = 2 * np.pi * n / (dims[mu] * dims[nu])
    theta = np.zeros((V, 4))
    theta[:, nu] = phi * c[:, mu]
    last = c[:, mu] == dims[mu] - 1
    theta[last, mu] = -phi * dims[mu] * c[last, nu]
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = np.exp(1j * theta)
    U[:, :, 1, 1] = np.exp(-1j * theta)
    U[:, :, 2, 2] = 1.0
    return U, phi


@pytest.mark.parametrize("mu,nu,xi", [(0, 1, 1.0), (1, 3, 2.5), (2, 3, 1.0)])
def test_constant_abelian_field_closed_form(mu, nu, xi):
    dims = [4, 6, 4, 6]
    U, phi = _abelian_flux(dims, mu, nu, 1)
    leaf = np.diag([np.exp(1j * phi), np.exp(-1j * phi), 1.0])
    Q = clover.clover_leaves(U, dims, mu, nu)
    assert np.abs(Q - 4 * leaf[None]).max() <= 1e-13
    F = clover.field_strength(U, dims, mu, nu)
    assert np.abs(F - np.diag([np.sin(phi), -np.sin(phi), 0.0])[None]).max() <= 1e-14
    for a in range(4):
        for b in range(a + 1, 4):
            if (a, b) != (mu, nu):
                assert np.abs(clover.field_strength(U, dims, a, b)).max() <= 1e-14
    c_sw = 1.7
    w = np.array([1.0, 1.0, 1.0, 1.0 / xi])
    C = clover.clover_term(U, dims, c_sw, xi)
    amp = 0.5 * c_sw * w[mu] * w[nu] * np.sin(phi)
    want = np.sort(np.array([amp] * 4 + [-amp] * 4 + [0.0] * 4))
    ev = np.linalg.eigvalsh(C[7])
    assert np.abs(np.sort(ev) - want).max() <= 1e-13
    if (mu, nu) == (0, 1):
        # sigma_xy = -diag(s3, s3): spin 0 sees +amp F/sin, spin 1 -amp F/sin, same for spins 2, 3
        d = np.diag(C[3]).real
        f = np.array([1.0, -1.0, 0.0])
        assert np.abs(d - amp * np.concatenate([f, -f, f, -f])).max() <= 1e-14


def test_clover_hermitian_chiral_blocks_and_free_field():
    dims = [4, 4, 4, 4]
    U = synth.gauge_field(dims, 0.4, 1, config=91)
    C = clover.clover_term(U, dims, 1.3, 2.0)
    assert np.abs(C - np.conj(np.swapaxes(C, -1, -2))).max() <= 1e-15
    assert np.abs(C[:, :6, 6:]).max() == 0.0 and np.abs(C[:, 6:, :6]).max() == 0.0
    assert np.abs(clover.clover_term(synth.unit_gauge(dims), dims, 1.3)).max() == 0.0


def test_gamma5_hermiticity_with_clover():
    dims = [2, 2, 2, 4]
    U = synth.gauge_field(dims, 0.6, 0, config=92)
    D = WilsonOp(U, dims, -0.3, 1.5, c_sw=1.1).dense()
    g5 = np.kron(np.eye(lattice.volume(dims)), gamma5_full())
    assert np.abs(g5 @ D @ g5 - D.conj().T).max() <= 1e-14 * np.abs(D).max()
    # and the clover term is really there
    assert np.abs(D - WilsonOp(U, dims, -0.3, 1.5).dense()).max() > 1e-2


def test_gauge_covariance_of_clover():
    dims = [4, 4, 2, 4]
    U = synth.gauge_field(dims, 0.5, 0, config=93)
    G = synth.random_gauge_transform(lattice.volume(dims), config=93)
    nbr = lattice.neighbors(dims)
    UG = np.stack([G @ U[:, mu] @ np.conj(np.swapaxes(G[nbr[:, 2 * mu]], -1, -2)) for mu in range(4)], axis=1)
    C, CG = clover.clover_term(U, dims, 0.9), clover.clover_term(UG, dims, 0.9)
    Gs = np.einsum("st,xab->xsatb", np.eye(4), G).reshape(-1, 12, 12)  # 1_spin (x) G(x)
    assert np.abs(CG - Gs @ C @ np.conj(np.swapaxes(Gs, -1, -2))).max() <= 1e-13


def test_galerkin_with_clover_matches_dense():
    dims, block = [4, 4, 4, 4], [2, 2, 2, 2]
    U = synth.gauge_field(dims, 0.3, 0, config=94)
    op = WilsonOp(U, dims, -0.4, 1.0, c_sw=1.2)
    psi = as_columns(synth.gaussian_vectors(16, 256, 12, config=94, level=0))
    A = chiral.chiral_blocks(psi, dims, block)
    Pb, _ = chiral.prolongator_blocks(A, 8)
    Dc = galerkin.galerkin(op, Pb, block).dense()
    P = chiral.prolongator_dense(Pb, dims, block, 12)
    want = P.conj().T @ op.dense() @ P
    assert np.abs(Dc - want).max() <= 1e-13 * np.abs(want).max()


def test_mg_solve_with_clover_matches_dense_lu():
    dims = [4, 4, 4, 4]
    U = synth.gauge_field(dims, 0.3, 0, config=95)
    op = WilsonOp(U, dims, -0.4, 1.0, c_sw=1.0)
    v0 = synth.gaussian_vectors(16, 256, 12, config=95, level=0)
    levels = omg.mg_setup(op, [16], [8], [[2, 2, 2, 2]], [20], [as_columns(v0)])
    b = as_columns(synth.gaussian_rhs(1, 256, config=95))
    x, info = omg.mg_solve(levels, b, tol=1e-10)
    D = op.dense()
    xd = np.linalg.solve(D, b.reshape(-1))
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x.reshape(-1) - xd) / np.linalg.norm(xd) <= 2 * kappa * 1e-10
    assert np.linalg.norm(b.reshape(-1) - D @ x.reshape(-1)) / np.linalg.norm(b) <= 1e-10
