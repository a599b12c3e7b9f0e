"""Pins of the oracle's geometry, gamma matrices and Wilson-Dirac operator.

Each check compares the oracle with something it does not compute itself:
brute-force enumeration, the Clifford algebra, the closed-form free-field
spectrum and plane-wave symbol, gamma5-hermiticity and gauge covariance.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import synth
from oracle import lattice
from oracle.gamma import gamma, gamma5, identity4, gamma5_full
from oracle.stencil import as_columns
from oracle.wilson import WilsonOp, free_field_eigenvalues, free_field_symbol


# ---------------------------------------------------------------- P1 maps
def test_site_index_and_neighbours_brute_force():
    dims = [4, 2, 6, 2]
    V = lattice.volume(dims)
    nbr = lattice.neighbors(dims)
    crd = lattice.coords(dims)
    s = 0
    for t in range(dims[3]):
        for z in range(dims[2]):
            for y in range(dims[1]):
                for x in range(dims[0]):
                    c = (x, y, z, t)
                    assert tuple(crd[s]) == c
                    for mu in range(4):
                        for k, sg in enumerate((1, -1)):
                            cc = list(c)
                            cc[mu] = (cc[mu] + sg) % dims[mu]
                            want = cc[0] + dims[0] * (cc[1] + dims[1] * (cc[2] + dims[2] * cc[3]))
                            assert nbr[s, 2 * mu + k] == want
                    s += 1
    assert s == V


def test_block_maps_brute_force():
    dims, block = [4, 2, 6, 2], [2, 1, 3, 2]
    cd = lattice.coarse_dims(dims, block)
    assert cd == [2, 2, 2, 1]
    j, l = lattice.block_maps(dims, block)
    bs = lattice.block_sites(dims, block)
    seen = np.zeros(lattice.volume(dims), dtype=int)
    for s, c in enumerate(lattice.coords(dims)):
        X = [c[m] // block[m] for m in range(4)]
        r = [c[m] % block[m] for m in range(4)]
        jj = X[0] + cd[0] * (X[1] + cd[1] * (X[2] + cd[2] * X[3]))
        ll = r[0] + block[0] * (r[1] + block[1] * (r[2] + block[2] * r[3]))
        assert j[s] == jj and l[s] == ll
        assert bs[jj, ll] == s
        seen[bs[jj, ll]] += 1
    assert (seen == 1).all()
    with pytest.raises(ValueError):
        lattice.coarse_dims([4, 4, 4, 4], [3, 2, 2, 2])


# ---------------------------------------------------------------- P2 gamma
def test_gamma_algebra():
    for mu in range(4):
        assert np.allclose(gamma[mu], gamma[mu].conj().T, atol=0)
        for nu in range(4):
            anti = gamma[mu] @ gamma[nu] + gamma[nu] @ gamma[mu]
            assert np.array_equal(anti, 2.0 * (mu == nu) * identity4)
        assert np.array_equal(gamma5 @ gamma[mu] + gamma[mu] @ gamma5, np.zeros((4, 4)))
    assert np.array_equal(gamma5, np.diag([1, 1, -1, -1]).astype(complex))


# ---------------------------------------------------------------- P3 gamma5-hermiticity
@pytest.mark.parametrize("xi", [1.0, 3.5])
def test_gamma5_hermiticity_dense(xi):
    dims = [2, 2, 2, 4]
    U = synth.gauge_field(dims, 0.7, 0, config=11)
    D = WilsonOp(U, dims, -0.3, xi).dense()
    G5 = np.kron(np.eye(lattice.volume(dims)), gamma5_full())
    assert np.abs(G5 @ D @ G5 - D.conj().T).max() <= 1e-14 * np.abs(D).max()


def test_gamma5_hermiticity_matrix_free():
    dims = [4, 4, 4, 6]
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.5, 1, config=12)
    op = WilsonOp(U, dims, -0.2, 2.0)
    phi, chi = (as_columns(synth.gaussian_rhs(1, V, config=12, index=i)) for i in (0, 1))
    g5 = gamma5_full().diagonal()[None, :, None]
    lhs = np.vdot(phi, g5 * op.apply(g5 * chi))
    rhs = np.conj(np.vdot(chi, op.apply(phi)))
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs)


# ---------------------------------------------------------------- P4 free field
@pytest.mark.parametrize("dims,xi,m0", [([2, 2, 2, 2], 1.0, -0.4), ([2, 2, 2, 4], 3.5, 0.1)])
def test_free_field_spectrum_closed_form(dims, xi, m0):
    D = WilsonOp(synth.unit_gauge(dims), dims, m0, xi).dense()
    ev = np.linalg.eigvals(D)
    ref = free_field_eigenvalues(dims, m0, xi)
    cost = np.abs(ev[:, None] - ref[None, :])
    r, c = linear_sum_assignment(cost)
    assert cost[r, c].max() <= 1e-10


def test_free_field_plane_wave_symbol():
    dims = [4, 6, 4, 8]
    V = lattice.volume(dims)
    m0, xi = -0.25, 3.5
    op = WilsonOp(synth.unit_gauge(dims), dims, m0, xi)
    rng = np.random.default_rng(5)
    crd = lattice.coords(dims)
    for n in ([1, 0, 0, 0], [0, 1, 2, 3], [3, 5, 1, 7]):
        p = 2 * np.pi * np.asarray(n) / np.asarray(dims)
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * crd @ p)
        v = (phase[:, None, None] * chi[None]).reshape(V, 12, 1)
        out = op.apply(v).reshape(V, 4, 3)
        want = phase[:, None, None] * (free_field_symbol(p, m0, xi) @ chi)[None]
        assert np.abs(out - want).max() <= 1e-13


def test_zero_momentum_mode_is_m0():
    # the 1/xi weight sits in the Wilson diagonal as well as the temporal hop
    dims = [2, 2, 2, 4]
    V = lattice.volume(dims)
    op = WilsonOp(synth.unit_gauge(dims), dims, 0.123, 3.5)
    v = np.ones((V, 12, 1), dtype=complex)
    assert np.abs(op.apply(v) - 0.123 * v).max() <= 1e-15


# ---------------------------------------------------------------- P5 gauge covariance
def test_gauge_covariance():
    dims = [4, 4, 2, 4]
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.6, 0, config=13)
    G = synth.random_gauge_transform(V, config=13)
    nbr = lattice.neighbors(dims)
    UG = np.empty_like(U)
    for mu in range(4):
        UG[:, mu] = G @ U[:, mu] @ np.conj(np.swapaxes(G[nbr[:, 2 * mu]], -1, -2))
    v = as_columns(synth.gaussian_rhs(2, V, config=13))
    Gf = lambda w: np.einsum("xab,xsbc->xsac", G, w.reshape(V, 4, 3, -1)).reshape(V, 12, -1)
    op, opG = WilsonOp(U, dims, -0.1, 1.0), WilsonOp(UG, dims, -0.1, 1.0)
    assert np.abs(opG.apply(Gf(v)) - Gf(op.apply(v))).max() <= 1e-13


def test_synthetic_links_are_su3():
    U = synth.gauge_field([4, 4, 4, 4], 0.25, 3, config=2)
    M = U.reshape(-1, 3, 3)
    assert np.abs(np.conj(np.swapaxes(M, -1, -2)) @ M - np.eye(3)).max() <= 1e-14
    assert np.abs(np.linalg.det(M) - 1).max() <= 1e-14


def test_stencil_form_matches_hopping_form():
    dims = [2, 4, 2, 4]
    V = lattice.volume(dims)
    op = WilsonOp(synth.gauge_field(dims, 0.4, 1, config=14), dims, -0.5, 2.0)
    st = op.to_stencil()
    v = as_columns(synth.gaussian_rhs(3, V, config=14))
    assert np.abs(st.apply(v) - op.apply(v)).max() <= 1e-14
    sites = np.array([0, 5, V - 1])
    assert np.abs(op.apply_at(v, sites) - op.apply(v)[sites]).max() <= 1e-14
