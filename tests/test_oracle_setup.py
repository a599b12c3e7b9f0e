"""Pins of the oracle's smoother, chiral SVD truncation, prolongator and Galerkin product.

References used: MR orthogonality identities, Eckart-Young, the Gram spectrum,
gamma5 P = P sigma3, brute-force dense P^dag D P, sigma3-hermiticity of D_c,
unitary similarity at full rank (k = N_r, free-field closed form), the
conventional (QR) span at k = m', and gauge covariance of the whole setup.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import synth
from oracle import chiral, galerkin, lattice, mg, mr
from oracle.gamma import gamma5_full
from oracle.stencil import StencilOp, as_columns
from oracle.wilson import WilsonOp, free_field_eigenvalues


def spectrum_distance(a, b):
    """Largest distance between two multisets of eigenvalues under the best matching."""
    cost = np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :])
    r, c = linear_sum_assignment(cost)
    return cost[r, c].max()


def _c1(eps=0.3, m0=-0.4, dims=(4, 4, 4, 4), config=1):
    dims = list(dims)
    U = synth.gauge_field(dims, eps, 0, config=config)
    return WilsonOp(U, dims, m0, 1.0)


def _vectors(op, m, config=1, level=0):
    return as_columns(synth.gaussian_vectors(m, op.V, op.N, config=config, level=level))


# ---------------------------------------------------------------- P6 MR smoother
def test_mr_smoother_identities():
    op = _c1()
    psi0 = _vectors(op, 4)
    hist = []
    psi = mr.mr_null(op, psi0, 20, history=hist)
    h = np.array(hist)
    assert (np.diff(h, axis=0) <= 1e-12 * h[:-1]).all()  # residual never grows
    # final residual is -D psi (recursion consistent with the definition)
    r_direct = -op.apply(psi)
    assert np.allclose(np.sqrt(mr.cdot(r_direct, r_direct).real), h[-1], rtol=1e-10)
    # one step: the new residual is orthogonal to q = D r
    r = -op.apply(psi0)
    q = op.apply(r)
    a = mr.cdot(q, r) / mr.cdot(q, q).real
    rn = r - a * q
    assert np.abs(mr.cdot(q, rn)).max() <= 1e-13 * np.abs(mr.cdot(q, r)).max()
    psi1 = mr.mr_null(op, psi0, 1)
    assert np.abs(-op.apply(psi1) - rn).max() <= 1e-13 * np.abs(rn).max()


def test_mr_zero_residual_is_fixed_point():
    op = _c1()
    b = _vectors(op, 1)
    e = mr.mr_solve(op, op.apply(b), b, 3)  # exact start: alpha guarded to 0
    assert np.isfinite(e).all() and np.abs(e - b).max() <= 1e-13


# ---------------------------------------------------------------- P7 SVD
def test_truncated_svd_eckart_young_and_phase():
    rng = np.random.default_rng(3)
    nr, m, k = 96, 16, 8
    # decaying spectrum like smoothed test vectors
    Q1 = np.linalg.qr(rng.standard_normal((nr, m)) + 1j * rng.standard_normal((nr, m)))[0]
    Q2 = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))[0]
    s_true = np.logspace(0, -3, m)
    A = (Q1 * s_true) @ Q2.conj().T
    Uk, s = chiral.truncated_svd(A, k)
    assert np.allclose(s, s_true, rtol=1e-12, atol=1e-15 * s_true[0])
    assert (np.diff(s) <= 0).all()
    # spectrum also from the Gram matrix (a different computation)
    g = np.sqrt(np.sort(np.linalg.eigvalsh(A.conj().T @ A))[::-1].clip(0))
    assert np.abs(g - s).max() <= 1e-12 * s[0]
    assert np.abs(Uk.conj().T @ Uk - np.eye(k)).max() <= 1e-14
    # Eckart-Young: best rank-k error is the tail of the spectrum
    E = A - Uk @ (Uk.conj().T @ A)
    assert np.isclose(np.linalg.norm(E) ** 2, np.sum(s[k:] ** 2), rtol=1e-10)
    # U_k spans the top-k left singular space: A^dag u_i = sigma_i v_i is consistent
    # and the phase convention makes <u_i, sum_j a_j> real positive
    t = Uk.conj().T @ A.sum(axis=1)
    assert np.all(t.real > 0) and np.abs(t.imag).max() <= 1e-13 * np.abs(t).max()


def test_truncation_rank_errors():
    A = np.ones((6, 4), dtype=complex)
    with pytest.raises(ValueError):
        chiral.prolongator_blocks(A[None, None].repeat(2, 1), 5)


# ---------------------------------------------------------------- P8 prolongator structure
def test_prolongator_chirality_and_orthonormality():
    op = _c1()
    block = [2, 2, 2, 2]
    psi = mr.normalize_columns(mr.mr_null(op, _vectors(op, 16), 5))
    A = chiral.chiral_blocks(psi, op.dims, block)
    # the chiral split takes spins 1,2 (alpha=0) and 3,4 (alpha=1) of each site
    bs = lattice.block_sites(op.dims, block)
    j, ll = 3, 5
    x = bs[j, ll]
    assert np.array_equal(A[j, 0, 6 * ll:6 * ll + 6], psi[x, 0:6])
    assert np.array_equal(A[j, 1, 6 * ll:6 * ll + 6], psi[x, 6:12])
    assert np.array_equal(chiral.unblock(A, op.dims, block), psi)
    Pb, S = chiral.prolongator_blocks(A, 8)
    P = chiral.prolongator_dense(Pb, op.dims, block, 12)
    assert P.shape == (12 * op.V, 2 * 8 * 16)
    g5 = np.kron(np.eye(op.V), gamma5_full())
    s3 = np.kron(np.eye(16), np.diag([1.0] * 8 + [-1.0] * 8))
    assert np.array_equal(g5 @ P, P @ s3)  # exactly: off-chirality entries are 0
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() <= 1e-14
    # restriction / prolongation agree with the dense matrix
    v = _vectors(op, 2, level=3)
    vc = chiral.restrict(Pb, v, op.dims, block)
    assert np.abs(vc.reshape(-1, 2) - P.conj().T @ v.reshape(-1, 2)).max() <= 1e-14
    assert np.abs(chiral.prolong(Pb, vc, op.dims, block).reshape(-1, 2) - P @ vc.reshape(-1, 2)).max() <= 1e-14


# ---------------------------------------------------------------- P9/P10 Galerkin
@pytest.mark.parametrize("dims,block", [
    ([4, 4, 4, 4], [2, 2, 2, 2]),   # coarse extent 2 in every direction
    ([4, 2, 4, 2], [2, 2, 2, 1]),   # coarse extent 1 in y (hops go to X), 2 elsewhere
    ([6, 2, 2, 4], [2, 2, 2, 2]),   # coarse extent 3 in x
])
def test_galerkin_dense_and_sigma3_hermiticity(dims, block):
    op = _c1(dims=dims, config=21)
    psi = mr.normalize_columns(mr.mr_null(op, _vectors(op, 12, config=21), 6))
    A = chiral.chiral_blocks(psi, dims, block)
    Pb, _ = chiral.prolongator_blocks(A, 5)
    Dc = galerkin.galerkin(op, Pb, block)
    P = chiral.prolongator_dense(Pb, dims, block, 12)
    ref = P.conj().T @ op.dense() @ P
    assert np.abs(Dc.dense() - ref).max() <= 1e-13 * np.abs(ref).max()
    s3 = np.diag(Dc.chirality())
    nbr = Dc.nbr
    for j in range(Dc.V):
        assert np.abs(Dc.X[j].conj().T - s3 @ Dc.X[j] @ s3).max() <= 1e-14
        for mu in range(4):
            jp = nbr[j, 2 * mu]
            assert np.abs(Dc.Ym[mu, jp] - s3 @ Dc.Yp[mu, j].conj().T @ s3).max() <= 1e-14
    # sampled blocks reproduce the full computation
    X, Yp, Ym = galerkin.galerkin(op, Pb, block, blocks=[0, Dc.V - 1])
    assert np.array_equal(X[1], Dc.X[-1]) and np.array_equal(Ym[:, 0], Dc.Ym[:, 0])


# ---------------------------------------------------------------- P11 full basis
def test_full_rank_basis_gives_unitary_similarity_free_field():
    dims, block = [2, 2, 2, 4], [2, 2, 2, 2]   # two blocks, N_r = 6*16 = 96
    op = WilsonOp(synth.unit_gauge(dims), dims, -0.3, 1.0)
    psi = mr.normalize_columns(mr.mr_null(op, _vectors(op, 96, config=31), 2))
    Pb, _ = chiral.prolongator_blocks(chiral.chiral_blocks(psi, dims, block), 96)
    Dc = galerkin.galerkin(op, Pb, block)
    a = np.linalg.eigvals(Dc.dense())
    assert spectrum_distance(a, free_field_eigenvalues(dims, -0.3, 1.0)) <= 1e-10


# ---------------------------------------------------------------- P12 k = m' vs conventional
def test_k_equals_m_reproduces_conventional_span():
    op = _c1(config=41)
    block = [2, 2, 2, 2]
    psi = mr.normalize_columns(mr.mr_null(op, _vectors(op, 12, config=41), 10))
    A = chiral.chiral_blocks(psi, op.dims, block)
    Pb, _ = chiral.prolongator_blocks(A, 12)
    Qb = chiral.conventional_blocks(A)
    for j in range(A.shape[0]):
        for a in range(2):
            Pi1 = Pb[j, a] @ Pb[j, a].conj().T
            Pi2 = Qb[j, a] @ Qb[j, a].conj().T
            assert np.abs(Pi1 - Pi2).max() <= 1e-13
    e1 = np.linalg.eigvals(galerkin.galerkin(op, Pb, block).dense())
    e2 = np.linalg.eigvals(galerkin.galerkin(op, Qb, block).dense())
    assert spectrum_distance(e1, e2) <= 1e-11


# ---------------------------------------------------------------- P5 setup covariance
def test_setup_is_gauge_covariant():
    dims, block = [4, 4, 4, 4], [2, 2, 2, 2]
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.3, 0, config=51)
    G = synth.random_gauge_transform(V, config=51)
    nbr = lattice.neighbors(dims)
    UG = np.empty_like(U)
    for mu in range(4):
        UG[:, mu] = G @ U[:, mu] @ np.conj(np.swapaxes(G[nbr[:, 2 * mu]], -1, -2))
    Gf = lambda w: np.einsum("xab,xsbc->xsac", G, w.reshape(V, 4, 3, -1)).reshape(V, 12, -1)
    op, opG = WilsonOp(U, dims, -0.4, 1.0), WilsonOp(UG, dims, -0.4, 1.0)
    v0 = as_columns(synth.gaussian_vectors(16, V, 12, config=51))
    L1 = mg.mg_setup(op, [16], [8], [block], [20], [v0])
    L2 = mg.mg_setup(opG, [16], [8], [block], [20], [Gf(v0)])
    P1 = chiral.site_blocks(L1[0].Pb, dims, block, 12)
    P2 = chiral.site_blocks(L2[0].Pb, dims, block, 12)
    assert np.abs(P2 - Gf(P1)).max() <= 1e-12
    assert np.abs(L1[1].op.X - L2[1].op.X).max() <= 1e-12
    assert np.abs(L1[1].op.Yp - L2[1].op.Yp).max() <= 1e-12


# ---------------------------------------------------------------- three levels
def test_three_level_galerkin_dense():
    dims = [4, 4, 4, 4]
    op = _c1(config=61)
    iv = mg.init_vectors_for([dims, [2, 2, 2, 2]], [12, 16], [16, 24], 61, synth.gaussian_vectors)
    L = mg.mg_setup(op, [16, 24], [8, 10], [[2, 2, 2, 2], [2, 2, 2, 2]], [10, 10], iv)
    D1, D2 = L[1].op, L[2].op
    assert D2.V == 1 and D2.N == 20
    P1 = chiral.prolongator_dense(L[1].Pb, D1.dims, [2, 2, 2, 2], 16)
    ref = P1.conj().T @ D1.dense() @ P1
    assert np.abs(D2.dense() - ref).max() <= 1e-13 * np.abs(ref).max()
    s3 = np.diag(D2.chirality())
    assert np.abs(ref.conj().T - s3 @ ref @ s3).max() <= 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------- coarse test vectors
def test_coarse_test_vectors_are_sigma_vdag():
    """Sigma_k V_k^dag = U_k^dag A (Sec. 3, after Eq. (5)): per block and chirality its
    rows are orthogonal with norms sigma_1..sigma_k of LAPACK's singular values of A,
    and U_k (Sigma_k V_k^dag) leaves exactly the discarded tail, sum_{i>k} sigma_i^2
    (Eckart-Young).  The coarse field puts chirality a in components a k .. a k + k - 1,
    and it equals the restriction P^dag psi of the same vectors."""
    op = _c1(config=5)
    block, k, m = [2, 2, 2, 2], 8, 16
    psi = mr.normalize_columns(mr.mr_null(op, _vectors(op, m, config=5), 10))
    A = chiral.chiral_blocks(psi, op.dims, block)
    Pb, _ = chiral.prolongator_blocks(A, k)
    C = chiral.coarse_test_vectors(A, Pb)
    d = A.shape[0]
    assert C.shape == (d, 2 * k, m)
    for j in range(d):
        for a in range(2):
            s = np.linalg.svd(A[j, a], compute_uv=False)
            Ca = C[j, a * k:(a + 1) * k]
            G = Ca @ Ca.conj().T
            assert np.abs(G - np.diag(s[:k] ** 2)).max() <= 1e-12 * s[0] ** 2
            tail = np.linalg.norm(A[j, a] - Pb[j, a] @ Ca) ** 2
            assert abs(tail - (s[k:] ** 2).sum()) <= 1e-12 * s[0] ** 2
    assert np.abs(C - chiral.restrict(Pb, psi, op.dims, block)).max() <= 1e-13


def test_three_level_setup_from_coarse_test_vectors():
    """With coarse_init the second step starts from the first m'_1 coarse test vectors
    of the first: with no sweeps its kept (normalised) vectors are those, and an
    m'_1 above m'_0 is refused."""
    dims = [4, 4, 4, 4]
    op = _c1(config=61)
    iv0 = _vectors(op, 16, config=61)
    L = mg.mg_setup(op, [16, 12], [8, 8], [[2, 2, 2, 2], [2, 2, 2, 2]], [10, 0], [iv0, None],
                    keep_vectors=True, coarse_init=True)
    A = chiral.chiral_blocks(L[0].vectors, dims, [2, 2, 2, 2])
    C = chiral.coarse_test_vectors(A, L[0].Pb)[:, :, :12]
    ref = mr.normalize_columns(C)
    assert np.abs(L[1].vectors - ref).max() <= 1e-14
    with pytest.raises(ValueError):
        mg.mg_setup(op, [16, 24], [8, 8], [[2, 2, 2, 2], [2, 2, 2, 2]], [10, 0], [iv0, None], coarse_init=True)
