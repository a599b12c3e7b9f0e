"""GPU parity of the chiral rank-k setup (MR smoother, chiral SVD, P, Galerkin) and
of the transfer and coarse operators, against the FP64 oracle.

Bars (plain FP64 form, same seeded inputs on both sides):
  * block / aggregate maps bit-exact;
  * smoothed, normalised test vectors: 1e-12 relative (max-norm per vector);
  * singular values: |d sigma_i| <= 1e-12 * sigma_1 (Weyl);
  * per (block, chirality) projector U_k U_k^dag: relative Frobenius error
    <= max(1e-12, 10 eps sqrt(N_r) sigma_1 / (sigma_k - sigma_{k+1})) (Wedin);
  * P columns element-wise (phase convention fixes them) with the per-column
    bound 10 eps sqrt(N_r) sigma_1 / (min gap to the neighbouring sigma);
  * coarse spectrum (basis independent); coarse links element-wise within
    2 ||D||_2 max_i ||dp_i|| (dp_i the measured difference of column i, itself
    within the column bound) and again after Procrustes alignment of the bases;
    restriction / prolongation with the tolerance the same dp implies;
  * the Galerkin identity D_c v = P^dag D P v at any size (GPU only).
Reduced-precision setup (FP32 smoother): the spread of the oracle's recursion
under FP32-sized perturbations (see _check_fp32_smoother).
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import synth
from oracle import chiral, galerkin, lattice as olat, mg as omg, mr
from oracle.stencil import as_columns, as_fields
from oracle.wilson import WilsonOp
from parity_bounds import (compare_coarse_links, compare_prolongators, fp32_setup_spread, fp32_smoother_spread,
                           wilson_norm_bound)

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _spec_dist(a, b):
    cost = np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :])
    r, c = linear_sum_assignment(cost)
    return cost[r, c].max()


def _build(crk, dims, block, m, k, n_smooth, eps=0.3, m0=-0.4, xi=1.0, config=1, form=0, n_ape=0):
    U = synth.gauge_field(dims, eps, n_ape, config=config)
    V = olat.volume(dims)
    v0 = synth.gaussian_vectors(m, V, 12, config=config, level=0)
    lat = crk.Lattice(dims, m0, xi)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[m], k=[k], block=[block], n_smooth=[n_smooth], setup_form=form,
                      init_vectors=[v0])
    op = WilsonOp(U, dims, m0, xi)
    ref = omg.mg_setup(op, [m], [k], [block], [n_smooth], [as_columns(v0)], keep_vectors=True)
    ref[0].init = as_columns(v0)
    return lat, H, op, ref


CASES = [
    # dims, block, m', k, sweeps: C1 (4^4, 2^4 blocks, m'=16 -> k=8, 20 MR)
    ([4, 4, 4, 4], [2, 2, 2, 2], 16, 8, 20),
    ([4, 2, 4, 2], [2, 2, 2, 1], 20, 8, 6),     # coarse extent 1 in y, 2 elsewhere; m' off-tile
    ([6, 4, 2, 4], [2, 2, 2, 2], 24, 16, 5),    # coarse extent 3 in x
]


@pytest.mark.parametrize("dims,block,m,k,ns", CASES)
def test_setup_fp64_matches_oracle(crk, dims, block, m, k, ns):
    print(f"setup parity dims={dims} block={block} m={m} k={k} sweeps={ns}", flush=True)
    lat, H, op, ref = _build(crk, dims, block, m, k, ns)
    L0, L1 = ref[0], ref[1]
    # maps
    j, l = olat.block_maps(dims, block)
    bm = H.block_map(0)
    assert np.array_equal(bm[:, 0], j) and np.array_equal(bm[:, 1], l)
    # smoothed, normalised vectors
    vg = H.vectors(0)
    vo = as_fields(L0.vectors)
    err = np.abs(vg - vo).max(axis=(1, 2)) / np.abs(vo).max(axis=(1, 2))
    assert err.max() <= 1e-12, err.max()
    # singular values
    sg, so = H.sigma(0), L0.sigma
    assert np.abs(sg - so).max() <= 1e-12 * so[..., 0].max()
    # projectors and every column; dcol = the columns' largest difference (2-norm)
    Pg, Po = H.prolongator(0), L0.Pb
    dcol = compare_prolongators(Pg, Po, sg, so, k)
    # coarse operator: basis-independent spectrum, and the links element-wise with
    # the tolerance the columns' difference implies (and after Procrustes alignment)
    X, Yp, Ym = H.coarse_links(0)
    from oracle.stencil import StencilOp
    Dg = StencilOp(L1.op.dims, X, Yp, Ym).dense()
    Do = L1.op.dense()
    scale = np.abs(Do).max()
    assert _spec_dist(np.linalg.eigvals(Dg), np.linalg.eigvals(Do)) <= 1e-10 * scale
    compare_coarse_links((X, Yp, Ym), (L1.op.X, L1.op.Yp, L1.op.Ym), dcol, wilson_norm_bound(-0.4, 1.0),
                         L1.op.dims, Pg, Po)
    # transfers and coarse apply against the oracle's
    V = olat.volume(dims)
    v = synth.gaussian_rhs(3, V, config=7)
    rc_g = H.restrict(0, v)
    rc_o = as_fields(chiral.restrict(Po, as_columns(v), dims, block))
    vb = np.sqrt((np.abs(v) ** 2).sum(axis=2)).max() * np.sqrt(olat.volume(block))
    assert np.abs(rc_g - rc_o).max() <= dcol * vb + 1e-12 * np.abs(rc_o).max()
    pv_g = H.prolong(0, rc_o)
    pv_o = as_fields(chiral.prolong(Po, as_columns(rc_o), dims, block))
    assert np.abs(pv_g - pv_o).max() <= dcol * np.abs(rc_o).sum(axis=2).max() + 1e-12 * np.abs(pv_o).max()
    # the coarse apply on the same input, with the GPU's own links in the oracle's stencil
    ca_g = H.coarse_apply(1, rc_o)
    ca_o = as_fields(StencilOp(L1.op.dims, X, Yp, Ym).apply(as_columns(rc_o)))
    assert np.abs(ca_g - ca_o).max() <= 1e-12 * np.abs(ca_o).max()


@pytest.mark.parametrize("k", [8, 16, 32])
def test_galerkin_identity_every_tile_height(crk, k):
    """D_c v = P^dag D P v on 8^4 with 4^4 blocks for 2k = 16, 32 and 64 (every
    tile height of the fine Galerkin kernel), all through the GPU operators in FP64."""
    dims, block = [8, 8, 8, 8], [4, 4, 4, 4]
    print("galerkin identity 8^4 k =", k, flush=True)
    U = synth.gauge_field(dims, 0.3, 1, config=9)
    lat = crk.Lattice(dims, -0.3, 1.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[32], k=[k], block=[block], n_smooth=[6], setup_form=1)
    try:
        vc = synth.gaussian_vectors(3, H.volume(1), 2 * k, config=9, level=5)
        lhs = H.coarse_apply(1, vc)
        rhs = H.restrict(0, lat.dirac_apply(H.prolong(0, vc), 0))
        err = np.abs(lhs - rhs).max() / np.abs(rhs).max()
        assert err <= 1e-12, err
    finally:
        H.close()


def test_galerkin_identity_and_sigma3_full_size(crk):
    """16^3x32, xi = 3.5, 4^4 blocks, m' = 48 -> k = 24 (the anisotropic workload), FP32 smoother."""
    dims, block = [16, 16, 16, 32], [4, 4, 4, 4]
    print("galerkin identity 16^3x32", flush=True)
    U = synth.gauge_field(dims, 0.2, 3, config=2)
    lat = crk.Lattice(dims, -0.05, 3.5)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[48], k=[24], block=[block], n_smooth=[20], setup_form=1)
    Vc, N = H.volume(1), 48
    vc = synth.gaussian_vectors(4, Vc, N, config=2, level=5)
    # D_c v  vs  P^dag D P v, all on the GPU (FP64 operators)
    lhs = H.coarse_apply(1, vc)
    Pv = H.prolong(0, vc)
    rhs = H.restrict(0, lat.dirac_apply(Pv, 0))
    err = np.abs(lhs - rhs).max() / np.abs(rhs).max()
    assert err <= 1e-12, err
    # sigma3-hermiticity of the stored links
    X, Yp, Ym = H.coarse_links(0)
    s3 = np.diag([1.0] * 24 + [-1.0] * 24)
    nbr = olat.neighbors(H.dims[1])
    scale = np.abs(X).max()
    for jj in range(0, Vc, 37):
        assert np.abs(X[jj].conj().T - s3 @ X[jj] @ s3).max() <= 1e-12 * scale
        for mu in range(4):
            assert np.abs(Ym[mu, nbr[jj, 2 * mu]] - s3 @ Yp[mu, jj].conj().T @ s3).max() <= 1e-12 * scale
    # P^dag P = 1 per block and singular values descending
    P = H.prolongator(0)
    G = np.einsum("jari,jarl->jail", P.conj(), P)
    assert np.abs(G - np.eye(24)).max() <= 1e-12
    s = H.sigma(0)
    assert (np.diff(s, axis=-1) <= 1e-15).all()
    t = H.timing(0)
    print("setup timing", t, flush=True)


def _check_fp32_smoother(H, op, ref, block, k, n_smooth, tag):
    """FP32 smoother, FP64 SVD/Galerkin against the FP64 oracle.  Bounds from the
    oracle's own recursion under FP32-sized perturbations (parity_bounds.
    fp32_smoother_spread: n_terms u32 per operator entry, 2 u32 per update):
    vectors within that spread, singular values within 10 times theirs."""
    dv, ds = fp32_smoother_spread(op, ref[0].init, n_smooth, block, k)
    vg = H.vectors(0)
    vo = as_fields(ref[0].vectors)
    err = (np.abs(vg - vo).max(axis=(1, 2)) / np.abs(vo).max(axis=(1, 2))).max()
    serr = np.abs(H.sigma(0) - ref[0].sigma).max()
    print(f"fp32 smoother {tag}: vector error {err:.3g} (bound {dv:.3g}), sigma error {serr:.3g} "
          f"(bound {10 * ds:.3g})", flush=True)
    assert err <= dv
    assert serr <= 10 * ds


def test_setup_fp32_smoother_bounds(crk):
    dims, block = [4, 4, 4, 4], [2, 2, 2, 2]
    lat, H, op, ref = _build(crk, dims, block, 16, 8, 20, form=1)
    _check_fp32_smoother(H, op, ref, block, 8, 20, "2^4 blocks")


def test_setup_fp32_smoother_4x4_blocks(crk):
    """The FP32 smoother on the block-staged fine operator (4^4 blocks, block-major
    order, MR partial sums fused into the operator launch).  Extent 4 in y and t
    puts one block along them (neighbours wrap into the block)."""
    dims, block = [8, 4, 8, 4], [4, 4, 4, 4]
    print("fp32 smoother, 4^4 blocks", dims, flush=True)
    lat, H, op, ref = _build(crk, dims, block, 16, 8, 20, form=1, m0=-0.2)
    _check_fp32_smoother(H, op, ref, block, 8, 20, "4^4 blocks")


def test_setup_rejects_bad_parameters(crk):
    lat = crk.Lattice([4, 4, 4, 4], -0.4, 1.0)
    lat.load_gauge(synth.gauge_field([4, 4, 4, 4], 0.3, 0, config=1))
    with pytest.raises(crk.CrkError):
        crk.Hierarchy(lat, m_prime=[16], k=[12], block=[[2, 2, 2, 2]], n_smooth=[2])  # k not multiple of 8
    with pytest.raises(crk.CrkError):
        crk.Hierarchy(lat, m_prime=[16], k=[8], block=[[3, 2, 2, 2]], n_smooth=[2])   # block does not divide
    with pytest.raises(crk.CrkError):
        crk.Hierarchy(lat, m_prime=[8], k=[16], block=[[2, 2, 2, 2]], n_smooth=[2])   # k > m'


def test_three_level_setup_matches_oracle(crk):
    """4^4 -> 2^4 blocks -> 2^4 blocks: level-2 coarse operator of the recursion (sigma_3 chirality)."""
    dims = [4, 4, 4, 4]
    U = synth.gauge_field(dims, 0.3, 0, config=61)
    iv0 = synth.gaussian_vectors(16, 256, 12, config=61, level=0)
    iv1 = synth.gaussian_vectors(24, 16, 16, config=61, level=1)
    lat = crk.Lattice(dims, -0.4, 1.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[16, 24], k=[8, 16], block=[[2, 2, 2, 2], [2, 2, 2, 2]], n_smooth=[10, 10],
                      setup_form=0, init_vectors=[iv0, iv1])
    op = WilsonOp(U, dims, -0.4, 1.0)
    ref = omg.mg_setup(op, [16, 24], [8, 16], [[2, 2, 2, 2], [2, 2, 2, 2]], [10, 10],
                       [as_columns(iv0), as_columns(iv1)], keep_vectors=True)
    # level-1 smoothed vectors and singular values
    v1 = H.vectors(1)
    vo = as_fields(ref[1].vectors)
    err = (np.abs(v1 - vo).max(axis=(1, 2)) / np.abs(vo).max(axis=(1, 2))).max()
    assert err <= 1e-11, err
    assert np.abs(H.sigma(1) - ref[1].sigma).max() <= 1e-11 * ref[1].sigma.max()
    # level-2 operator: spectrum (basis independent) and sigma3-hermiticity
    from oracle.stencil import StencilOp
    X, Yp, Ym = H.coarse_links(1)
    D2 = StencilOp(ref[2].op.dims, X, Yp, Ym).dense()
    D2o = ref[2].op.dense()
    sc = np.abs(D2o).max()
    assert _spec_dist(np.linalg.eigvals(D2), np.linalg.eigvals(D2o)) <= 1e-10 * sc
    s3 = np.diag([1.0] * 16 + [-1.0] * 16)
    assert np.abs(D2.conj().T - s3 @ D2 @ s3).max() <= 1e-12 * sc
    # level-1 -> level-2 Galerkin identity on the GPU operators
    vc = synth.gaussian_vectors(3, 1, 32, config=62, level=0)
    lhs = H.coarse_apply(2, vc)
    rhs = H.restrict(1, H.coarse_apply(1, H.prolong(1, vc)))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("form", [0, 1])
def test_coarse_test_vectors_start_the_second_step(crk, form):
    """coarse_init: the second coarsening step starts from P^dag of the first m'_1
    normalised fine test vectors, the coarse test vectors Sigma_k V_k^dag of
    Sec. 3 (after Eq. (5)).  With no sweeps on the second step its kept vectors
    are those (the oracle computes them from its SVD blocks); with sweeps the
    level-2 singular values follow the oracle's.  FP64 setup to 1e-11; FP32
    within the spread of the oracle's two-step setup under FP32-sized
    perturbations (parity_bounds.fp32_setup_spread), singular values within 10
    times theirs."""
    dims = [4, 4, 4, 4]
    U = synth.gauge_field(dims, 0.3, 0, config=61)
    iv0 = synth.gaussian_vectors(16, 256, 12, config=61, level=0)
    lat = crk.Lattice(dims, -0.4, 1.0)
    lat.load_gauge(U)
    op = WilsonOp(U, dims, -0.4, 1.0)
    blocks = [[2, 2, 2, 2], [2, 2, 2, 2]]
    for ns in ([10, 0], [10, 6]):
        H = crk.Hierarchy(lat, m_prime=[16, 12], k=[8, 8], block=blocks, n_smooth=ns, setup_form=form,
                          init_vectors=[iv0, None], coarse_init=True)
        ref = omg.mg_setup(op, [16, 12], [8, 8], blocks, ns, [as_columns(iv0), None], keep_vectors=True,
                           coarse_init=True)
        if form == 0:
            tol, stol = 1e-11, 1e-11 * ref[1].sigma.max()
        else:
            (_, _), (dv, ds) = fp32_setup_spread(op, [as_columns(iv0), None], [16, 12], ns, blocks, [8, 8])
            tol, stol = dv, 10 * ds
        v1 = H.vectors(1)
        vo = as_fields(ref[1].vectors)
        err = (np.abs(v1 - vo).max(axis=(1, 2)) / np.abs(vo).max(axis=(1, 2))).max()
        serr = np.abs(H.sigma(1) - ref[1].sigma).max()
        print(f"coarse_init form {form} sweeps {ns}: vector error {err:.3g} (bound {tol:.3g}), sigma error "
              f"{serr:.3g} (bound {stol:.3g})", flush=True)
        assert err <= tol, (ns, err)
        assert serr <= stol
        H.close()
    with pytest.raises(crk.CrkError):
        crk.Hierarchy(lat, m_prime=[16, 24], k=[8, 8], block=blocks, n_smooth=[2, 2], init_vectors=[iv0, None],
                      coarse_init=True)


def test_chunked_smoother_and_batched_svd_equal_full(crk):
    """Smoothing the fine-level test vectors in chunks and running the block SVDs
    in batches (what the library does when device memory is short) gives the same
    hierarchy bit for bit: every vector runs its own recursion with reductions
    that do not depend on the other vectors, and every block is factorised alone."""
    dims, block = [4, 4, 4, 4], [2, 2, 2, 2]
    U = synth.gauge_field(dims, 0.3, 0, config=1)
    v0 = synth.gaussian_vectors(16, 256, 12, config=1, level=0)
    lat = crk.Lattice(dims, -0.4, 1.0)
    lat.load_gauge(U)
    out = []
    for chunk, batch in ((0, 0), (8, 0), (5, 3), (0, 1)):
        H = crk.Hierarchy(lat, m_prime=[16], k=[8], block=[block], n_smooth=[20], setup_form=crk.FORM_FP64,
                          init_vectors=[v0], smooth_chunk=chunk, svd_batch=batch)
        out.append((H.sigma(0), H.vectors(0), H.timing(0), H.prolongator(0), H.coarse_links(0)))
        H.close()
    for s, v, t, P, X in out[1:]:
        assert np.array_equal(s, out[0][0]) and np.array_equal(v, out[0][1])
        assert np.array_equal(P, out[0][3]) and all(np.array_equal(a, b) for a, b in zip(X, out[0][4]))
    assert out[1][2]["dslash_count"] == 2 * 20 and out[2][2]["dslash_count"] == 4 * 20


def test_deferred_psi_updates_equal_per_sweep(crk):
    """The fine-level smoother may apply the psi updates of several sweeps in one
    pass over psi (each sweep still forms its residual): per element the fused
    multiply-adds are those of one update per sweep, in the same order, so the
    hierarchy is bitwise the same for every depth, with ragged last groups
    (20 sweeps in groups of 3), chunked vectors, and both setup precisions."""
    dims, block = [4, 4, 4, 8], [2, 2, 2, 2]
    U = synth.gauge_field(dims, 0.3, 0, config=4)
    v0 = synth.gaussian_vectors(16, 512, 12, config=4, level=0)
    lat = crk.Lattice(dims, -0.4, 1.0)
    lat.load_gauge(U)
    for form in (crk.FORM_FP64, crk.FORM_FP32):
        for sweeps in (20, 7, 1):
            out = []
            for defer, chunk in ((1, 0), (2, 0), (3, 0), (8, 0), (0, 0), (3, 5)):
                H = crk.Hierarchy(lat, m_prime=[16], k=[8], block=[block], n_smooth=[sweeps], setup_form=form,
                                  init_vectors=[v0], smooth_chunk=chunk, smooth_defer=defer)
                out.append((H.vectors(0), H.sigma(0), H.coarse_links(0)))
                H.close()
            for v, s, X in out[1:]:
                assert np.array_equal(v, out[0][0]), (form, sweeps)
                assert np.array_equal(s, out[0][1]) and all(np.array_equal(a, b) for a, b in zip(X, out[0][2]))
    with pytest.raises(crk.CrkError):
        crk.Hierarchy(lat, m_prime=[16], k=[8], block=[block], n_smooth=[4], init_vectors=[v0], smooth_defer=9)
    lat.close()
