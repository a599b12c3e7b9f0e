"""Error bounds and comparisons shared by the GPU parity tests.

Every bound here is derived from the arithmetic the kernels do, with the unit
roundoffs u of the storage and accumulation precisions; the docstrings give
the derivation.  Nothing here runs on the GPU.
"""
import numpy as np

from oracle.stencil import StencilOp, as_columns, as_fields

EPS = np.finfo(float).eps
U64 = 2.0 ** -53
U32 = 2.0 ** -24
U16 = 2.0 ** -11
SUB16 = 2.0 ** -25  # half the spacing of binary16 subnormals (2^-24): absolute RNE error below 2^-14


def coarse_apply_bounds(X, Yp, Ym, dims, v):
    """Element-wise forward-error bounds of the coarse operator
    (D_c v)(j) = X(j) v(j) + sum_mu [Y_{+mu}(j) v(j+mu) + Y_{-mu}(j) v(j-mu)]
    in its three forms, for input fields v [nrhs, Vc, N].

    Each output entry is a sum of n = 9 N complex products.  With
    S = sum_j |A_ij| |v_j| (the stencil of |links| applied to |v|):

    * FP64 / FP32 links and vectors, accumulation in the same precision:
      |err| <= sqrt(2) (n + 4) u S  (complex products and an n-term sum).
    * FP16S: the kernel stores each link block as binary16 of a/s (one FP32
      scale s per block) and, per link and RHS, rounds the neighbour's vector
      to binary16 of v/w with w the largest |Re|, |Im| of that neighbour site's
      column.  Each stored factor is off by at most u16 of itself, or by
      2^-25 of its scale below the normal range, so one real product is off by
      at most (2 u16 + u16^2) |a||v| + 2^-25 (1 + u16) (w |a| + s |v|) + 2^-50 s w.
      The products of binary16 numbers are exact in FP32; the MFMA sums, the
      rescaling by s w and the sum over the nine links add
      sqrt(2) (n + 6) u32 of the magnitudes.  With W_j = w of the site j's
      column broadcast over its components:
      |err| <= (2 u16 + u16^2) S + sqrt(2) (n + 6) u32 (1 + 3 u16) S
               + 2^-25 (1 + u16) (stencil(|A|) W + s_max sum|v|) + 2^-50 s_max W_max 9N.
    Returns (bounds dict form -> array like v, S, n).
    """
    N = X.shape[-1]
    n = 9 * N
    op_abs = StencilOp(dims, np.abs(X), np.abs(Yp), np.abs(Ym))
    va = np.abs(v)
    S = as_fields(op_abs.apply(as_columns(va))).real
    w = np.maximum(np.abs(v.real), np.abs(v.imag)).max(axis=2, keepdims=True)  # [nrhs, Vc, 1]
    Wf = np.broadcast_to(w, v.shape)
    SW = as_fields(op_abs.apply(as_columns(Wf))).real
    smax = max(np.abs(X).max(), np.abs(Yp).max(), np.abs(Ym).max())
    vsum = va.sum(axis=(1, 2))[:, None, None]
    b16 = ((2 * U16 + U16 ** 2) * S + np.sqrt(2) * (n + 6) * U32 * (1 + 3 * U16) * S
           + SUB16 * (1 + U16) * (SW + smax * vsum) + 2.0 ** -50 * smax * w.max() * n)
    return {0: np.sqrt(2) * (n + 4) * U64 * S, 1: np.sqrt(2) * (n + 4) * U32 * S, 2: b16}, S, n


def wedin_bound(s, k, nr):
    """Projector error bound of a rank-k truncation computed to backward error
    10 eps sqrt(N_r) sigma_1 (Wedin's sin-theta theorem)."""
    gap = s[k - 1] - (s[k] if k < s.size else 0.0)
    return max(1e-12, 10 * EPS * np.sqrt(nr) * s[0] / gap)


def column_bound(s, i, nr):
    """Bound on a single singular vector: backward error over the distance to
    the neighbouring singular values."""
    neigh = [abs(s[i] - s[i - 1]) if i > 0 else np.inf, abs(s[i] - s[i + 1]) if i + 1 < s.size else s[i]]
    return max(1e-12, 10 * EPS * np.sqrt(nr) * s[0] / min(neigh))


def procrustes(Po, Pg):
    """Unitary W (k x k) minimising ||Po W - Pg||_F: the polar factor of Po^dag Pg."""
    u, _, vh = np.linalg.svd(Po.conj().T @ Pg)
    return u @ vh


def wilson_norm_bound(m0, xi):
    """||D||_2 <= |m0 + sum w| + sum_mu w_mu: each direction's two hops
    -w/2 [(1 - g) U T_+ + (1 + g) U^dag T_-] have norm <= w (the two projectors
    (1 -+ g)/2 are orthogonal)."""
    w = np.array([1.0, 1.0, 1.0, 1.0 / xi])
    return abs(m0 + w.sum()) + w.sum()


def aligned_links(X, Yp, Ym, Wb, nbr):
    """Express coarse links in another basis: with W_j = diag(W_{j,0}, W_{j,1})
    per coarse site, X'(j) = W_j^dag X(j) W_j and Y'_{+-mu}(j) = W_j^dag Y(j) W_{j+-mu}."""
    d = X.shape[0]
    Wd = np.zeros_like(X)
    k = Wb.shape[-1]
    for j in range(d):
        Wd[j, :k, :k] = Wb[j, 0]
        Wd[j, k:, k:] = Wb[j, 1]
    WdH = np.conj(np.swapaxes(Wd, -1, -2))
    Xa = WdH @ X @ Wd
    Ypa = np.stack([WdH @ Yp[mu] @ Wd[nbr[:, 2 * mu]] for mu in range(4)])
    Yma = np.stack([WdH @ Ym[mu] @ Wd[nbr[:, 2 * mu + 1]] for mu in range(4)])
    return Xa, Ypa, Yma


def compare_prolongators(Pg, Po, sg, so, k):
    """Singular values, projectors (Wedin) and every column (phase convention)
    of two sets of prolongator blocks [d, 2, N_r, k].  Returns the largest
    column difference in 2-norm, max_i ||Pg[:, i] - Po[:, i]||_2, which bounds
    what the columns' difference does to every quantity built from P."""
    nr = Po.shape[2]
    assert np.abs(sg - so).max() <= 1e-12 * so[..., 0].max(), np.abs(sg - so).max() / so[..., 0].max()
    dcol = 0.0
    for jj in range(Po.shape[0]):
        for a in range(2):
            s = so[jj, a]
            bound = wedin_bound(s, k, nr)
            Pi_g = Pg[jj, a] @ Pg[jj, a].conj().T
            Pi_o = Po[jj, a] @ Po[jj, a].conj().T
            e = np.linalg.norm(Pi_g - Pi_o) / np.linalg.norm(Pi_o)
            assert e <= bound, (jj, a, e, bound)
            assert np.abs(Pg[jj, a].conj().T @ Pg[jj, a] - np.eye(k)).max() <= 1e-13
            for i in range(k):
                cb = column_bound(s, i, nr)
                ce = np.abs(Pg[jj, a][:, i] - Po[jj, a][:, i]).max()
                assert ce <= cb, (jj, a, i, ce, cb)
                dcol = max(dcol, float(np.linalg.norm(Pg[jj, a][:, i] - Po[jj, a][:, i])))
    return dcol


def compare_coarse_links(gpu_links, ora_links, dcol, normD, cdims, Pg=None, Po=None):
    """Coarse links of the GPU hierarchy against the oracle's, element by element.

    D_c(a, b) = p_a^dag D p_b over a block (hop part for Y), so replacing the
    columns p by p + dp changes an entry by at most 2 ||D||_2 max ||dp||_2
    (unit columns) plus the FP64 rounding of the products.  When both P are
    given, the links are also compared after Procrustes alignment of the
    oracle's basis onto the GPU's per (block, chirality): that comparison is
    independent of the basis chosen inside the kept subspace.
    Returns the largest element-wise difference relative to the largest link entry."""
    from oracle import lattice as olat
    Xg, Ypg, Ymg = gpu_links
    Xo, Ypo, Ymo = ora_links
    scale = max(np.abs(Xo).max(), np.abs(Ypo).max(), np.abs(Ymo).max())
    tol = 2 * normD * dcol + 1e-12 * scale
    err = max(np.abs(Xg - Xo).max(), np.abs(Ypg - Ypo).max(), np.abs(Ymg - Ymo).max())
    assert err <= tol, (err, tol)
    if Pg is not None:
        Wb = np.stack([[procrustes(Po[j, a], Pg[j, a]) for a in range(2)] for j in range(Po.shape[0])])
        nbr = olat.neighbors(cdims)
        Xa, Ypa, Yma = aligned_links(Xo, Ypo, Ymo, Wb, nbr)
        # ||Po W - Pg||_2 per block bounds the aligned difference the same way
        dal = max(float(np.linalg.norm(Po[j, a] @ Wb[j, a] - Pg[j, a], 2))
                  for j in range(Po.shape[0]) for a in range(2))
        tol_a = 2 * normD * dal + 1e-12 * scale
        err_a = max(np.abs(Xg - Xa).max(), np.abs(Ypg - Ypa).max(), np.abs(Ymg - Yma).max())
        assert err_a <= tol_a, (err_a, tol_a)
    return err / scale


def fp32_smoother_spread(op, psi0, n_iter, blocks, k, n_terms=10, replays=3, seed=0):
    """Expected spread of the FP32 smoother's normalised test vectors and of the
    singular values built from them, from the oracle's own recursion with FP32
    rounding modelled as relative perturbations: every operator output entry (a
    sum of about n_terms complex products) is multiplied by 1 + n_terms u32 xi,
    every update psi += a r, r -= a q and the inner products by 1 + 2 u32 xi,
    with xi independent complex normals of unit size.  The MR steps, which
    feed alpha back into the vectors, amplify these as the kernels' roundings
    would; the largest deviation over a few replays from the unperturbed
    recursion (per vector, max-norm, relative) and of the singular values
    (absolute) are returned.  The smoother tests allow the vector spread itself
    and 10 times the singular-value spread (the SVD of the GPU path runs in FP64
    on vectors whose rounding differs from the replays' model)."""
    levels = fp32_setup_spread(op, [psi0], [None], [n_iter], [blocks], [k], n_terms=n_terms, replays=replays,
                               seed=seed)
    return levels[0]


def fp32_setup_spread(op, init, m_prime, n_smooth, blocks, k, n_terms=10, replays=3, seed=0):
    """fp32_smoother_spread through a whole (coarse_init) setup: each step's MR
    smoother runs under the same perturbations on that step's operator, and a
    step with init[l] None starts from the first m_prime[l] coarse test vectors
    of the (perturbed) step before it.  Returns [(vector spread, sigma spread)]
    per step."""
    from oracle import chiral, galerkin, mr

    rng = np.random.default_rng(seed)

    def pert(x, rel):
        xi = (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)) / np.sqrt(2.0)
        return x * (1.0 + rel * xi)

    def smooth(o, psi0, n_iter, perturb):
        p = (lambda x, rel: pert(x, rel)) if perturb else (lambda x, rel: x)
        psi = np.array(psi0, dtype=np.complex128, copy=True)
        r = p(-o.apply(psi), n_terms * U32)
        for _ in range(int(n_iter)):
            q = p(o.apply(r), n_terms * U32)
            qq = mr.cdot(q, q).real * (1.0 + (2 * U32 * rng.standard_normal(q.shape[-1]) if perturb else 0.0))
            qr = mr.cdot(q, r)
            a = np.where(qq > 0, qr / np.where(qq > 0, qq, 1.0), 0.0)
            psi = p(psi + a * r, 2 * U32)
            r = p(r - a * q, 2 * U32)
        return mr.normalize_columns(psi)

    def run(perturb):
        out, o, coarse = [], op, None
        for l in range(len(blocks)):
            iv = init[l] if init[l] is not None else np.ascontiguousarray(coarse[:, :, :m_prime[l]])
            psi = smooth(o, iv, n_smooth[l], perturb)
            A = chiral.chiral_blocks(psi, o.dims, blocks[l])
            Pb, S = chiral.prolongator_blocks(A, k[l])
            coarse = chiral.coarse_test_vectors(A, Pb)
            out.append((psi, S))
            o = galerkin.galerkin(o, Pb, blocks[l])
        return out

    ref = run(False)
    res = [(0.0, 0.0) for _ in blocks]
    for _ in range(replays):
        got = run(True)
        for l, ((v, s), (rv, rs)) in enumerate(zip(got, ref)):
            dv = float((np.abs(v - rv).max(axis=(0, 1)) / np.abs(rv).max(axis=(0, 1))).max())
            res[l] = (max(res[l][0], dv), max(res[l][1], float(np.abs(s - rs).max())))
    return res
