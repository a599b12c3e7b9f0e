"""GPU parity of the Galerkin coarse operator on MFMA (Eq. (4)) and of the
restriction P^dag and prolongation P (Eq. (6)) in their precision forms, against
the oracle's stencil and transfers built from the same FP64 links and P.

The operator is (D_c v)(j) = X(j) v(j) + sum_mu [Y_{+mu}(j) v(j+mu) + Y_{-mu}(j) v(j-mu)]:
nine 2k x 2k blocks per coarse site.  Each output entry is an inner product of
n = 9 * 2k complex terms, so with unit roundoff u of the accumulation and
S = sum_j |A_ij| |v_j| (the oracle's stencil applied to |links| and |v|):

  * FP64 and FP32 forms: |err| <= sqrt(2) (n + 4) u S  (rounded inputs, complex
    products and the sum; standard forward bound of a dot product);
  * FP16S (binary16 links of x/s with one FP32 scale s per link block, and
    the neighbour's vector column rounded to binary16 of v/w per link and RHS,
    w its largest |Re|, |Im|; exact binary16 products, FP32 accumulation):
    both factors carry a relative rounding u16 (or 2^-25 of their scale below
    the normal range), so
    |err| <= (2 u16 + u16^2) S + sqrt(2) (n + 6) u32 (1 + 3 u16) S
             + 2^-25 (1 + u16) (stencil(|A|) W + s_max sum|v|) + tiny,
    W the per-site w broadcast over components (parity_bounds.coarse_apply_bounds).

A dropped, mis-signed or transposed block changes an entry by a whole term,
about S / n, which these bounds exclude (FP64/FP32 at most 0.05 S / n; FP16S at
most 0.75 S / n plus its subnormal terms).
RHS counts 1, 5 and 13 leave MFMA tile columns empty.

Transfers: a coarse entry of P^dag v sums n = 6 |block| terms, a fine entry of
P v_c sums n = k terms; the FP32 and FP16S forms both use the FP32 copy of P
and FP32 vectors, so |err| <= sqrt(2) (n + 4) u32 S with S from |P| and |v|.
"""
import numpy as np
import pytest

import synth
from oracle import chiral
from oracle.stencil import StencilOp, as_columns, as_fields
from parity_bounds import coarse_apply_bounds

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24
U16 = 2.0 ** -11


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _hierarchy(crk, m_prime, k):
    dims = [8, 8, 8, 16]
    U = synth.gauge_field(dims, 0.3, 1, config=21)
    lat = crk.Lattice(dims, -0.4, 1.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, m_prime=[m_prime], k=[k], block=[[4, 4, 4, 4]], n_smooth=[10],
                      setup_form=crk.FORM_FP32)
    return lat, H


@pytest.mark.parametrize("m_prime,k", [(16, 8), (48, 24)])
def test_coarse_operator_forms_match_oracle(crk, m_prime, k):
    lat, H = _hierarchy(crk, m_prime, k)
    try:
        X, Yp, Ym = H.coarse_links(0)
        Vc, N = X.shape[0], X.shape[-1]
        assert N == 2 * k
        cdims = [2, 2, 2, 4]
        op = StencilOp(cdims, X, Yp, Ym)
        for nrhs in (1, 5, 13):
            v = synth.gaussian_vectors(nrhs, Vc, N, config=30 + nrhs, level=1)
            ref = as_fields(op.apply(as_columns(v)))
            bounds, S, n = coarse_apply_bounds(X, Yp, Ym, cdims, v)
            for form in (crk.FORM_FP64, crk.FORM_FP32, crk.FORM_FP16S):
                out = H.coarse_apply(1, v, form=form)
                worst = (np.abs(out - ref) / bounds[form]).max()
                assert worst <= 1.0, (form, nrhs, worst)
            # and not trivially: a dropped term would be about S / n
            assert (bounds[1] <= 0.05 * S / n).all()
            sub = bounds[2] - ((2 * U16 + U16 ** 2) * S + np.sqrt(2) * (n + 6) * U32 * (1 + 3 * U16) * S)
            assert (bounds[2] <= 0.75 * S / n + sub).all()
    finally:
        H.close()


@pytest.mark.parametrize("m_prime,k", [(16, 8), (48, 24)])
def test_transfer_forms_match_oracle(crk, m_prime, k):
    lat, H = _hierarchy(crk, m_prime, k)
    try:
        dims, block = [8, 8, 8, 16], [4, 4, 4, 4]
        P = H.prolongator(0)
        Pa = np.abs(P)
        V, Vc = 8 * 8 * 8 * 16, 32
        n_r = 6 * 4 ** 4
        for nrhs in (1, 5):
            v = synth.gaussian_vectors(nrhs, V, 12, config=40 + nrhs, level=0)
            vc = synth.gaussian_vectors(nrhs, Vc, 2 * k, config=50 + nrhs, level=1)
            r_ref = as_fields(chiral.restrict(P, as_columns(v), dims, block))
            r_S = as_fields(chiral.restrict(Pa, as_columns(np.abs(v)), dims, block))
            p_ref = as_fields(chiral.prolong(P, as_columns(vc), dims, block))
            p_S = as_fields(chiral.prolong(Pa, as_columns(np.abs(vc)), dims, block))
            for form in (crk.FORM_FP64, crk.FORM_FP32, crk.FORM_FP16S):
                u = U64 if form == crk.FORM_FP64 else U32
                rg = H.restrict(0, v, form=form)
                worst = (np.abs(rg - r_ref) / (np.sqrt(2) * (n_r + 4) * u * r_S)).max()
                assert worst <= 1.0, ("restrict", form, nrhs, worst)
                pg = H.prolong(0, vc, form=form)
                worst = (np.abs(pg - p_ref) / (np.sqrt(2) * (k + 4) * u * p_S)).max()
                assert worst <= 1.0, ("prolong", form, nrhs, worst)
    finally:
        H.close()


def _to_device_layout(crk, H, level, v):
    """Host [R, V, N] complex128 -> complex64 array in the hierarchy's level layout (as crk.h states it)."""
    R, V, N = v.shape
    pos = H.get(level, crk.GET_DEVICE_ORDER).astype(np.int64)
    v32 = v.astype(np.complex64)
    if level == 0:
        Vp = (V + 63) // 64 * 64
        out = np.zeros(R * Vp * 12, dtype=np.complex64)
        r = np.arange(R)[:, None, None]
        c = np.arange(12)[None, None, :]
        p = pos[None, :, None]
        out[(r * Vp + 64 * (p // 64)) * 12 + 64 * c + p % 64] = v32
    else:
        out = np.zeros(V * N * R, dtype=np.complex64)
        r = np.arange(R)[:, None, None]
        c = np.arange(N)[None, None, :]
        p = pos[None, :, None]
        out[(p * N + c) * R + r] = v32
    return out


def _from_device_layout(crk, H, level, a, R):
    V, N = H.volume(level), H.ncomp[level]
    pos = H.get(level, crk.GET_DEVICE_ORDER).astype(np.int64)
    r = np.arange(R)[:, None, None]
    c = np.arange(N)[None, None, :]
    p = pos[None, :, None]
    if level == 0:
        Vp = (V + 63) // 64 * 64
        return a[(r * Vp + 64 * (p // 64)) * 12 + 64 * c + p % 64].astype(np.complex128)
    return a[(p * N + c) * R + r].astype(np.complex128)


def test_apply_dev_equals_host_apply(crk):
    """The device-buffer entry point runs the same kernels as the host one:
    FP32 results are bitwise equal on both levels once the layout stated in
    crk.h is applied; a zero RHS count is a no-op and aliasing is refused."""
    import torch
    lat, H = _hierarchy(crk, 16, 8)
    try:
        dev = torch.device("cuda", 0)
        for level in (0, 1):
            V, N = H.volume(level), H.ncomp[level]
            R = 3
            v = synth.gaussian_vectors(R, V, N, config=60 + level, level=level)
            host = H.coarse_apply(level, v, form=crk.FORM_FP32)
            nb = H.field_bytes(level, crk.FORM_FP32, R)
            a = _to_device_layout(crk, H, level, v)
            assert a.nbytes == nb
            d_in = torch.from_numpy(a).to(dev)
            d_out = torch.zeros_like(d_in)
            H.apply_dev(level, d_in, d_out, R, crk.FORM_FP32)
            torch.cuda.synchronize()
            got = _from_device_layout(crk, H, level, d_out.cpu().numpy(), R)
            assert np.array_equal(got, host), (level, np.abs(got - host).max())
            H.apply_dev(level, d_in, d_out, 0, crk.FORM_FP32)
            with pytest.raises(crk.CrkError):
                H.apply_dev(level, d_in, d_in, R, crk.FORM_FP32)
        assert H.field_bytes(5, crk.FORM_FP32, 1) == -1
    finally:
        H.close()
