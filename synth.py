"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *draws* inputs: random SU(3) gauge links (optionally smoothed
by APE-like projections), Gaussian test vectors, Gaussian and point-source
right-hand sides, and Poisson arrival times.  It contains none of the
multigrid method's arithmetic (no Dirac operator, no smoother, no SVD, no
Galerkin product, no solver), so both sides of every parity check can consume
the same buffers without sharing method code.

Seeding: every stream is ``numpy.random.default_rng([config, purpose, index])``
with purpose 0 = gauge field, 1 = test vectors (index = level), 2 = right-hand
sides (index = RHS or request id), 3 = arrival times.

Conventions (also those of the C ABI):
  * site index s = x0 + L0*(x1 + L1*(x2 + L2*x3)), direction mu = 0..3 = x,y,z,t;
  * gauge array U[s, mu, a, b] = colour matrix U_mu(x)[a][b], complex128;
  * spinor component index 3*spin + colour; fields are [rhs, site, 12].
"""
from __future__ import annotations

import numpy as np


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def _coords(dims):
    L = [int(d) for d in dims]
    s = np.arange(volume(L), dtype=np.int64)
    c = np.empty((s.size, 4), dtype=np.int64)
    r = s.copy()
    for mu in range(4):
        c[:, mu] = r % L[mu]
        r //= L[mu]
    return c


def _shift(dims, mu, sign):
    """Site index of x + sign*mu (periodic) for every site x."""
    L = [int(d) for d in dims]
    c = _coords(L)
    c[:, mu] = (c[:, mu] + sign) % L[mu]
    return c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))


def _expi_hermitian(H, eps):
    """exp(i*eps*H) for a batch of Hermitian 3x3 matrices, via eigendecomposition."""
    w, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ab,...b,...cb->...ac", Q, ph, Q.conj())


def project_su3(M):
    """Nearest unitary (polar factor) followed by removal of the determinant phase.

    W = M (M^dag M)^(-1/2) computed from the SVD M = X S Y^dag as W = X Y^dag,
    then W <- W / det(W)^(1/3) with the principal cube root.
    """
    X, _, Yh = np.linalg.svd(M)
    W = X @ Yh
    det = np.linalg.det(W)
    phase = np.exp(-1j * np.angle(det) / 3.0)
    return W * phase[..., None, None]


def _ape_step(U, dims, alpha):
    """One APE-like smoothing step, all links updated from the old field."""
    V = U.shape[0]
    fwd = [_shift(dims, mu, +1) for mu in range(4)]
    bwd = [_shift(dims, mu, -1) for mu in range(4)]
    new = np.empty_like(U)
    dag = lambda A: np.conj(np.swapaxes(A, -1, -2))
    for mu in range(4):
        S = np.zeros((V, 3, 3), dtype=np.complex128)
        for nu in range(4):
            if nu == mu:
                continue
            # upper staple U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
            S += U[:, nu] @ U[fwd[nu], mu] @ dag(U[fwd[mu], nu])
            # lower staple U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
            xm = bwd[nu]
            S += dag(U[xm, nu]) @ U[xm, mu] @ U[fwd[mu][xm], nu]
        new[:, mu] = project_su3((1.0 - alpha) * U[:, mu] + (alpha / 6.0) * S)
    return new


def gauge_field(dims, eps, n_ape=0, config=0, ape_alpha=0.5):
    """Random SU(3) links U = exp(i*eps*H), H Gaussian traceless Hermitian.

    A has Re, Im ~ N(0,1) per entry, drawn in the order (site, mu, row, col,
    re/im); H = (A + A^dag)/2 - tr/3.  Then ``n_ape`` APE-like projections with
    weight ``ape_alpha`` on the six staples.  Returns complex128 [V, 4, 3, 3].
    """
    V = volume(dims)
    rng = np.random.default_rng([int(config), 0, 0])
    z = rng.standard_normal((V, 4, 3, 3, 2))
    A = z[..., 0] + 1j * z[..., 1]
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    U = _expi_hermitian(H, eps)
    for _ in range(int(n_ape)):
        U = _ape_step(U, dims, ape_alpha)
    return np.ascontiguousarray(U)


def gauge_field_device(dims, eps, n_ape=0, config=0, ape_alpha=0.5, device="cuda", progress=None):
    """The gauge_field recipe evaluated with torch on a device, for volumes where
    the host version takes minutes (same random draw; the matrix functions are
    computed differently, so links agree with gauge_field to rounding, not bits).

    exp(i eps H) by torch.linalg.matrix_exp; the SU(3) projection is the polar
    factor from the Newton iteration W <- (W + W^-dag)/2 (3x3 inverse by
    cofactors) followed by the determinant-phase removal of project_su3.
    Returns complex128 [V, 4, 3, 3] on the host.
    """
    import torch

    def note(msg):
        if progress:
            progress(msg)

    V = volume(dims)
    rng = np.random.default_rng([int(config), 0, 0])
    U = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device=device)
    chunk = 1 << 20  # sites per host draw (keeps host memory bounded)
    for s0 in range(0, V, chunk):
        n = min(chunk, V - s0)
        z = torch.from_numpy(rng.standard_normal((n, 4, 3, 3, 2))).to(device)
        A = torch.complex(z[..., 0], z[..., 1])
        H = 0.5 * (A + A.conj().transpose(-1, -2))
        tr = torch.diagonal(H, dim1=-2, dim2=-1).sum(-1).real / 3.0
        H = H - tr[..., None, None] * torch.eye(3, dtype=H.dtype, device=device)
        U[s0:s0 + n] = torch.linalg.matrix_exp(1j * eps * H)
    note("gauge: exp(i eps H) done")

    def dag(M):
        return M.conj().transpose(-1, -2).contiguous()

    def inv3(M):
        a, b, c = M[..., 0, 0], M[..., 0, 1], M[..., 0, 2]
        d, e, f = M[..., 1, 0], M[..., 1, 1], M[..., 1, 2]
        g, h, i = M[..., 2, 0], M[..., 2, 1], M[..., 2, 2]
        A_, B_, C_ = e * i - f * h, -(d * i - f * g), d * h - e * g
        det = a * A_ + b * B_ + c * C_
        adj = torch.stack([torch.stack([A_, -(b * i - c * h), b * f - c * e], -1),
                           torch.stack([B_, a * i - c * g, -(a * f - c * d)], -1),
                           torch.stack([C_, -(a * h - b * g), a * e - b * d], -1)], -2)
        return adj / det[..., None, None], det

    def project(M):
        W = M
        for _ in range(30):
            Wi, _ = inv3(W)
            Wn = 0.5 * (W + dag(Wi))
            done = (Wn - W).abs().max().item() < 1e-15
            W = Wn
            if done:
                break
        _, det = inv3(W)
        return W * torch.exp(-1j * torch.angle(det) / 3.0)[..., None, None]

    c = torch.from_numpy(_coords(dims)).to(device)
    L = torch.tensor([int(x) for x in dims], device=device)

    def shift(mu, sign):
        cc = c.clone()
        cc[:, mu] = (cc[:, mu] + sign) % L[mu]
        return cc[:, 0] + L[0] * (cc[:, 1] + L[1] * (cc[:, 2] + L[2] * cc[:, 3]))

    fwd = [shift(mu, +1) for mu in range(4)]
    bwd = [shift(mu, -1) for mu in range(4)]
    for step in range(int(n_ape)):
        new = torch.empty_like(U)
        for mu in range(4):
            S = torch.zeros((V, 3, 3), dtype=U.dtype, device=device)
            for nu in range(4):
                if nu == mu:
                    continue
                S += U[:, nu] @ U[fwd[nu], mu] @ dag(U[fwd[mu], nu])
                xm = bwd[nu]
                S += dag(U[xm, nu]) @ U[xm, mu] @ U[fwd[mu][xm], nu]
            new[:, mu] = project((1.0 - ape_alpha) * U[:, mu] + (ape_alpha / 6.0) * S)
            del S
        U = new
        note(f"gauge: smoothing step {step + 1} of {n_ape} done")
    out = U.cpu().numpy()
    del U
    return np.ascontiguousarray(out)


def unit_gauge(dims):
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gaussian_vectors(m, n_sites, n_comp=12, config=0, level=0):
    """m complex Gaussian vectors [m, n_sites, n_comp], Re/Im ~ N(0,1),
    drawn in the order (vector, site, component, re/im)."""
    rng = np.random.default_rng([int(config), 1, int(level)])
    z = rng.standard_normal((int(m), int(n_sites), int(n_comp), 2))
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def gaussian_rhs(nrhs, n_sites, config=0, index=0, n_comp=12):
    """nrhs complex Gaussian right-hand sides [nrhs, n_sites, n_comp]."""
    rng = np.random.default_rng([int(config), 2, int(index)])
    z = rng.standard_normal((int(nrhs), int(n_sites), int(n_comp), 2))
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def point_sources(n_sites, site=0):
    """12 point sources at ``site``, one per (spin, colour): [12, n_sites, 12]."""
    b = np.zeros((12, int(n_sites), 12), dtype=np.complex128)
    for c in range(12):
        b[c, site, c] = 1.0
    return b


def poisson_arrivals(rate, n, config=0, index=0):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng([int(config), 3, int(index)])
    return np.cumsum(rng.exponential(1.0 / float(rate), size=int(n)))


def random_gauge_transform(V, config=0):
    """Random SU(3) matrices G(x), [V, 3, 3] (for covariance checks)."""
    rng = np.random.default_rng([int(config), 4, 0])
    z = rng.standard_normal((V, 3, 3, 2))
    return project_su3(z[..., 0] + 1j * z[..., 1])
