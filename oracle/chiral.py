"""Chiral split, chiral rank-k truncation and the block prolongator.

Paper, Sec. 2, Eq. (2): the test vectors are split into chiral components,
alpha = 0 taking spins 1,2 and alpha = 1 spins 3,4 (on coarse levels the first
and second half of the components, sigma_3 chirality).

Paper, Sec. 3, Eq. (5): for each block Lambda_j and chirality alpha the SVD
Psi^(alpha)(Lambda_j) = U Sigma V^dag is truncated to its k dominant left
singular vectors (m >= k), the best rank-k approximation; Eq. (6): those
vectors u_i^(alpha), restricted to Lambda_j, are the columns of P, which is
n x 2kd and needs no further orthonormalisation.  With k = m the span is that
of the conventional, orthonormalised chirally split basis of Eq. (3).

Block matrix rows (reading of the paper, which leaves the order open): row
h*l + c' holds component alpha*h + c' of local site l, where h is the number of
components per chirality (6 on the fine level: 3*spin' + colour; k on coarse
levels).  Coarse degrees of freedom are ordered (coarse site j, alpha, i).

Phase convention (singular vectors are unique only up to a phase): column i of
U_k is multiplied by conj(s_i)/|s_i| with s_i = sum_j V_{j i}, i.e. the sum of
the entries of the matching right singular vector becomes real positive.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def chiral_blocks(psi, dims, block):
    """Psi^(alpha)(Lambda_j) for all blocks: psi [V, N, m] -> A [d, 2, h*|Lambda|, m]."""
    bs = lattice.block_sites(dims, block)
    d, nb = bs.shape
    V, N, m = psi.shape
    h = N // 2
    t = psi[bs]  # [d, nb, N, m]
    return np.ascontiguousarray(
        t.reshape(d, nb, 2, h, m).transpose(0, 2, 1, 3, 4).reshape(d, 2, nb * h, m)
    )


def unblock(A, dims, block):
    """Inverse of chiral_blocks: A [d, 2, h*|Lambda|, C] -> field [V, 2h, C]."""
    bs = lattice.block_sites(dims, block)
    d, nb = bs.shape
    _, _, nr, C = A.shape
    h = nr // nb
    out = np.zeros((lattice.volume(dims), 2 * h, C), dtype=np.complex128)
    out[bs] = A.reshape(d, 2, nb, h, C).transpose(0, 2, 1, 3, 4).reshape(d, nb, 2 * h, C)
    return out


def truncated_svd(A, k):
    """Rank-k truncation of one block matrix A [N_r, m] (Eq. (5)).

    Returns (U_k [N_r, k] phase-fixed, sigma [min(N_r, m)] descending).
    """
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    k = int(k)
    Uk = U[:, :k].copy()
    ssum = np.conj(Vh[:k]).sum(axis=1)  # s_i = sum_j V_{j i}
    mag = np.abs(ssum)
    ph = np.where(mag > 0, np.conj(ssum) / np.where(mag > 0, mag, 1.0), 1.0)
    return Uk * ph[None, :], s


def prolongator_blocks(A, k):
    """Per-(block, chirality) U_k (Eq. (6)): A [d, 2, N_r, m] -> (P [d, 2, N_r, k], sigma [d, 2, r])."""
    d, two, nr, m = A.shape
    r = min(nr, m)
    if not (1 <= k <= r):
        raise ValueError(f"need 1 <= k <= min(m, N_r) = {r}, got k = {k}")
    P = np.empty((d, 2, nr, k), dtype=np.complex128)
    S = np.empty((d, 2, r))
    for j in range(d):
        for a in range(2):
            P[j, a], S[j, a] = truncated_svd(A[j, a], k)
    return P, S


def conventional_blocks(A):
    """Conventional setup (Eq. (3)): orthonormalise each chirally split block by QR."""
    d, two, nr, m = A.shape
    Q = np.empty((d, 2, nr, m), dtype=np.complex128)
    for j in range(d):
        for a in range(2):
            Q[j, a] = np.linalg.qr(A[j, a])[0]
    return Q


def site_blocks(Pb, dims, block, N):
    """P(x): the N x 2k block of P at every site, [V, N, 2k] (zero off-chirality)."""
    j, l = lattice.block_maps(dims, block)
    d, _, nr, k = Pb.shape
    nb = lattice.volume(block)
    h = N // 2
    assert nr == nb * h
    Px = np.zeros((j.size, N, 2 * k), dtype=np.complex128)
    for a in range(2):
        Px[:, a * h:(a + 1) * h, a * k:(a + 1) * k] = Pb[:, a].reshape(d, nb, h, k)[j, l]
    return Px


def prolongator_dense(Pb, dims, block, N):
    """Dense P, n x 2kd: row s*N + comp, column 2k*j + k*alpha + i."""
    j, _ = lattice.block_maps(dims, block)
    k = Pb.shape[-1]
    d = Pb.shape[0]
    Px = site_blocks(Pb, dims, block, N)
    V = j.size
    P = np.zeros((V * N, 2 * k * d), dtype=np.complex128)
    for x in range(V):
        P[x * N:(x + 1) * N, 2 * k * j[x]:2 * k * (j[x] + 1)] = Px[x]
    return P


def restrict(Pb, v, dims, block):
    """R v = P^dag v: fine [V, N, C] -> coarse [d, 2k, C]."""
    Av = chiral_blocks(v, dims, block)
    out = np.einsum("jari,jarc->jaic", np.conj(Pb), Av)
    d, _, k, C = out.shape
    return out.reshape(d, 2 * k, C)


def coarse_test_vectors(A, Pb):
    """Coarse test vectors (Sec. 3, after Eq. (5)): for block j and chirality a the
    truncated SVD A_{j,a} ~ U_k Sigma_k V_k^dag leaves Sigma_k V_k^dag = U_k^dag A_{j,a}
    (U_k with the prolongator's phase convention), the coordinates of the m' test
    vectors in the kept basis.  Returned as a coarse field [d, 2k, m']: component
    a k + i of coarse site j."""
    C = np.einsum("jari,jarc->jaic", np.conj(Pb), A)
    d, _, k, m = C.shape
    return C.reshape(d, 2 * k, m)


def prolong(Pb, vc, dims, block):
    """P vc: coarse [d, 2k, C] -> fine [V, N, C]."""
    d, _, nr, k = Pb.shape
    C = vc.shape[-1]
    t = np.einsum("jari,jaic->jarc", Pb, vc.reshape(d, 2, k, C))
    return unblock(t, dims, block)
