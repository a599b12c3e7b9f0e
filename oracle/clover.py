"""Clover (Sheikholeslami-Wohlert) site term of the Wilson-clover operator.

Test infrastructure: the plain FP64 oracle of what the HIP path computes; only
the tests, the smoke check and the benchmark's CPU baseline use it.

Both of the paper's ensembles are clover actions (Sec. 4: an anisotropic clover
lattice and clover on HISQ), but the paper does not write the term out.  This
oracle uses the standard form, added to the Wilson site term:

  C(x) = -(c_sw / 2) sum_{mu < nu} w_mu w_nu sigma_{mu nu} (x) F_{mu nu}(x),
  sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
  F_{mu nu}(x) = (1 / 8i) [ (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) - (1/3) tr(...) ],

with Q_{mu nu}(x) the sum of the four plaquettes ("clover leaves") in the
(mu, nu) plane that start and end at x, taken counter-clockwise, and w the
anisotropy weights of the hops (w_t = 1/xi, so temporal planes carry 1/xi).
F is Hermitian and traceless, sigma_{mu nu} is Hermitian and commutes with
gamma5, so C(x) is Hermitian and block diagonal in the chirality of Eq. (2):
two 6 x 6 blocks per site (spins 1,2 and spins 3,4), and gamma5 D gamma5 = D^dag
still holds.  The operator's site term becomes the 12 x 12 matrix
(m0 + sum_mu w_mu) 1 + C(x).
"""
from __future__ import annotations

import numpy as np

from . import lattice
from .gamma import gamma


def sigma_munu(mu, nu):
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (4 x 4)."""
    return 0.5j * (gamma[mu] @ gamma[nu] - gamma[nu] @ gamma[mu])


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def clover_leaves(U, dims, mu, nu):
    """Q_{mu nu}(x): the four plaquettes in the (mu, nu) plane around x, [V, 3, 3]."""
    nbr = lattice.neighbors(dims)
    fm, bm = nbr[:, 2 * mu], nbr[:, 2 * mu + 1]
    fn, bn = nbr[:, 2 * nu], nbr[:, 2 * nu + 1]
    Um, Un = U[:, mu], U[:, nu]
    x = np.arange(U.shape[0])
    # x -> x+mu -> x+mu+nu -> x+nu -> x
    q = Um[x] @ Un[fm] @ _dag(Um[fn]) @ _dag(Un[x])
    # x -> x+nu -> x+nu-mu -> x-mu -> x
    q = q + Un[x] @ _dag(Um[bm[fn]]) @ _dag(Un[bm]) @ Um[bm]
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + _dag(Um[bm]) @ _dag(Un[bn[bm]]) @ Um[bn[bm]] @ Un[bn]
    # x -> x-nu -> x-nu+mu -> x+mu -> x
    q = q + _dag(Un[bn]) @ Um[bn] @ Un[fm[bn]] @ _dag(Um[x])
    return q


def field_strength(U, dims, mu, nu):
    """F_{mu nu}(x), Hermitian and traceless, [V, 3, 3]."""
    Q = clover_leaves(U, dims, mu, nu)
    A = Q - _dag(Q)
    tr = np.trace(A, axis1=-2, axis2=-1) / 3.0
    A = A - tr[:, None, None] * np.eye(3)
    return A / 8j


def clover_term(U, dims, c_sw, xi=1.0):
    """C(x) as [V, 12, 12] (index 3*spin + colour)."""
    U = np.asarray(U, dtype=np.complex128)
    w = np.array([1.0, 1.0, 1.0, 1.0 / float(xi)])
    V = U.shape[0]
    C = np.zeros((V, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            F = field_strength(U, dims, mu, nu)
            s = sigma_munu(mu, nu)
            C += (-0.5 * c_sw * w[mu] * w[nu]) * np.einsum("st,xab->xsatb", s, F).reshape(V, 12, 12)
    return C
