"""Wilson-Dirac operator D on a periodic 4-D lattice (paper, Secs. 1-2).

The paper names the Wilson-Dirac operator without writing it out; this oracle
uses the standard mass form with Wilson parameter r = 1 and an anisotropy
weight w_mu = (1, 1, 1, 1/xi) on the temporal hops and in the Wilson diagonal:

  (D psi)(x) = (m0 + sum_mu w_mu) psi(x)
             - 1/2 sum_mu w_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
                                + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ].

With xi = 1 the diagonal is m0 + 4.  In the free field (U = 1) a plane wave
e^{ipx} chi is mapped to e^{ipx} D(p) chi with
D(p) = m0 + sum_mu w_mu (1 - cos p_mu) + i sum_mu w_mu gamma_mu sin p_mu.
With c_sw != 0 the site term becomes (m0 + sum_mu w_mu) 1 + C(x), C the clover
term of oracle.clover (the Wilson-clover operator of the paper's ensembles).

Vectors are [V, 12, C] (component index 3*spin + colour).
"""
from __future__ import annotations

import numpy as np

from . import lattice
from .gamma import gamma, identity4
from .stencil import StencilOp


def weights(xi):
    return np.array([1.0, 1.0, 1.0, 1.0 / float(xi)])


class WilsonOp:
    """D in hopping form; same interface as StencilOp (diag_apply / hop / apply)."""

    def __init__(self, U, dims, m0, xi=1.0, c_sw=0.0):
        self.dims = [int(d) for d in dims]
        self.U = np.asarray(U, dtype=np.complex128)
        self.V = lattice.volume(self.dims)
        assert self.U.shape == (self.V, 4, 3, 3)
        self.m0 = float(m0)
        self.xi = float(xi)
        self.w = weights(xi)
        self.N = 12
        self.h = 6
        self.nbr = lattice.neighbors(self.dims)
        self.Ubwd = [
            np.conj(np.swapaxes(self.U[self.nbr[:, 2 * mu + 1], mu], -1, -2)) for mu in range(4)
        ]
        self.c_sw = float(c_sw)
        self.site = None  # [V, 12, 12] site term when the clover term is on
        if self.c_sw != 0.0:
            from .clover import clover_term
            self.site = self.diag * np.eye(12, dtype=np.complex128)[None] + clover_term(self.U, self.dims, self.c_sw,
                                                                                        self.xi)

    @property
    def diag(self):
        return self.m0 + self.w.sum()

    def diag_apply(self, v, sites=None):
        if self.site is None:
            return self.diag * v
        X = self.site if sites is None else self.site[sites]
        return X @ v

    def hop(self, mu, sign, v_nb, sites=None):
        """-1/2 w_mu (1 -+ gamma_mu) (x) U  applied to v_nb[x] = v(x + sign*mu)."""
        if sign > 0:
            link = self.U[:, mu]
            spin = identity4 - gamma[mu]
        else:
            link = self.Ubwd[mu]
            spin = identity4 + gamma[mu]
        if sites is not None:
            link = link[sites]
        n, _, C = v_nb.shape
        t = v_nb.reshape(n, 4, 3, C).transpose(0, 2, 1, 3).reshape(n, 3, 4 * C)
        t = link @ t  # colour
        t = t.reshape(n, 3, 4, C).transpose(0, 2, 1, 3).reshape(n, 4, 3 * C)
        t = spin @ t  # spin
        return (-0.5 * self.w[mu]) * t.reshape(n, 12, C)

    def apply(self, v):
        out = self.diag_apply(v)
        for mu in range(4):
            out = out + self.hop(mu, +1, v[self.nbr[:, 2 * mu]])
            out = out + self.hop(mu, -1, v[self.nbr[:, 2 * mu + 1]])
        return out

    def apply_at(self, v, sites):
        """(D v)(x) for the listed sites only (v given on the whole lattice)."""
        sites = np.asarray(sites, dtype=np.int64)
        out = self.diag_apply(v[sites], sites=sites)
        for mu in range(4):
            out = out + self.hop(mu, +1, v[self.nbr[sites, 2 * mu]], sites=sites)
            out = out + self.hop(mu, -1, v[self.nbr[sites, 2 * mu + 1]], sites=sites)
        return out

    def chirality(self):
        return np.concatenate([np.ones(6), -np.ones(6)])

    def to_stencil(self):
        """Explicit StencilOp with X = diag * 1, Y_{+-mu}(x) = -w/2 (1 -+ gamma_mu) (x) link."""
        V = self.V
        if self.site is None:
            X = np.broadcast_to(self.diag * np.eye(12, dtype=np.complex128), (V, 12, 12)).copy()
        else:
            X = self.site.copy()
        Yp = np.empty((4, V, 12, 12), dtype=np.complex128)
        Ym = np.empty((4, V, 12, 12), dtype=np.complex128)
        for mu in range(4):
            c = -0.5 * self.w[mu]
            Yp[mu] = c * np.einsum("st,xab->xsatb", identity4 - gamma[mu], self.U[:, mu]).reshape(V, 12, 12)
            Ym[mu] = c * np.einsum("st,xab->xsatb", identity4 + gamma[mu], self.Ubwd[mu]).reshape(V, 12, 12)
        return StencilOp(self.dims, X, Yp, Ym)

    def dense(self):
        return self.to_stencil().dense()


def free_field_symbol(p, m0, xi):
    """D(p) (4x4 spin matrix) of the free Wilson operator for momentum p[4]."""
    w = weights(xi)
    p = np.asarray(p, dtype=np.float64)
    M = (m0 + np.sum(w * (1.0 - np.cos(p)))) * identity4
    for mu in range(4):
        M = M + 1j * w[mu] * np.sin(p[mu]) * gamma[mu]
    return M


def free_field_eigenvalues(dims, m0, xi):
    """Closed-form spectrum of the free Wilson operator (each value 6-fold: 2 spins x 3 colours).

    lambda(p) = m0 + sum w (1 - cos p) +- i sqrt(sum w^2 sin^2 p), p_mu = 2 pi n_mu / L_mu.
    """
    w = weights(xi)
    vals = []
    for c in lattice.coords(dims):
        p = 2 * np.pi * c / np.asarray(dims, dtype=np.float64)
        re = m0 + np.sum(w * (1 - np.cos(p)))
        im = np.sqrt(np.sum(w**2 * np.sin(p) ** 2))
        vals += [re + 1j * im] * 6 + [re - 1j * im] * 6
    return np.array(vals)
