"""Nearest-neighbour block-stencil operators (the common form of every level).

Every operator of the hierarchy is a nearest-neighbour stencil on a periodic
4-D lattice with N = 2h degrees of freedom per site, chirality alpha = 0 on
components [0, h) and alpha = 1 on [h, 2h):

  (A v)(x) = X(x) v(x) + sum_mu [ Y_{+mu}(x) v(x+mu) + Y_{-mu}(x) v(x-mu) ].

On the fine level this is the Wilson-Dirac operator (h = 6: spins 1,2 and 3,4
of Eq. (2)); on coarse levels it is the Galerkin product R D P of Eq. (4), whose
chirality is sigma_3 (paper, Sec. 2 last paragraph: gamma5 on level l > 0 is
sigma_3, i.e. first half vs second half of the coarse components).

Vectors are arrays [V, N, C]: site, component, column (right-hand side).
"""
from __future__ import annotations

import numpy as np

from . import lattice


class StencilOp:
    """Explicit stencil: X [V, N, N], Yp [4, V, N, N], Ym [4, V, N, N]."""

    def __init__(self, dims, X, Yp, Ym):
        self.dims = [int(d) for d in dims]
        self.X = np.asarray(X, dtype=np.complex128)
        self.Yp = np.asarray(Yp, dtype=np.complex128)
        self.Ym = np.asarray(Ym, dtype=np.complex128)
        self.V = lattice.volume(self.dims)
        self.N = self.X.shape[-1]
        self.h = self.N // 2
        self.nbr = lattice.neighbors(self.dims)

    def diag_apply(self, v, sites=None):
        X = self.X if sites is None else self.X[sites]
        return X @ v

    def hop(self, mu, sign, v_nb, sites=None):
        """Y_{sign*mu}(x) v(x + sign*mu), given v_nb[x] = v(x + sign*mu)."""
        Y = (self.Yp if sign > 0 else self.Ym)[mu]
        if sites is not None:
            Y = Y[sites]
        return Y @ v_nb

    def apply(self, v):
        out = self.diag_apply(v)
        for mu in range(4):
            out = out + self.hop(mu, +1, v[self.nbr[:, 2 * mu]])
            out = out + self.hop(mu, -1, v[self.nbr[:, 2 * mu + 1]])
        return out

    def chirality(self):
        """Per-site chirality matrix: +1 on the first h components, -1 on the rest."""
        return np.concatenate([np.ones(self.h), -np.ones(self.h)])

    def dense(self):
        """Dense matrix of the operator (small lattices only), index s*N + comp."""
        V, N = self.V, self.N
        D = np.zeros((V * N, V * N), dtype=np.complex128)
        for x in range(V):
            D[x * N:(x + 1) * N, x * N:(x + 1) * N] += self.X[x]
            for mu in range(4):
                for k, Y in ((0, self.Yp), (1, self.Ym)):
                    y = self.nbr[x, 2 * mu + k]
                    D[x * N:(x + 1) * N, y * N:(y + 1) * N] += Y[mu, x]
        return D


def as_columns(field):
    """[R, V, N] -> [V, N, R]."""
    return np.ascontiguousarray(np.transpose(np.asarray(field), (1, 2, 0)))


def as_fields(cols):
    """[V, N, R] -> [R, V, N]."""
    return np.ascontiguousarray(np.transpose(np.asarray(cols), (2, 0, 1)))
