"""Galerkin coarse operator D_{l+1} = R D_l P with R = P^dag (paper, Sec. 2, Eq. (4)).

Because P is block diagonal (Eq. (6)) the product is again a nearest-neighbour
stencil on the coarse lattice L/b with 2k components per coarse site.  With
P(x) the N x 2k block of P at fine site x and Y_{+-mu}(x) the fine hops:

  X(j)       = sum_{x in Lambda_j} P(x)^dag [ X_f(x) P(x)
                   + sum_{+-mu : x+-mu in Lambda_j} Y_{+-mu}(x) P(x+-mu) ]
  Y_{+-mu}(j) = sum_{x in Lambda_j, x+-mu not in Lambda_j} P(x)^dag Y_{+-mu}(x) P(x+-mu)

A coarse extent of 1 sends every hop into X; with coarse extent 2 both
Y_{+mu}(j) and Y_{-mu}(j) reach the same neighbour and the dense D_c holds
their sum (the stencil apply adds them automatically).
"""
from __future__ import annotations

import numpy as np

from . import lattice
from .chiral import site_blocks
from .stencil import StencilOp


def galerkin(op, Pb, block, blocks=None):
    """Coarse stencil of ``op`` (WilsonOp or StencilOp) for the prolongator blocks Pb.

    ``blocks`` optionally restricts the computation to a list of coarse sites
    (the other entries of X/Y are left zero); used to sample large lattices.
    Returns (StencilOp on the coarse lattice) when blocks is None, else
    (X, Yp, Ym) arrays for the requested blocks only.
    """
    dims = op.dims
    cd = lattice.coarse_dims(dims, block)
    d = lattice.volume(cd)
    k2 = 2 * Pb.shape[-1]
    jx, _ = lattice.block_maps(dims, block)
    Px = site_blocks(Pb, dims, block, op.N)
    nbr = op.nbr
    if blocks is None:
        sites = np.arange(jx.size)
        sel = np.arange(d)
    else:
        sel = np.asarray(blocks, dtype=np.int64)
        bs = lattice.block_sites(dims, block)
        sites = bs[sel].reshape(-1)
    pos = np.full(d, -1, dtype=np.int64)
    pos[sel] = np.arange(sel.size)
    row = pos[jx[sites]]  # output slot of each selected fine site

    X = np.zeros((sel.size, k2, k2), dtype=np.complex128)
    Yp = np.zeros((4, sel.size, k2, k2), dtype=np.complex128)
    Ym = np.zeros((4, sel.size, k2, k2), dtype=np.complex128)
    Pd = np.conj(np.swapaxes(Px[sites], -1, -2))  # P(x)^dag

    # site-diagonal term
    np.add.at(X, row, Pd @ op.diag_apply(Px[sites], sites=sites))
    for mu in range(4):
        for k, sign, Y in ((0, +1, Yp), (1, -1, Ym)):
            y = nbr[sites, 2 * mu + k]
            contrib = Pd @ op.hop(mu, sign, Px[y], sites=sites)
            inside = jx[y] == jx[sites]
            np.add.at(X, row[inside], contrib[inside])
            np.add.at(Y[mu], row[~inside], contrib[~inside])
    if blocks is not None:
        return X, Yp, Ym
    return StencilOp(cd, X, Yp, Ym)
