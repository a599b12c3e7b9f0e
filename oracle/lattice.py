"""Lattice geometry: site index, periodic neighbours, block (aggregate) maps.

Paper, Sec. 2: the smooth test vectors are blocked by a domain decomposition
Lambda = {Lambda_1..Lambda_d} of the lattice, d = |Lambda| blocks, each block
becoming one coarse site.  Blocks here are hypercubes of extent b_mu; the same
maps are reused on every coarse lattice.

  site index   s(x) = x0 + L0*(x1 + L1*(x2 + L2*x3))
  neighbour    x +- mu (mod L_mu)
  block        j(x) = s_c(floor(x / b)) on the coarse lattice L/b
  local index  l(x) = s_b(x mod b) on the block lattice b
"""
from __future__ import annotations

import numpy as np


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def lex(c, dims):
    """Lexicographic index of coordinate rows c[..., 4] in a box of extent dims."""
    L = [int(d) for d in dims]
    c = np.asarray(c, dtype=np.int64)
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def coords(dims):
    """Coordinates [V, 4] of every site, in site-index order."""
    L = [int(d) for d in dims]
    s = np.arange(volume(L), dtype=np.int64)
    out = np.empty((s.size, 4), dtype=np.int64)
    for mu in range(4):
        out[:, mu] = s % L[mu]
        s = s // L[mu]
    return out


def neighbors(dims):
    """[V, 8] periodic neighbour table; column 2*mu is x+mu, column 2*mu+1 is x-mu."""
    L = [int(d) for d in dims]
    c = coords(L)
    out = np.empty((c.shape[0], 8), dtype=np.int64)
    for mu in range(4):
        for k, sgn in enumerate((+1, -1)):
            cc = c.copy()
            cc[:, mu] = (cc[:, mu] + sgn) % L[mu]
            out[:, 2 * mu + k] = lex(cc, L)
    return out


def coarse_dims(dims, block):
    dims = [int(d) for d in dims]
    block = [int(b) for b in block]
    for L, b in zip(dims, block):
        if b < 1 or L % b != 0:
            raise ValueError(f"block extent {b} does not divide lattice extent {L}")
    return [L // b for L, b in zip(dims, block)]


def block_maps(dims, block):
    """Aggregate map site -> (j, l): block index j(x) and local index l(x)."""
    cd = coarse_dims(dims, block)
    c = coords(dims)
    b = np.asarray(block, dtype=np.int64)
    j = lex(c // b, cd)
    l = lex(c % b, block)
    return j, l


def block_sites(dims, block):
    """[d, |Lambda_j|] table: block_sites[j, l] = site index s with j(s)=j, l(s)=l."""
    j, l = block_maps(dims, block)
    d = volume(coarse_dims(dims, block))
    nb = volume(block)
    out = np.full((d, nb), -1, dtype=np.int64)
    out[j, l] = np.arange(j.size, dtype=np.int64)
    return out
