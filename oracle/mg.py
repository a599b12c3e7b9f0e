"""Multigrid setup recursion and the MG-preconditioned flexible GCR solve.

Setup (paper, Sec. 2 and 3), on each level l = 0 .. L-2:
  1. smoother on D_l psi_i ~ 0 from m' random vectors (Eq. (1));
  2. normalise each psi_i, chiral split per block (Eq. (2));
  3. SVD per (block, chirality), keep k left singular vectors (Eq. (5)) -> P (Eq. (6));
  4. D_{l+1} = P^dag D_l P (Eq. (4)); chirality on level l+1 is sigma_3.

Solve (paper, Sec. 2 last paragraph: the hierarchy is used as a K-cycle
preconditioner of a flexible outer solver such as GCR).  The paper gives no
cycle parameters; this oracle fixes (and the GPU library uses the same):
  * outer flexible GCR, restart 16, stop on the TRUE residual
    ||b - D x|| / ||b|| <= tol (recomputed at claimed convergence and at each
    restart);
  * K-cycle on level l: no pre-smoothing; r_c = P^dag r; e_c from flexible GCR
    on D_{l+1} started at 0, preconditioned by the level-(l+1) cycle, run to
    relative residual tau = 0.1 or 20 iterations (the coarsest level runs
    unpreconditioned GCR to tau or 50 iterations); e = P e_c; then 4 MR steps
    on D_l e = r starting from e;
  * classical Gram-Schmidt (one pass) of each new w = D z against the stored,
    normalised w's; z receives the same combination.
Vectors are single columns [V, N, 1]; each right-hand side is solved alone.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import lattice
from .chiral import chiral_blocks, coarse_test_vectors, prolongator_blocks, prolong, restrict
from .galerkin import galerkin
from .mr import cdot, mr_null, mr_solve, normalize_columns


@dataclass
class Level:
    op: object
    block: list | None = None
    Pb: np.ndarray | None = None
    sigma: np.ndarray | None = None
    vectors: np.ndarray | None = None  # smoothed (normalised) test vectors


@dataclass
class CycleParams:
    tau: float = 0.1
    inner_maxit: int = 20
    coarsest_maxit: int = 50
    nu_pre: int = 0
    nu_post: int = 4
    restart: int = 16


def mg_setup(fine_op, m_prime, k, blocks, n_smooth, init_vectors, normalize=True, keep_vectors=False,
             coarse_init=False):
    """Build the hierarchy.  init_vectors[l] is [V_l, N_l, m'_l] (complex Gaussian).
    With coarse_init, a coarsening step l >= 1 whose init_vectors[l] is None starts
    from the first m'_l coarse test vectors Sigma_k V_k^dag of step l - 1."""
    levels = []
    op = fine_op
    n_coarse = len(blocks)
    coarse = None
    for l in range(n_coarse):
        iv = init_vectors[l]
        if iv is None:
            if not (coarse_init and coarse is not None and m_prime[l] <= coarse.shape[-1]):
                raise ValueError("no initial vectors for step %d" % l)
            iv = np.ascontiguousarray(coarse[:, :, :m_prime[l]])
        psi = mr_null(op, iv, n_smooth[l])
        if normalize:
            psi = normalize_columns(psi)
        A = chiral_blocks(psi, op.dims, blocks[l])
        Pb, S = prolongator_blocks(A, k[l])
        coarse = coarse_test_vectors(A, Pb)
        Dc = galerkin(op, Pb, blocks[l])
        levels.append(Level(op, list(blocks[l]), Pb, S, psi if keep_vectors else None))
        op = Dc
    levels.append(Level(op))
    return levels


def _norm(v):
    return float(np.sqrt(cdot(v, v).real.sum()))


def fgcr(op, b, tol, maxit, restart, precond=None, true_residual=False, counter=None, level=0):
    """Flexible GCR from x = 0.  Returns (x, iterations, converged, rel_resid)."""
    x = np.zeros_like(b)
    bn = _norm(b)
    if bn == 0.0:
        return x, 0, True, 0.0
    r = b.copy()
    Z, W = [], []
    it = 0
    rn = bn
    converged = False
    while it < maxit:
        z = precond(r) if precond is not None else r.copy()
        w = op.apply(z)
        if W:
            c = [cdot(wj, w) for wj in W]  # classical Gram-Schmidt coefficients
            for cj, zj, wj in zip(c, Z, W):
                w = w - cj * wj
                z = z - cj * zj
        nw = _norm(w)
        it += 1
        if counter is not None:
            counter[level] = counter.get(level, 0) + 1
        if not np.isfinite(nw) or nw == 0.0:
            break  # breakdown
        w = w / nw
        z = z / nw
        a = cdot(w, r)
        x = x + a * z
        r = r - a * w
        Z.append(z)
        W.append(w)
        rn = _norm(r)
        if rn <= tol * bn:
            if not true_residual:
                converged = True
                break
            r = b - op.apply(x)
            rn = _norm(r)
            Z, W = [], []
            if rn <= tol * bn:
                converged = True
                break
        elif len(W) >= restart:
            if true_residual:
                r = b - op.apply(x)
                rn = _norm(r)
            Z, W = [], []
    return x, it, converged, rn / bn


def kcycle(levels, l, r, cp: CycleParams, counter=None):
    """Approximate D_l^{-1} r by one K-cycle (see module docstring)."""
    lev = levels[l]
    op = lev.op
    e = np.zeros_like(r)
    if cp.nu_pre > 0:
        e = mr_solve(op, r, e, cp.nu_pre)
        rc = restrict(lev.Pb, r - op.apply(e), op.dims, lev.block)
    else:
        rc = restrict(lev.Pb, r, op.dims, lev.block)
    nxt = l + 1
    cop = levels[nxt].op
    if nxt == len(levels) - 1:
        ec, _, _, _ = fgcr(cop, rc, cp.tau, cp.coarsest_maxit, cp.coarsest_maxit, None,
                           counter=counter, level=nxt)
    else:
        ec, _, _, _ = fgcr(cop, rc, cp.tau, cp.inner_maxit, cp.inner_maxit,
                           lambda v: kcycle(levels, nxt, v, cp, counter),
                           counter=counter, level=nxt)
    e = e + prolong(lev.Pb, ec, op.dims, lev.block)
    if cp.nu_post > 0:
        e = mr_solve(op, r, e, cp.nu_post)
    return e


def mg_solve(levels, b, tol=1e-10, maxit=200, cp: CycleParams | None = None):
    """Solve D x = b (b [V, 12, 1]) with K-cycle-preconditioned FGCR.

    Returns (x, info) with info = {iters, level_iters, converged, true_rel_resid}.
    """
    cp = cp or CycleParams()
    counter = {}
    op = levels[0].op
    precond = (lambda v: kcycle(levels, 0, v, cp, counter)) if len(levels) > 1 else None
    x, it, conv, _ = fgcr(op, b, tol, maxit, cp.restart, precond, true_residual=True,
                          counter=counter, level=0)
    rr = _norm(b - op.apply(x)) / max(_norm(b), 1e-300)
    info = {
        "iters": it,
        "level_iters": [counter.get(l, 0) for l in range(len(levels))],
        "converged": conv,
        "true_rel_resid": rr,
    }
    return x, info


def init_vectors_for(levels_dims, comps, m_prime, config, gen):
    """Columns [V_l, N_l, m'_l] from a generator gen(m, V, N, config, level) -> [m, V, N]."""
    out = []
    for l, (dims, N, m) in enumerate(zip(levels_dims, comps, m_prime)):
        v = gen(m, lattice.volume(dims), N, config=config, level=l)
        out.append(np.ascontiguousarray(np.transpose(v, (1, 2, 0))))
    return out
