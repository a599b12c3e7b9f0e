"""Pins of the oracle's flexible GCR and the MG-preconditioned solve.

References: dense LU solves (numpy.linalg.solve) on small systems, the true
residual, the forward-error bound 2*kappa*tol, and the full-rank hierarchy
with an exact coarse solve acting as D^{-1} (one outer iteration).
"""
import numpy as np

import synth
from oracle import chiral, galerkin, lattice, mg, mr
from oracle.stencil import as_columns
from oracle.wilson import WilsonOp


def _setup(dims=(4, 4, 4, 4), m=16, k=8, eps=0.3, m0=-0.4, config=1, n_smooth=20):
    dims = list(dims)
    U = synth.gauge_field(dims, eps, 0, config=config)
    op = WilsonOp(U, dims, m0, 1.0)
    iv = mg.init_vectors_for([dims], [12], [m], config, synth.gaussian_vectors)
    return op, mg.mg_setup(op, [m], [k], [[2, 2, 2, 2]], [n_smooth], iv)


def test_unpreconditioned_gcr_matches_dense_solve():
    op, _ = _setup()
    b = as_columns(synth.gaussian_rhs(1, op.V, config=1))
    x, it, conv, rr = mg.fgcr(op, b, 1e-12, 2000, 2000, None, true_residual=True)
    xd = np.linalg.solve(op.dense(), b.reshape(-1))
    assert conv and rr <= 1e-12
    assert np.linalg.norm(x.reshape(-1) - xd) <= 1e-9 * np.linalg.norm(xd)


def test_mg_solve_c1_against_dense_with_kappa_bound():
    op, levels = _setup()
    b = as_columns(synth.gaussian_rhs(1, op.V, config=1))
    x, info = mg.mg_solve(levels, b, tol=1e-10)
    D = op.dense()
    xd = np.linalg.solve(D, b.reshape(-1))
    s = np.linalg.svd(D, compute_uv=False)
    kappa = s[0] / s[-1]
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    assert np.linalg.norm(b.reshape(-1) - D @ x.reshape(-1)) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x.reshape(-1) - xd) <= 2 * kappa * 1e-10 * np.linalg.norm(xd)
    assert info["level_iters"][0] == info["iters"] and info["level_iters"][1] > 0


def test_full_rank_hierarchy_with_exact_coarse_solve_is_direct():
    dims = [2, 2, 2, 4]
    U = synth.gauge_field(dims, 0.4, 0, config=7)
    op = WilsonOp(U, dims, -0.2, 1.0)
    iv = mg.init_vectors_for([dims], [12], [96], 7, synth.gaussian_vectors)
    levels = mg.mg_setup(op, [96], [96], [[2, 2, 2, 2]], [2], iv)
    b = as_columns(synth.gaussian_rhs(1, op.V, config=7))
    cp = mg.CycleParams(tau=1e-14, coarsest_maxit=2000)
    x, info = mg.mg_solve(levels, b, tol=1e-10, cp=cp)
    assert info["converged"] and info["iters"] == 1


def test_three_level_solve_converges():
    dims = [4, 4, 4, 4]
    U = synth.gauge_field(dims, 0.3, 0, config=8)
    op = WilsonOp(U, dims, -0.4, 1.0)
    iv = mg.init_vectors_for([dims, [2, 2, 2, 2]], [12, 16], [16, 24], 8, synth.gaussian_vectors)
    levels = mg.mg_setup(op, [16, 24], [8, 12], [[2, 2, 2, 2], [2, 2, 2, 2]], [20, 20], iv)
    b = as_columns(synth.gaussian_rhs(1, op.V, config=8))
    x, info = mg.mg_solve(levels, b, tol=1e-10)
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    assert len(info["level_iters"]) == 3 and min(info["level_iters"]) > 0


def test_zero_rhs_returns_zero():
    op, levels = _setup()
    b = np.zeros((op.V, 12, 1), dtype=complex)
    x, info = mg.mg_solve(levels, b)
    assert info["converged"] and info["iters"] == 0 and not x.any()
