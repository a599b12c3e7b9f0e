"""Minimal-residual (MR) iterations.

Paper, Sec. 2, Eq. (1): the smoother is applied to the homogeneous system
D psi_i ~ 0 from m random initial guesses, producing the test vectors
Psi = [psi_1 .. psi_m].  The paper does not name its smoother; this oracle
uses MR with relaxation 1, each vector independent.  With <a,b> = sum conj(a) b:

  r = -D psi
  repeat n times:  q = D r;  alpha = <q,r>/<q,q>;  psi += alpha r;  r -= alpha q

(a step with <q,q> = 0 uses alpha = 0).  The same MR step, started from the
residual rho = b - D e of a system D e = b, is the K-cycle post-smoother.
Vectors are [V, N, C]; every column has its own alpha.
"""
from __future__ import annotations

import numpy as np


def cdot(a, b):
    """Column-wise <a, b> = sum over sites and components of conj(a) * b -> [C]."""
    return np.einsum("xnc,xnc->c", np.conj(a), b)


def _alpha(q, r):
    qq = cdot(q, q).real
    qr = cdot(q, r)
    return np.where(qq > 0, qr / np.where(qq > 0, qq, 1.0), 0.0)


def mr_null(op, psi0, n_iter, history=None):
    """n_iter MR steps on op(psi) = 0 starting from psi0 [V, N, C]; returns psi."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    r = -op.apply(psi)
    for _ in range(int(n_iter)):
        q = op.apply(r)
        a = _alpha(q, r)
        psi = psi + a * r
        r = r - a * q
        if history is not None:
            history.append(np.sqrt(cdot(r, r).real))
    return psi


def mr_solve(op, b, e0, n_iter):
    """n_iter MR steps on op(e) = b starting from e0; returns e."""
    e = np.array(e0, dtype=np.complex128, copy=True)
    rho = b - op.apply(e)
    for _ in range(int(n_iter)):
        q = op.apply(rho)
        a = _alpha(q, rho)
        e = e + a * rho
        rho = rho - a * q
    return e


def normalize_columns(psi):
    """psi_i <- psi_i / ||psi_i||_2 (columns with zero norm are left unchanged)."""
    n = np.sqrt(cdot(psi, psi).real)
    return psi / np.where(n > 0, n, 1.0)
