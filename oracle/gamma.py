"""Dirac matrices in a chiral basis.

Paper, Sec. 2, Eq. (2): the projectors 1 +- gamma5 split the spin index so that
spins beta = 1,2 form chirality alpha = 0 and spins beta = 3,4 form alpha = 1.
That requires gamma5 = diag(1, 1, -1, -1), which holds in the chiral basis

  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = 1, 2, 3),
  gamma_4 = [[0, 1], [1, 0]],
  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.

Spin indices here are 0-based (beta = 0..3); gamma[mu] for mu = 0..3 is the
matrix of direction x, y, z, t.
"""
from __future__ import annotations

import numpy as np

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_Z = np.zeros((2, 2), dtype=np.complex128)
_I = np.eye(2, dtype=np.complex128)

gamma = np.array(
    [np.block([[_Z, -1j * s], [1j * s, _Z]]) for s in (_s1, _s2, _s3)]
    + [np.block([[_Z, _I], [_I, _Z]])]
)
gamma5 = gamma[0] @ gamma[1] @ gamma[2] @ gamma[3]
identity4 = np.eye(4, dtype=np.complex128)


def gamma5_full():
    """gamma5 acting on the 12 spin-colour components (index 3*spin + colour)."""
    return np.kron(gamma5, np.eye(3))
