"""Pauli-measurement tensor of a matrix product state (section 5.3) -- test
infrastructure, like the rest of this package.

For an n-qubit MPS u = [U_1, ..., U_n] the density matrix rho = u u^dagger is
an MPO with cores X_k(:, i, j, :) = U_k(:, i, :) kron conj(U_k(:, j, :)).  The
measurement tensor T*(a) = Tr(rho W_a), W_a = sigma_{a_1} kron ... kron
sigma_{a_n}, has the TT cores Y_k(:, a, :) = sum_{i,j} X_k(:, i, j, :)
sigma_a(j, i) (the trace pairs row i of rho with column i of W).  The cores
are complex while T* is real; `real_tt` writes the real part as a real TT of
twice the ranks and `measurement_truth` rounds it to the true ranks with the
TT-SVD of a TT (Algorithm 1), which is exact because the real tensor's
unfoldings have the same ranks as the complex ones.
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import tt

# the section's Pauli order: identity, X, Y, Z
PAULI = [np.array([[1, 0], [0, 1]], dtype=complex),
         np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]


def mpo_cores(mps: Sequence[np.ndarray]) -> List[np.ndarray]:
    """X_k(a a', i, j, b b') = U_k(a, i, b) conj(U_k(a', j, b'))."""
    out = []
    for u in mps:
        sl, d, sr = u.shape
        x = np.einsum("aib,cjd->acijbd", u, np.conj(u)).reshape(sl * sl, d, d, sr * sr)
        out.append(x)
    return out


def measurement_cores(mps: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Complex TT cores of T*(a) = Tr(rho W_a): Y_k(:, a, :) = sum_ij X_k(:, i, j, :) sigma_a(j, i)."""
    out = []
    for x in mpo_cores(mps):
        y = np.stack([np.einsum("pijq,ji->pq", x, s) for s in PAULI], axis=1)
        out.append(y)
    return out


def real_tt(cores: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Real TT (ranks doubled) of the real part of a complex TT.

    A row state a + i b times A + i B is (aA - bB) + i(aB + bA), i.e. the real
    pair [a, b] times [[A, B], [-B, A]]; the first core is the pair [Re, Im] and
    the last keeps the real part [[A], [-B]].
    """
    m = len(cores)
    out = []
    for k, c in enumerate(cores):
        a, b = c.real, c.imag
        if k == 0:
            out.append(np.concatenate([a, b], axis=2))
        elif k == m - 1:
            out.append(np.concatenate([a, -b], axis=0))
        else:
            top = np.concatenate([a, b], axis=2)
            bot = np.concatenate([-b, a], axis=2)
            out.append(np.concatenate([top, bot], axis=0))
    return out


def measurement_truth(mps: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Real TT cores of T* with ranks s_k^2 (left-orthogonal)."""
    ranks = [1] + [u.shape[2] ** 2 for u in mps[:-1]] + [1]
    return tt.tt_round(real_tt(measurement_cores(mps)), ranks)


def density_matrix(mps: Sequence[np.ndarray]) -> np.ndarray:
    """Dense rho = u u^dagger (tiny systems only); qubit 1 is the most significant bit."""
    u = mps[0]
    for c in mps[1:]:
        u = np.tensordot(u, c, axes=([u.ndim - 1], [0]))
    v = u.reshape(-1)
    return np.outer(v, np.conj(v))
