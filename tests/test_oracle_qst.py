"""Pins for the quantum-state-tomography workload (section 5.3): the TT of the
Pauli measurements equals Tr(rho W_a) computed from the dense density matrix,
is real, has TT ranks s^2, and its identity entry is Tr(rho)."""

import itertools
import math

import numpy as np

from oracle import qst, tt
from paper_2501_13385_amd import workloads as wl


def kron_all(ms):
    out = np.array([[1.0 + 0j]])
    for m in ms:
        out = np.kron(out, m)
    return out


def test_measurement_tt_equals_dense_trace():
    mps = wl.random_mps(3, 2, wl.make_rng(5))
    rho = qst.density_matrix(mps)
    cores = qst.measurement_cores(mps)
    truth = qst.measurement_truth(mps)
    full = tt.tt_full(truth)
    for a in itertools.product(range(4), repeat=3):
        w = kron_all([qst.PAULI[i] for i in a])
        ref = np.trace(rho @ w)
        assert abs(ref.imag) <= 1e-12 * abs(np.trace(rho))
        v = cores[0][:, a[0], :]
        for k in range(1, 3):
            v = v @ cores[k][:, a[k], :]
        assert abs(v[0, 0] - ref) <= 1e-12 * abs(np.trace(rho))
        assert abs(full[a] - ref.real) <= 1e-11 * abs(np.trace(rho))


def test_measurement_tensor_has_ranks_s_squared_and_trace_entry():
    mps = wl.random_mps(5, 2, wl.make_rng(6))
    truth = qst.measurement_truth(mps)
    assert tt.ranks_of(truth) == [1, 4, 4, 4, 4, 1]
    full = tt.tt_full(qst.real_tt(qst.measurement_cores(mps)))
    for i in range(1, 5):
        sv = np.linalg.svd(tt.separation(full, i), compute_uv=False)
        assert int(np.sum(sv > 1e-10 * sv[0])) == 4 and sv[3] > 1e-6 * sv[0]
    np.testing.assert_allclose(tt.tt_full(truth), full, atol=1e-12 * np.abs(full).max())
    rho = qst.density_matrix(mps)
    assert abs(full[(0,) * 5] - np.trace(rho).real) <= 1e-12 * abs(np.trace(rho))
