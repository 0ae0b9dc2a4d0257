"""Pins of the real-time propagation oracle (Sec. II.B rotation rule under
U_Q(theta) = exp(-i theta Q / 2)): exhaustive dense checks of one gate,
whole untruncated runs against the dense Heisenberg product, and the
conservation of sum c^2 (unitarity) without truncation."""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla

import itpp_workloads as W
from oracle import dense as D
from oracle import realtime as RT


def dense_of(S):
    return sum(c * D.pauli_matrix(P) for P, c in S.items())


@pytest.mark.parametrize("theta", [0.3, -1.1])
def test_gate_rule_exhaustive_two_qubits(theta):
    letters = ["".join(t) for t in itertools.product("IXYZ", repeat=2)]
    for Q in letters[1:]:
        U = sla.expm(-0.5j * theta * D.pauli_matrix(Q))
        for P in letters:
            want = U.conj().T @ D.pauli_matrix(P) @ U
            got = dense_of(dict(RT.gate_contributions_real(P, 1.0, Q, math.cos(theta), math.sin(theta))))
            assert np.abs(want - got).max() < 1e-13, (P, Q)


@pytest.mark.parametrize("n,periodic", [(3, False), (4, True)])
def test_untruncated_run_equals_dense_heisenberg_product(n, periodic):
    w = W.tfim_workload("t", n, 1.0, 0.7, periodic, 1, 0.05, 0.3, 0.0, 1 << 40)
    S0 = {"I" * n: 1.0, "Z" + "I" * (n - 1): 0.5, "X" * n: -0.25}
    S, _ = RT.evolve_real(S0, w.strings, w.alphas, w.schedule, 0.07, 3, 0.0, 1 << 40)
    O = dense_of(S0)
    for _ in range(3):
        for k, m in w.schedule:
            U = sla.expm(-0.5j * w.alphas[k] * m * 0.07 * D.pauli_matrix(w.strings[k]))
            O = U.conj().T @ O @ U
    assert np.abs(dense_of(S) - O).max() < 1e-12
    assert S["I" * n] == 1.0


def test_l2_norm_is_conserved_without_truncation():
    w = W.random_two_flip_workload("r", 6, 8, 4, 0.1, 3, 0.0, 1 << 40)
    S0 = {"I" * 6: 1.0, "XZIYII": 0.4, "IIZZII": -0.3}
    S, _ = RT.evolve_real(S0, w.strings, w.alphas, w.schedule, 0.13, 4, 0.0, 1 << 40)
    assert math.fsum(c * c for c in S.values()) == pytest.approx(math.fsum(c * c for c in S0.values()), rel=1e-13)
    assert len(S) > len(S0)
