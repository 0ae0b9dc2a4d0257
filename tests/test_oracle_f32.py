"""Pins of the single-precision oracle form.  Every coefficient of the FP32
form must be a binary32 number, must differ from the FP64 result only by the
rounding error of binary32 arithmetic (at most a few units of 2^-24 per gate,
since every coefficient is bounded by the identity coefficient), and the
Python and C++ oracles must agree bit for bit.  The FP64 oracle and the dense
Trotterized state it is pinned to are the independent reference.  CPU only."""
import math

import numpy as np
import pytest

import itpp_workloads as W
from oracle import c_oracle, dense, itpp

U32 = 2.0 ** -24   # unit roundoff of binary32


@pytest.fixture(scope="module", autouse=True)
def _built():
    c_oracle.build(force=False)


def _is_f32(x):
    return float(np.float32(x)) == float(x)


def _max_err(S, A):
    keys = set(S) | set(A)
    return max(abs(float(S.get(k, 0.0)) - float(A.get(k, 0.0))) for k in keys)


@pytest.mark.parametrize("n,periodic,order", [(4, True, 1), (5, False, 2), (6, True, 1)])
def test_f32_untruncated_vs_dense(n, periodic, order):
    """Untruncated FP32 run vs the dense Trotterized state: error within the
    binary32 rounding bound, and strictly nonzero (the run is really FP32)."""
    w = W.tfim_workload("t", n, 1.0, 0.7, periodic, order, 0.05, 0.6, 0.0, 1 << 40)
    S, st = itpp.run_workload(w, precision="f32")
    rho = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    A = dense.pauli_coefficients(rho, tol=1e-14)
    G = st["n_gates"]
    err = _max_err(S, A)
    assert 0.0 < err < 6 * G * U32
    assert all(_is_f32(c) for c in S.values())
    assert float(S["I" * n]) == 1.0


def test_f32_config1_observables_vs_dense():
    w = W.config1()
    S, st = itpp.run_workload(w, precision="f32")
    rho_t = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    G = st["n_gates"]
    for name, (strs, coefs) in w.observables.items():
        O = sum(c * dense.pauli_matrix(s) for s, c in zip(strs, coefs))
        v = itpp.expect(S, strs, coefs)
        scale = sum(abs(c) for c in coefs)
        assert abs(v - dense.expectation(rho_t, O)) < 6 * G * U32 * scale, name


def test_f32_single_site_closed_form():
    """J = 0: H = -h sum X_j, every site evolves alone and a_{X_j} follows
    the tanh addition law, so a = tanh(beta h) exactly in real arithmetic."""
    n, h, dtau, beta = 3, 0.8, 0.05, 1.0
    w = W.tfim_workload("t", n, 0.0, h, False, 1, dtau, beta, 0.0, 1 << 40)
    S, st = itpp.run_workload(w, precision="f32")
    want = math.tanh(beta * h)
    G_site = w.n_steps
    for j in range(n):
        P = "I" * j + "X" + "I" * (n - 1 - j)
        assert abs(float(S[P]) - want) < 6 * G_site * U32
    # products of single-site factors
    P = "X" * n
    assert abs(float(S[P]) - want ** n) < 6 * n * G_site * U32


@pytest.mark.parametrize("seed", [0, 5])
def test_f32_python_c_bitexact_capped(seed):
    w = W.random_workload("r", 12, 14, seed, 0.15, 5, 1e-6, 150)
    S, _ = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, w.delta, w.K,
                       precision="f32")
    o = c_oracle.run_workload(w, precision="f32")
    assert len(S) == 150
    assert o.state() == {k: float(v) for k, v in S.items()}


def test_f32_python_c_bitexact_config1_prefix():
    w = W.config1()
    S, st = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 5, w.delta, w.K,
                        precision="f32")
    o = c_oracle.run_workload(w, n_steps=5, precision="f32")
    assert o.state() == {k: float(v) for k, v in S.items()}
    assert o.term_updates() == st["term_updates"]


def test_f32_config3_shape_python_c_bitexact():
    w = W.config3(K=512)
    assert w.precision == "f32" and w.n == 128
    S, _ = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 1, w.delta, w.K,
                       precision="f32")
    o = c_oracle.run_workload(w, n_steps=1)
    assert len(S) == 512
    assert o.state() == {k: float(v) for k, v in S.items()}


def test_f32_thresholded_close_to_f64():
    """Threshold truncation only: both precisions keep the same strings here
    and every observable agrees within the binary32 rounding bound."""
    w = W.config1()
    w.delta = 1e-4
    S32, st = itpp.run_workload(w, precision="f32")
    S64, _ = itpp.run_workload(w, precision="f64")
    assert set(S32) == set(S64)
    G = st["n_gates"]
    for name, (strs, coefs) in w.observables.items():
        scale = sum(abs(c) for c in coefs)
        d = itpp.expect(S32, strs, coefs) - itpp.expect(S64, strs, coefs)
        assert abs(d) < 6 * G * U32 * scale, name
