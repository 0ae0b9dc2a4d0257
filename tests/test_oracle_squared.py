"""Pins of the squared-state observable oracle (Sec. II.C, <O>_{2 tau}):
dense matrices for random states, the exact thermal state at twice the
imaginary time, and small cases worked by hand."""
import math

import numpy as np
import pytest

import itpp_workloads as W
from oracle import dense as D
from oracle import squared as SQ


def random_state(n, count, seed):
    rng = np.random.default_rng(seed)
    S = {"I" * n: 1.0}
    while len(S) < count:
        P = "".join(rng.choice(list("IXYZ"), size=n))
        S[P] = float(rng.uniform(-0.6, 0.6))
    return S


@pytest.mark.parametrize("n,count,seed", [(2, 9, 0), (3, 30, 1), (4, 80, 2)])
def test_matches_dense_traces(n, count, seed):
    S = random_state(n, count, seed)
    rho = sum(a * D.pauli_matrix(P) for P, a in S.items()) / 2 ** n
    obs = random_state(n, 6, seed + 10)
    strings, coefs = list(obs), list(obs.values())
    O = sum(o * D.pauli_matrix(Q) for Q, o in zip(strings, coefs))
    num, purity = SQ.squared_expectation(S, strings, coefs)
    r2 = rho @ rho
    assert purity == pytest.approx(2 ** n * np.trace(r2).real, rel=1e-13)
    assert num == pytest.approx(2 ** n * np.trace(O @ r2).real, rel=1e-12, abs=1e-14)


def test_exact_state_gives_the_thermal_value_at_twice_the_time():
    n, tau = 5, 0.35
    strings, alphas, _ = W.tfim_terms(n, 1.0, 0.8, True)
    H = D.hamiltonian(strings, alphas)
    S = D.pauli_coefficients(D.exact_thermal(H, tau), tol=1e-15)
    assert S["I" * n] == pytest.approx(1.0)
    num, purity = SQ.squared_expectation(S, strings, alphas)
    want = D.expectation(D.exact_thermal(H, 2 * tau), H)
    assert num / purity == pytest.approx(want, rel=1e-10)


def test_hand_cases():
    # rho ~ I + 0.5 X + 0.3 Y: Z anticommutes with X and Y and ZI = Z is absent
    S = {"I": 1.0, "X": 0.5, "Y": 0.3}
    assert SQ.squared_expectation(S, ["Z"], [1.0]) == (0.0, 1.0 + 0.25 + 0.09)
    # O = I gives the purity itself
    num, purity = SQ.squared_expectation(S, ["I"], [1.0])
    assert num == purity
    # O = X: X I = X and X X = I, each with sign +1: 2 * 1 * 0.5
    assert SQ.squared_expectation(S, ["X"], [1.0])[0] == pytest.approx(1.0)
    # two qubits, Z Z applied to X X: (Z X)(Z X) = (iY)(iY) = - Y Y
    S2 = {"II": 1.0, "XX": 0.25, "YY": 0.5}
    assert SQ.squared_expectation(S2, ["ZZ"], [1.0])[0] == pytest.approx(-2 * 0.25 * 0.5)
    assert math.isclose(SQ.squared_expectation(S2, ["ZZ"], [1.0])[1], 1 + 0.0625 + 0.25)
