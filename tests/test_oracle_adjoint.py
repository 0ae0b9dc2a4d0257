"""Pins of the reverse-mode oracle against independent derivatives: central
finite differences of the frozen-support forward map (truncation binding),
finite differences of the dense Trotterized state, the closed forms of the
commuting special cases h = 0 and J = 0, and the exact thermal variance
(specific heat) from exact diagonalisation.  CPU only."""
import math

import numpy as np
import pytest

import itpp_workloads as W
from oracle import adjoint as AD
from oracle import dense, itpp


def _fd_frozen(w, recs, obs, eps=1e-5):
    """Central differences of the frozen-support map for every alpha_k and dtau."""
    strs, coefs = obs

    def L(alphas, dtau):
        S = AD.forward_frozen(w.n, w.strings, recs, alphas, dtau)
        return itpp.expect(S, strs, coefs)

    da = []
    for k in range(len(w.alphas)):
        ap = list(w.alphas)
        am = list(w.alphas)
        ap[k] += eps
        am[k] -= eps
        da.append((L(ap, w.dtau) - L(am, w.dtau)) / (2 * eps))
    dd = (L(w.alphas, w.dtau + eps) - L(w.alphas, w.dtau - eps)) / (2 * eps)
    return da, dd


@pytest.mark.parametrize("seed,K,delta", [(0, 60, 1e-4), (3, 1 << 20, 2e-3), (5, 25, 0.0)])
def test_adjoint_matches_frozen_support_fd(seed, K, delta):
    """Truncation binding (cap or threshold): the adjoint equals central
    differences of the map with every gate's kept set replayed."""
    w = W.random_workload("r", 6, 8, seed, 0.2, 3, delta, K, max_weight=3, local=False)
    H = (w.strings, w.alphas)
    a, recs = AD.forward_record(w.n, w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, w.delta, w.K)
    assert any(len(r.kept) < len(itpp.apply_gate(r.a_in, w.strings[r.term], 1.1, 0.3)) for r in recs)
    L, dth, _ = AD.backward(w.n, w.strings, recs, a, *H)
    da, dd = AD.parameter_gradients(w.strings, w.alphas, recs, dth, w.dtau)
    fa, fd = _fd_frozen(w, recs, H)
    scale = max(1.0, max(abs(x) for x in fa))
    assert max(abs(x - y) for x, y in zip(da, fa)) < 1e-7 * scale
    assert abs(dd - fd) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("n,periodic,order", [(4, True, 1), (5, False, 2)])
def test_adjoint_matches_dense_trotter_fd(n, periodic, order):
    """Untruncated: the adjoint of <H> and <X_0> against central differences
    of the dense Trotterized state (independent of the Pauli machinery)."""
    w = W.tfim_workload("t", n, 1.0, 0.7, periodic, order, 0.05, 0.4, 0.0, 1 << 40)
    obs = {"H": (w.strings, w.alphas), "X0": (["X" + "I" * (n - 1)], [1.0])}
    eps = 1e-5
    for name, (strs, coefs) in obs.items():
        L, da, dd, _ = AD.gradients(w, strs, coefs)
        O = sum(c * dense.pauli_matrix(s) for s, c in zip(strs, coefs))

        def Ld(alphas, dtau):
            rho = dense.trotter_thermal(w.strings, alphas, w.schedule, dtau, w.n_steps)
            return dense.expectation(rho, O)

        assert abs(L - Ld(w.alphas, w.dtau)) < 1e-12
        fd = (Ld(w.alphas, w.dtau + eps) - Ld(w.alphas, w.dtau - eps)) / (2 * eps)
        assert abs(dd - fd) < 1e-7 * max(1.0, abs(fd)), name
        for k in (0, len(w.alphas) - 1):
            ap = list(w.alphas)
            am = list(w.alphas)
            ap[k] += eps
            am[k] -= eps
            fk = (Ld(ap, w.dtau) - Ld(am, w.dtau)) / (2 * eps)
            assert abs(da[k] - fk) < 1e-7 * max(1.0, abs(fk)), (name, k)


def _energy_derivs(w, J_terms, h_terms):
    """<H>, d<H>/dbeta, d<H>/dJ, d<H>/dh from the adjoint: alpha_ZZ = -J,
    alpha_X = -h, beta = N dtau with N fixed; the explicit derivative of the
    observable H with respect to J (or h) is -sum <ZZ> (or -sum <X>)."""
    L, da, dd, _ = AD.gradients(w, w.strings, w.alphas)
    a, _ = AD.forward_record(w.n, w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, w.delta, w.K)
    dbeta = dd / w.n_steps
    dJ = -sum(itpp.expect(a, [w.strings[k]], [1.0]) for k in J_terms) - sum(da[k] for k in J_terms)
    dh = -sum(itpp.expect(a, [w.strings[k]], [1.0]) for k in h_terms) - sum(da[k] for k in h_terms)
    return L, dbeta, dJ, dh


def test_h0_open_closed_form_derivatives():
    """h = 0, open chain: every term commutes, Trotter is exact and
    <H> = -J (n-1) tanh(beta J)."""
    n, J, beta = 6, 0.8, 0.7
    w = W.tfim_workload("t", n, J, 0.0, False, 1, 0.05, beta, 0.0, 1 << 40)
    nzz = n - 1
    L, dbeta, dJ, _ = _energy_derivs(w, range(nzz), range(nzz, len(w.strings)))
    t = math.tanh(beta * J)
    sech2 = 1.0 - t * t
    assert abs(L - (-J * nzz * t)) < 1e-13
    assert abs(dbeta - (-J * J * nzz * sech2)) < 1e-12
    assert abs(dJ - (-nzz * (t + beta * J * sech2))) < 1e-12


def test_j0_closed_form_derivatives():
    """J = 0: independent spins, <H> = -h n tanh(beta h)."""
    n, h, beta = 5, 1.3, 0.45
    w = W.tfim_workload("t", n, 0.0, h, True, 1, 0.05, beta, 0.0, 1 << 40)
    nzz = n
    L, dbeta, _, dh = _energy_derivs(w, range(nzz), range(nzz, len(w.strings)))
    t = math.tanh(beta * h)
    sech2 = 1.0 - t * t
    assert abs(L - (-h * n * t)) < 1e-13
    assert abs(dbeta - (-h * h * n * sech2)) < 1e-12
    assert abs(dh - (-n * (t + beta * h * sech2))) < 1e-12


def test_specific_heat_vs_exact_variance():
    """C = -beta^2 d<H>/dbeta equals beta^2 Var(H) of the exact thermal state
    up to the O(dtau^2) Trotter error."""
    n, beta = 6, 0.6
    w = W.tfim_workload("t", n, 1.0, 1.0, True, 2, 0.01, beta, 0.0, 1 << 40)
    L, dbeta, _, _ = _energy_derivs(w, range(n), range(n, 2 * n))
    H = dense.hamiltonian(w.strings, w.alphas)
    rho = dense.exact_thermal(H, beta)
    E = dense.expectation(rho, H)
    var = dense.expectation(rho, H @ H) - E * E
    C_adj = -beta * beta * dbeta
    C_ed = beta * beta * var
    assert abs(C_adj - C_ed) < 1e-3 * C_ed
    assert abs(L - E) < 1e-3 * abs(E)
