"""Pins of the oracle's Pauli-weight cutoff (second truncation rule of
Sec. II.B): strings with more non-identity letters than the cutoff are
dropped after every gate, with the coefficient threshold and before the cap.

* dense matrices: the cutoff is a linear projection in the Pauli basis, so
  untruncated ITPP with a cutoff equals the dense Trotter product with that
  projection after every gate (matrix exponentials, no Pauli-rule code);
* TFIM chains under the same dense projection, with the support check
  that cutoff 1 keeps span{I, X_i};
* a cutoff at or above n changes nothing;
* the C++ twin agrees bit for bit, with the cap binding."""
import pytest

import itpp_workloads as W
from oracle import c_oracle
from oracle import dense as D
from oracle import itpp as OR


def random_small(n, seed):
    strings, alphas = W.random_hamiltonian(n, 2 * n + 1, seed, max_weight=3)
    sched = [(k, 1.0) for k in range(len(strings))]
    return strings, alphas, sched


@pytest.mark.parametrize("n,seed,wmax,steps", [(3, 1, 1, 3), (3, 2, 2, 4), (4, 3, 2, 3), (4, 4, 3, 2)])
def test_matches_dense_projection(n, seed, wmax, steps):
    strings, alphas, sched = random_small(n, seed)
    S, _ = OR.evolve(n, strings, alphas, sched, 0.15, steps, 0.0, 10 ** 9, max_weight=wmax)
    ref = D.weight_projected_trotter(strings, alphas, sched, 0.15, steps, wmax)
    assert all(OR.pauli_weight(P) <= wmax for P in S)
    keys = set(S) | {P for P, v in ref.items() if abs(v) > 1e-13}
    err = max(abs(S.get(P, 0.0) - ref.get(P, 0.0)) for P in keys)
    assert err < 1e-12, err
    # the cutoff really bites: the unconstrained state has heavier strings
    S_all, _ = OR.evolve(n, strings, alphas, sched, 0.15, steps, 0.0, 10 ** 9)
    assert any(OR.pauli_weight(P) > wmax for P in S_all)


@pytest.mark.parametrize("periodic,order,wmax", [(True, 1, 1), (False, 2, 2), (True, 1, 3)])
def test_tfim_matches_dense_projection(periodic, order, wmax):
    """TFIM chains (first order and Strang) against the dense projection;
    with cutoff 1 the state stays in span{I, X_i}: a ZZ gate sends I only to
    weight 2 (dropped) and leaves X_i alone."""
    n, J, h, dtau, beta = 5, 0.8, 0.7, 0.05, 0.4
    w = W.tfim_workload("t", n, J, h, periodic, order, dtau, beta, 0.0, 10 ** 6)
    S, _ = OR.run_workload(w, max_weight=wmax)
    ref = D.weight_projected_trotter(w.strings, w.alphas, w.schedule, dtau, w.n_steps, wmax)
    keys = set(S) | {P for P, v in ref.items() if abs(v) > 1e-13}
    assert max(abs(S.get(P, 0.0) - ref.get(P, 0.0)) for P in keys) < 1e-12
    if wmax == 1:
        assert set(S) == {"I" * n} | {"I" * i + "X" + "I" * (n - 1 - i) for i in range(n)}


def test_cutoff_at_n_changes_nothing():
    w = W.tfim_workload("t", 6, 1.0, 0.9, True, 1, 0.05, 0.3, 1e-9, 300)
    a, _ = OR.run_workload(w)
    b, _ = OR.run_workload(w, max_weight=6)
    assert a == b


@pytest.mark.parametrize("wmax,K", [(2, 10 ** 6), (3, 150), (4, 400)])
def test_cpp_twin_bitwise(wmax, K):
    c_oracle.build(force=False)
    w = W.tfim_workload("t", 10, 1.0, 0.9, False, 2, 0.05, 0.3, 1e-10, K)
    S, _ = OR.run_workload(w, max_weight=wmax)
    o = c_oracle.run_workload(w, max_weight=wmax)
    assert o.state() == S
    assert all(OR.pauli_weight(P) <= wmax for P in S)
