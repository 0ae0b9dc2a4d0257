"""Squared-state observables on the GPU (itpp_expect_squared) against the
oracle's squared_expectation on the same state.

Both sides sum the same rounded terms o_j * (a_P * a_R) * s in different
orders with compensation, and |numerator| <= ||o||_1 * purity (since
|a_P a_R| <= (a_P^2 + a_R^2) / 2), so the numerator is compared to
1e-12 * ||o||_1 * purity and the purity to 1e-13 relative."""
import numpy as np
import pytest

import itpp_workloads as W
from oracle import c_oracle
from oracle import squared as SQ

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c_oracle.build(force=False)


def random_observable(n, count, seed, weight):
    rng = np.random.default_rng(seed)
    strings, coefs = [], []
    for _ in range(count):
        s = ["I"] * n
        for q in rng.choice(n, size=weight, replace=False):
            s[q] = "XYZ"[int(rng.integers(0, 3))]
        strings.append("".join(s))
        coefs.append(float(rng.uniform(-1, 1)))
    return strings, coefs


@pytest.mark.parametrize("builder,steps", [
    (lambda: W.config1(), 4),
    (lambda: W.config2(K=3000), 2),
    (lambda: W.config3(K=2000), 1),
    (lambda: W.random_two_flip_workload("r", 12, 14, 1, 0.05, 3, 1e-9, 3000), 3),
    (lambda: W.random_two_flip_workload("r", 100, 16, 3, 0.1, 2, 1e-12, 4000), 2),
])
def test_squared_matches_oracle(builder, steps):
    w = builder()
    e = P.engine_for(w)
    e.evolve(w.dtau, steps)
    o = c_oracle.run_workload(w, n_steps=steps)
    S = o.state()
    assert e.state() == S
    cases = list(w.observables.values()) + [random_observable(w.n, 12, 5, min(w.n, 3)),
                                            random_observable(w.n, 4, 6, min(w.n, 7))]
    for strings, coefs in cases:
        val, pur = e.expect_squared(strings, coefs)
        num_o, pur_o = SQ.squared_expectation(S, strings, coefs)
        assert pur == pytest.approx(pur_o, rel=1e-13)
        bound = 1e-12 * sum(abs(c) for c in coefs) * pur_o
        assert abs(val * pur - num_o) <= bound + 1e-300
    e.close()


def test_squared_edge_cases():
    w = W.config2(K=500)
    e = P.engine_for(w)
    e.evolve(w.dtau, 1)
    S = e.state()
    purity = sum(v * v for v in S.values())
    val, pur = e.expect_squared([], [])
    assert val == 0.0 and pur == pytest.approx(purity, rel=1e-13)
    val, pur = e.expect_squared(["I" * w.n], [2.0])
    assert val == pytest.approx(2.0, rel=1e-15)
    with pytest.raises(P.ItppError):
        e.expect_squared(["I" * w.n], [float("nan")])
    e.close()


def test_squared_untruncated_state_gives_the_thermal_energy_at_twice_beta():
    """Untruncated 12-site chain (J = 1, h = 0.5, dtau = 0.02) evolved to
    beta = 1: the squared state gives <H> at beta = 2, equal to the exact
    free-fermion thermal energy up to the first-order Trotter error."""
    from oracle import freefermion as FF
    from paper_2601_14400_amd import experiments as X

    n = 12
    strings, alphas, n_zz = X.tfim_hamiltonian(n, 1.0, 0.5, False)
    e = P.Engine(n, 0.0, 1 << 23)
    e.set_hamiltonian(strings, alphas)
    e.set_schedule(X.tfim_schedule(n_zz, n, 1))
    e.evolve(0.02, 50)
    val, pur = e.expect_squared(strings, alphas)
    exact2 = FF.thermal_energy(n, 1.0, 0.5, 2.0, False)
    exact1 = FF.thermal_energy(n, 1.0, 0.5, 1.0, False)
    assert abs(val - exact2) / abs(exact2) < 1e-3
    assert abs(e.expect(strings, alphas) - exact1) / abs(exact1) < 1e-3
    assert abs(exact2 - exact1) / abs(exact1) > 1e-2  # the two temperatures are told apart
    e.close()
