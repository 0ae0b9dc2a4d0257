"""Host logic of the experiment drivers (CPU): the chain and schedule they
build equal the workload module's, and the K(N, eps0) selection."""
import pytest

import itpp_workloads as W
from paper_2601_14400_amd import experiments as X


@pytest.mark.parametrize("n,periodic", [(3, False), (3, True), (8, False), (12, True)])
@pytest.mark.parametrize("order", [1, 2])
def test_tfim_terms_and_schedule_match_the_workload_module(n, periodic, order):
    s1, a1, nzz1 = X.tfim_hamiltonian(n, 1.0, 0.5, periodic)
    s2, a2, nzz2 = W.tfim_terms(n, 1.0, 0.5, periodic)
    assert (s1, a1, nzz1) == (s2, a2, nzz2)
    assert X.tfim_schedule(nzz1, n, order) == W.tfim_schedule(nzz2, n, order)


@pytest.mark.parametrize("beta,dtau", [(3.0, 0.04), (20.0, 0.04), (0.24, 0.04), (0.08, 0.04), (1.0, 0.03)])
def test_step_count(beta, dtau):
    assert X.n_steps_for(beta, dtau) == W.n_steps_for(beta, dtau)


def test_min_k_for_error():
    runs = [
        {"K": 512, "beta": [0.08, 0.24], "energy_per_site": [-0.50, -0.60]},
        {"K": 1024, "beta": [0.08, 0.24], "energy_per_site": [-0.52, -0.70]},
        {"K": 2048, "beta": [0.08, 0.24], "energy_per_site": [-0.52, -0.705]},
    ]
    assert X.min_k_for_error(runs, 0.08, -0.52, 1e-2) == 1024
    assert X.min_k_for_error(runs, 0.24, -0.70, 1e-2) == 1024
    assert X.min_k_for_error(runs, 0.24, -0.80, 1e-2) is None
    assert X.min_k_for_error(runs, 0.08, -0.505, 0.05) == 512
