"""The plain C++ dictionary oracle agrees bit for bit with the Python oracle
and is pinned on its own to a closed form at a size the Python oracle does
not reach quickly.  CPU only."""
import math

import numpy as np
import pytest

import itpp_workloads as W
from oracle import c_oracle, itpp


@pytest.fixture(scope="module", autouse=True)
def _built():
    c_oracle.build(force=False)


def test_config1_prefix_bitexact():
    w = W.config1()
    S, st = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 8, w.delta, w.K)
    o = c_oracle.run_workload(w, n_steps=8)
    assert o.state() == S
    assert o.term_updates() == st["term_updates"]


@pytest.mark.parametrize("seed", [0, 7])
def test_random_capped_bitexact(seed):
    w = W.random_workload("r", 12, 14, seed, 0.15, 5, 1e-10, 150)
    S, _ = itpp.run_workload(w)
    o = c_oracle.run_workload(w)
    assert len(S) == 150
    assert o.state() == S


def test_config2_shape_capped_bitexact():
    w = W.config2(K=512)
    S, _ = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 1, w.delta, w.K)
    o = c_oracle.run_workload(w, n_steps=1)
    assert o.state() == S


def test_h0_open_closed_form_n16():
    n, J, beta = 16, 1.0, 0.5
    w = W.tfim_workload("t", n, J, 0.0, False, 1, 0.05, beta, 0.0, 1 << 40)
    o = c_oracle.run_workload(w)
    S = o.state()
    t = math.tanh(beta * J)
    assert len(S) == 2 ** (n - 1)
    for P, c in S.items():
        z = np.array([1 if a == "Z" else 0 for a in P])
        b = np.cumsum(z) % 2
        assert abs(c - t ** int(b[:-1].sum())) < 1e-14


def test_export_is_canonical_order():
    w = W.config1()
    o = c_oracle.run_workload(w, n_steps=3)
    strs, coef = o.export()
    keys = [itpp.canonical_key(s) for s in strs]
    assert keys == sorted(keys)
