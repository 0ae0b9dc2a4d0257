"""Pauli-weight cutoff (ITPP_OPT_MAX_WEIGHT, Sec. II.B) on the GPU against
the oracles with the same cutoff, bit for bit: one- and two-word keys, the
cap binding across many tiles, FP32, a loaded state holding strings above
the cutoff, the real-time rule, and the option's errors."""
import pytest

import itpp_workloads as W
from oracle import c_oracle
from oracle import itpp as OR
from oracle import realtime as RT

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c_oracle.build(force=False)


def to_string(x, z, n):
    out = []
    for j in range(n):
        xb = (int(x[j >> 6]) >> (j & 63)) & 1
        zb = (int(z[j >> 6]) >> (j & 63)) & 1
        out.append("IXZY"[xb | (zb << 1)])
    return "".join(out)


def gpu_run(w, steps, wmax, **opts):
    e = P.engine_for(w)
    e.set_option("max_weight", wmax)
    for k, v in opts.items():
        e.set_option(k, v)
    st = e.evolve(w.dtau, steps)
    S = e.state()
    e.close()
    return st, S


@pytest.mark.parametrize("name,builder,steps,wmax", [
    ("tfim16_strang", lambda: W.tfim_workload("t", 16, 1.0, 0.9, False, 2, 0.05, 0.4, 1e-12, 1 << 20), 8, 3),
    ("tfim64_capped", lambda: W.config2(K=4096), 4, 2),
    ("tfim64_capped_w2", lambda: W.config2(K=3000), 6, 2),
    ("periodic64", lambda: W.tfim_workload("t", 64, 1.0, 1.0, True, 1, 0.02, 0.1, 1e-6, 20000), 5, 5),
    ("random100_y", lambda: W.random_two_flip_workload("r", 100, 16, 3, 0.1, 2, 1e-12, 3000), 2, 3),
    ("random64_y", lambda: W.random_two_flip_workload("r", 64, 20, 2, 0.1, 3, 1e-12, 5000), 3, 4),
])
def test_matches_oracle(name, builder, steps, wmax):
    w = builder()
    print(f"weight cutoff {name} n={w.n} K={w.K} steps={steps} wmax={wmax}", flush=True)
    st, S = gpu_run(w, steps, wmax)
    o = c_oracle.run_workload(w, n_steps=steps, max_weight=wmax)
    assert S == o.state()
    assert st["term_updates"] == o.term_updates()
    assert all(OR.pauli_weight(k) <= wmax for k in S)
    # the cutoff bites: without it the state holds heavier strings
    _, S_free = gpu_run(w, steps, 0)
    assert any(OR.pauli_weight(k) > wmax for k in S_free)


def test_shapes_and_graphs_agree():
    w = W.config2(K=4096)
    ref = gpu_run(w, 4, 2)[1]
    for opts in ({"gate_shape": 0}, {"gate_shape": 2}, {"graphs": 0}, {"speculation": 0}):
        assert gpu_run(w, 4, 2, **opts)[1] == ref, opts


def test_f32_matches_oracle():
    w = W.config2(K=3000)
    w.precision = "f32"
    st, S = gpu_run(w, 3, 2)
    o = c_oracle.run_workload(w, n_steps=3, max_weight=2)
    assert S == o.state()


def test_loaded_state_above_the_cutoff():
    """Strings of the loaded state above the cutoff are dropped by the first
    gate that produces them (their self outputs), as in the oracle."""
    w = W.tfim_workload("t", 12, 1.0, 0.9, True, 1, 0.05, 0.2, 1e-12, 1 << 20)
    x, z, c = W.synthetic_state_words(w.n, 600, seed=41, partner=w.strings[w.schedule[0][0]])
    S0 = {to_string(x[i], z[i], w.n): float(c[i]) for i in range(len(c))}
    assert max(OR.pauli_weight(k) for k in S0) > 4
    e = P.engine_for(w)
    e.set_option("max_weight", 4)
    e.load(S0)
    e.evolve(w.dtau, 2)
    got = e.state()
    e.close()
    ref, _ = OR.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 2, w.delta, w.K, S0=S0, max_weight=4)
    assert got == ref


def test_real_time_matches_oracle():
    w = W.tfim_workload("t", 12, 1.0, 0.7, False, 1, 0.05, 1.0, 1e-9, 1500)
    x, z, c = W.synthetic_state_words(w.n, 600, seed=31, partner=w.strings[w.schedule[0][0]])
    S0 = {to_string(x[i], z[i], w.n): float(c[i]) for i in range(len(c))}
    e = P.engine_for(w)
    e.load(S0)
    e.set_option("real_time", 1)
    e.set_option("max_weight", 5)
    e.evolve(0.11, 3)
    got = e.state()
    e.close()
    ref, _ = RT.evolve_real(S0, w.strings, w.alphas, w.schedule, 0.11, 3, w.delta, w.K, max_weight=5)
    assert got == ref


def test_option_errors():
    w = W.tfim_workload("t", 8, 1.0, 1.0, True, 1, 0.05, 0.1, 1e-9, 100)
    e = P.engine_for(w)
    for bad in (-1, 9, 2.5):
        with pytest.raises(P.ItppError):
            e.set_option("max_weight", bad)
    e.set_option("max_weight", 3)
    with pytest.raises(P.ItppError):
        e.set_adjoint(1)                  # no reverse sweep with a cutoff
    e.set_option("max_weight", 0)
    e.set_adjoint(1)
    with pytest.raises(P.ItppError):
        e.set_option("max_weight", 3)     # nor a cutoff with checkpoints
    e.close()
