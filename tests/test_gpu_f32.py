"""GPU parity of the single-precision form: the HIP engine with binary32
coefficients against the single-precision CPU oracle, element by element.

Every output coefficient is one binary32 product, or the binary32 sum of two
binary32 products, divided in binary64 by the identity coefficient and
rounded once to binary32, in the same order on both sides, so the states
must agree bit for bit (compared with ``==`` on the widened values)."""
import math

import pytest

import itpp_workloads as W
from oracle import c_oracle
from oracle import itpp as OR

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c_oracle.build(force=False)


def assert_same_state(S_ref, S_gpu):
    assert len(S_ref) == len(S_gpu)
    diff = [k for k in S_ref if S_gpu.get(k) != S_ref[k]]
    assert not diff, f"{len(diff)} coefficients differ, e.g. {diff[:3]} " \
                     f"{[(S_ref[k], S_gpu.get(k)) for k in diff[:3]]}"


def run_gpu(w, steps=None, **kw):
    e = P.engine_for(w, precision="f32", **kw)
    st = e.evolve(w.dtau, w.n_steps if steps is None else steps)
    return e, st, e.state()


def test_config1_f32_bitexact_and_observables():
    w = W.config1()
    e, st, S = run_gpu(w)
    o = c_oracle.run_workload(w, precision="f32")
    ref = o.state()
    assert_same_state(ref, S)
    assert len(S) == math.comb(16, 8)
    assert st["term_updates"] == o.term_updates()
    for name, (strs, coefs) in w.observables.items():
        g = e.expect(strs, coefs)
        r = OR.expect(ref, strs, coefs)
        assert abs(g - r) <= 1e-13 * max(1.0, abs(r)), name
    e.close()


def test_f32_stepwise_prefixes_match_python_oracle():
    w = W.config1()
    e = P.engine_for(w, precision="f32")
    S = None
    for step in range(3):
        e.evolve(w.dtau, 1)
        S, _ = OR.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 1, w.delta, w.K, S0=S,
                         precision="f32")
        assert_same_state({k: float(v) for k, v in S.items()}, e.state())
    e.close()


@pytest.mark.parametrize("n,terms,steps,seed", [(12, 14, 3, 1), (64, 20, 2, 2), (128, 18, 2, 4)])
def test_f32_random_hamiltonians_with_y_bitexact(n, terms, steps, seed):
    w = W.random_two_flip_workload("r", n, terms, seed, 0.1, steps, 1e-7, 1 << 20)
    e, st, S = run_gpu(w)
    ref = c_oracle.run_workload(w, precision="f32").state()
    assert_same_state(ref, S)
    e.close()


@pytest.mark.parametrize("K,steps", [(4096, 2), (777, 2), (20000, 1)])
def test_config3_shape_f32_capped_bitexact(K, steps):
    """n = 128 periodic (two-word keys), threshold 1e-7, reduced cap; binary32
    values tie far more often than binary64 ones, so the canonical tie-break
    at the cap is exercised on most gates."""
    w = W.config3(K=K)
    assert w.precision == "f32"
    e, st, S = run_gpu(w, steps=steps)
    o = c_oracle.run_workload(w, n_steps=steps)
    assert_same_state(o.state(), S)
    assert st["cap_hit"] == 1
    assert len(S) == K
    assert st["term_updates"] == o.term_updates()
    e.close()


def test_f32_massive_ties_h0():
    w = W.tfim_workload("t", 14, 1.0, 0.0, False, 1, 0.1, 0.6, 0.0, 200)
    e, st, S = run_gpu(w)
    ref, _ = OR.run_workload(w, precision="f32")
    assert_same_state({k: float(v) for k, v in ref.items()}, S)
    e.close()


def test_f32_massive_ties_h0_large_groups():
    w = W.tfim_workload("t", 16, 1.0, 0.0, False, 1, 0.1, 0.6, 0.0, 1500)
    e, st, S = run_gpu(w)
    ref, _ = OR.run_workload(w, precision="f32")
    assert_same_state({k: float(v) for k, v in ref.items()}, S)
    e.close()


@pytest.mark.parametrize("margin", [1.0, 0.5])
def test_f32_speculation_margin_does_not_change_results(margin):
    w = W.config3(K=3000)
    e = P.engine_for(w)
    e.set_option("spec_margin", margin)
    e.evolve(w.dtau, 2)
    S = e.state()
    e.close()
    e2 = P.engine_for(w)
    e2.set_option("speculation", 0)
    e2.evolve(w.dtau, 2)
    assert e2.state() == S
    e2.close()


def test_f32_and_f64_observables_close_without_cap():
    """Threshold-only truncation: the two precisions keep the same strings
    and every observable agrees within the binary32 rounding bound."""
    w = W.config1()
    w.delta = 1e-4
    e32, st, _ = run_gpu(w)
    e64 = P.engine_for(w, precision="f64")
    e64.evolve(w.dtau, w.n_steps)
    assert e32.num_terms() == e64.num_terms()
    G = st["n_gates"]
    for name, (strs, coefs) in w.observables.items():
        scale = sum(abs(c) for c in coefs)
        d = e32.expect(strs, coefs) - e64.expect(strs, coefs)
        assert abs(d) < 6 * G * 2.0 ** -24 * scale, name
    e32.close()
    e64.close()
