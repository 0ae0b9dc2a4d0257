"""itpp_expect_squared_noalloc (the entry point that allocates nothing)
against itpp_expect_squared on the same state: the same tables, kernels and
block partition, so the two agree bit for bit; both are also held to the
oracle's squared_expectation within the bound of the squared-state tests.
Two calls in a row, the second with fewer observable strings, then a second
context on the same GPU (one shared scratch area)."""
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


def check(e, S, strings, coefs):
    v0, p0 = e.expect_squared(strings, coefs)
    v1, p1 = e.expect_squared(strings, coefs, noalloc=True)
    assert v1 == v0 and p1 == p0
    num_o, pur_o = SQ.squared_expectation(S, strings, coefs)
    assert p1 == pytest.approx(pur_o, rel=1e-13)
    assert abs(v1 * p1 - num_o) <= 1e-12 * sum(abs(c) for c in coefs) * pur_o


@pytest.mark.parametrize("builder,steps", [
    (lambda: W.config2(K=3000), 2),
    (lambda: W.random_two_flip_workload("r", 100, 16, 3, 0.1, 2, 1e-12, 4000), 2),
])
def test_noalloc_matches_squared(builder, steps):
    w = builder()
    e = P.engine_for(w)
    e.evolve(w.dtau, steps)
    o = c_oracle.run_workload(w, n_steps=steps)
    S = o.state()
    assert e.state() == S
    big = random_observable(w.n, 300, 7, min(w.n, 3))
    small = random_observable(w.n, 5, 8, min(w.n, 2))
    check(e, S, *big)
    check(e, S, *small)
    for strings, coefs in w.observables.values():
        check(e, S, strings, coefs)
    # a second context on the same GPU shares the scratch area
    e2 = P.engine_for(w)
    e2.evolve(w.dtau, 1)
    o2 = c_oracle.run_workload(w, n_steps=1)
    check(e2, o2.state(), *small)
    check(e, S, *big)
    e2.close()
    e.close()


def test_noalloc_limits():
    w = W.config2(K=500)
    e = P.engine_for(w)
    e.evolve(w.dtau, 1)
    many = random_observable(w.n, 4097, 9, 1)
    with pytest.raises(P.ItppError):
        e.expect_squared(*many, noalloc=True)
    wide = (["X" * w.n] * 1025, [1.0] * 1025)   # 65600 sites in total
    with pytest.raises(P.ItppError):
        e.expect_squared(*wide, noalloc=True)
    ok = (["X" * w.n] * 1024, [1.0] * 1024)     # exactly 65536 sites
    v0, p0 = e.expect_squared(*ok)
    assert e.expect_squared(*ok, noalloc=True) == (v0, p0)
    assert e.expect_squared([], [], noalloc=True) == e.expect_squared([], [])
    e.close()
