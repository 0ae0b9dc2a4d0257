"""Real-time gates (ITPP_OPT_REAL_TIME) on the GPU against the real-time
oracle (Sec. II.B rule), from states loaded with itpp_import: bit-exact with
truncation, and the l2 norm conserved without it."""
import math

import pytest

import itpp_workloads as W
from oracle import realtime as RT

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def to_string(x, z, n):
    out = []
    for j in range(n):
        xb = (int(x[j >> 6]) >> (j & 63)) & 1
        zb = (int(z[j >> 6]) >> (j & 63)) & 1
        out.append("IXZY"[xb | (zb << 1)])
    return "".join(out)


def start_state(w, count, seed):
    x, z, c = W.synthetic_state_words(w.n, count, seed=seed, partner=w.strings[w.schedule[0][0]])
    return {to_string(x[i], z[i], w.n): float(c[i]) for i in range(len(c))}


def engine(w, S0):
    e = P.Engine(w.n, w.delta, w.K)
    e.set_hamiltonian(w.strings, w.alphas)
    e.set_schedule(w.schedule)
    e.load(S0)
    e.set_option("real_time", 1)
    return e


@pytest.mark.parametrize("builder,steps,count,dt", [
    (lambda: W.tfim_workload("t", 12, 1.0, 0.7, False, 1, 0.05, 1.0, 1e-9, 1500), 3, 600, 0.11),
    (lambda: W.config2(K=1200), 1, 800, 0.07),
    (lambda: W.random_two_flip_workload("r", 100, 14, 3, 0.1, 2, 1e-9, 1500), 2, 700, 0.09),
])
def test_real_time_matches_oracle(builder, steps, count, dt):
    w = builder()
    S0 = start_state(w, count, seed=31)
    e = engine(w, S0)
    st = e.evolve(dt, steps)
    S, updates = RT.evolve_real(S0, w.strings, w.alphas, w.schedule, dt, steps, w.delta, w.K)
    assert e.state() == S
    assert st["term_updates"] == updates
    assert st["cap_hit"] == 1
    with pytest.raises(P.ItppError):   # the reverse sweep replays imaginary-time gates only
        e.backward(w.strings, w.alphas)
    e.close()


def test_real_time_conserves_the_l2_norm_and_switches_back():
    """n = 8 holds at most 4^8 strings, below the cap: nothing is truncated,
    so sum c^2 is conserved (unitarity) up to rounding."""
    from oracle import c_oracle

    w = W.tfim_workload("t", 8, 1.0, 0.7, True, 1, 0.05, 1.0, 0.0, 1 << 20)
    S0 = start_state(w, 300, seed=32)
    e = engine(w, S0)
    st = e.evolve(0.1, 4)
    assert st["cap_hit"] == 0
    S = e.state()
    assert len(S) > len(S0)
    assert math.fsum(v * v for v in S.values()) == pytest.approx(math.fsum(v * v for v in S0.values()), rel=1e-12)
    # back to imaginary time from the real-time result
    e.set_option("real_time", 0)
    e.load(S)
    e.evolve(0.05, 1)
    c_oracle.build(force=False)
    o = c_oracle.COracle(w.n)
    o.load(S)
    o.evolve(w.strings, w.alphas, w.schedule, 0.05, 1, 0.0, 1 << 20)
    assert e.state() == o.state()
    e.close()


def test_real_time_many_tiles_matches_oracle():
    """n = 64, K = 2^15, a loaded state of 30000 strings: an X gate's join
    holds the whole state (7 or more tiles of the gate kernel), a ZZ gate's
    two joins split it; six gates from X_0 on, the cap binding."""
    w = W.config2(K=1 << 15)
    sched = w.schedule[63:] + w.schedule[:63]
    x, z, c = W.synthetic_state_words(w.n, 30000, seed=33, partner=w.strings[sched[0][0]])
    S0 = {to_string(x[i], z[i], w.n): float(c[i]) for i in range(len(c))}
    e = P.Engine(w.n, w.delta, w.K)
    e.set_hamiltonian(w.strings, w.alphas)
    e.set_schedule(sched)
    e.load(S0)
    e.set_option("real_time", 1)
    st = e.evolve_gates(0.07, 6)
    S, updates = RT.evolve_real(S0, w.strings, w.alphas, sched[:6], 0.07, 1, w.delta, w.K)
    assert st["cap_hit"] == 1
    assert e.state() == S
    assert st["term_updates"] == updates
    e.close()
