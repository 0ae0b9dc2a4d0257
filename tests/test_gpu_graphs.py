"""Step graphs: Trotter steps replayed from a recorded HIP graph give the
same states, bit for bit, as the same gates launched one by one (and as the
oracle), on the null stream (private capturable stream joined by events)
and on a caller's stream, across speculation retries, readouts, resets and
option changes."""
import pytest

import itpp_workloads as W
from oracle import c_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c_oracle.build(force=False)


def run(w, steps, graphs, **opts):
    e = P.engine_for(w)
    e.set_option("graphs", 1 if graphs else 0)
    for k, v in opts.items():
        e.set_option(k, v)
    st = e.evolve(w.dtau, steps)
    S = e.state()
    e.close()
    return st, S


CASES = {
    # 8 qubits periodic (16 gates a step), untruncated
    "config1": (W.config1, 20),
    # 16 qubits open chain (31 gates a step: two steps per graph)
    "tfim16_open_odd": (lambda: W.tfim_workload("t", 16, 1.0, 0.9, False, 1, 0.05, 0.6, 1e-9, 2000), 12),
    # 64 qubits open Strang (190 gates a step), cap binding, speculative
    "tfim64_capped": (lambda: W.config2(K=4096), 6),
    # 100 qubits (two-word keys), Y and XZ terms, cap binding
    "random100": (lambda: W.random_two_flip_workload("r", 100, 16, 3, 0.1, 8, 1e-12, 3000), 8),
    # periodic 64 qubits (128 gates a step), cap binding
    "tfim64_periodic": (lambda: W.tfim_workload("t", 64, 1.0, 1.0, True, 1, 0.02, 0.2, 1e-6, 5000), 10),
}


@pytest.mark.parametrize("name", list(CASES))
def test_replays_match_launches_and_oracle(name):
    builder, steps = CASES[name]
    w = builder()
    print(f"graphs {name} n={w.n} steps={steps}", flush=True)
    st_g, S_g = run(w, steps, True)
    st_d, S_d = run(w, steps, False)
    # recorded at the start of the third step (the first whose bit order
    # repeats); a redone speculative gate runs the rest of its step directly
    assert st_g["graph_steps"] >= (steps - 2 if st_g["spec_retries"] == 0 else 1), st_g
    assert st_d["graph_steps"] == 0
    assert S_g == S_d
    assert st_g["term_updates"] == st_d["term_updates"]
    assert st_g["n_gates"] == st_d["n_gates"]
    ref = c_oracle.run_workload(w, n_steps=steps).state()
    assert S_g == ref


def test_retries_inside_replayed_steps():
    """Margin 1 (no slack below the predicted K-th value) makes speculative
    gates fail and be redone; a failure inside a replayed step resumes from
    the failed gate with single launches and returns to replays at the next
    step."""
    w = W.config2(K=4096)
    st_g, S_g = run(w, 8, True, spec_margin=1.0)
    st_d, S_d = run(w, 8, False, spec_margin=1.0)
    print("retries", st_g["spec_retries"], st_d["spec_retries"], "graph steps", st_g["graph_steps"], flush=True)
    assert st_g["graph_steps"] > 0
    assert S_g == S_d


def test_caller_stream():
    import torch

    w = W.config2(K=4096)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        e = P.engine_for(w)
        st = e.evolve(w.dtau, 5)
        S = e.state()
        e.close()
    torch.cuda.synchronize()
    assert st["graph_steps"] >= 1
    _, S_d = run(w, 5, False)
    assert S == S_d


def test_interleaved_calls_and_resets():
    """Split runs, readouts between them, a reset, an option change and a
    different dtau all leave the results of one-by-one launches."""
    w = W.tfim_workload("t", 64, 1.0, 1.0, True, 1, 0.02, 0.2, 1e-6, 5000)
    e = P.engine_for(w)
    e.evolve(w.dtau, 3)
    e.expect(w.strings, w.alphas)
    e.evolve(w.dtau, 4)
    a = e.state()
    e.reset()
    e.evolve(w.dtau, 7)
    b = e.state()
    e.set_option("gate_shape", 0)          # drops the recorded step
    e.evolve(w.dtau, 3)
    c = e.state()
    e.evolve(1.5 * w.dtau, 3)              # another dtau: recorded anew
    d = e.state()
    e.close()
    r = P.engine_for(w)
    r.set_option("graphs", 0)
    r.evolve(w.dtau, 7)
    ra = r.state()
    r.set_option("gate_shape", 0)
    r.evolve(w.dtau, 3)
    rc = r.state()
    r.evolve(1.5 * w.dtau, 3)
    rd = r.state()
    r.close()
    assert a == ra and b == ra and c == rc and d == rd


def test_real_time_replays():
    w = W.tfim_workload("t", 64, 1.0, 1.0, True, 1, 0.05, 0.3, 1e-9, 20000)
    x, z, c = W.synthetic_state_words(w.n, 3000, seed=7, partner=w.strings[w.schedule[0][0]])
    out = []
    for graphs in (1, 0):
        e = P.engine_for(w)
        e.set_option("graphs", graphs)
        e.set_option("real_time", 1)
        e.import_words(x, z, c)
        st = e.evolve(w.dtau, 5)
        out.append((st["graph_steps"], e.state()))
        e.close()
    assert out[0][0] >= 1 and out[1][0] == 0
    assert out[0][1] == out[1][1]


def test_batch_instances_replay_steps():
    ws = W.config4_instances(seed=1, count=6, K=3000)
    steps = [5] * len(ws)
    b = P.batch_for(ws)
    st = b.evolve([w.dtau for w in ws], steps)
    for i, e in enumerate(b.instances):
        _, S = run(ws[i], steps[i], False)
        assert e.state() == S, i
        assert st[i]["graph_steps"] >= 1, (i, st[i])
    b.close()
