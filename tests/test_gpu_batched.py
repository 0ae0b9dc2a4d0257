"""Batched form: instances evolved concurrently in one arena are
bit-identical to single-instance runs (and to the oracle), for every gate
kernel shape and worker count the autotuner can choose."""
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


def small_instances(count=8, K=3000):
    ws = W.config4_instances(seed=1, count=count, K=K)
    ws[1].precision = "f32"
    return ws


def single_states(ws, steps, **opts):
    out = []
    for w, k in zip(ws, steps):
        e = P.engine_for(w)
        for name, v in opts.items():
            e.set_option(name, v)
        e.evolve(w.dtau, k)
        out.append(e.state())
        e.close()
    return out


@pytest.mark.parametrize("workers", [1, 4, 8])
def test_batch_matches_single_runs(workers):
    ws = small_instances()
    steps = [2 + (i % 3) for i in range(len(ws))]
    b = P.batch_for(ws)
    b.set_workers(workers)
    st = b.evolve([w.dtau for w in ws], steps)
    ref = single_states(ws, steps)
    for i, e in enumerate(b.instances):
        assert e.state() == ref[i], i
        assert st[i]["n_gates"] == steps[i] * 2 * ws[i].n
    b.close()


def test_batch_instance_matches_oracle():
    ws = small_instances(count=3, K=1500)
    b = P.batch_for(ws)
    b.evolve([w.dtau for w in ws], [2, 2, 2])
    for i in (0, 2):
        ref = c_oracle.run_workload(ws[i], n_steps=2).state()
        assert b.instances[i].state() == ref
    b.close()


@pytest.mark.parametrize("builder,steps", [
    (lambda: W.config2(K=4096), 3),
    (lambda: W.random_two_flip_workload("r", 100, 16, 3, 0.1, 2, 1e-12, 5000), 2),
    (lambda: W.config3(K=3000), 1),
])
def test_gate_shapes_agree(builder, steps):
    """Shapes 0, 1 and 2 and the automatic choice (the default) store the
    same state."""
    w = builder()
    ref = single_states([w], [steps], gate_shape=0)[0]
    for shape in (1, 2, 3):
        assert single_states([w], [steps], gate_shape=shape)[0] == ref, shape
    assert single_states([w], [steps])[0] == ref


def test_automatic_shape_across_its_switch():
    """The automatic shape runs the layer kernel while the state is small
    and shape 1 once it has passed 2^19 strings (recording the step graph
    anew); the state matches both fixed shapes bit for bit."""
    w = W.config2(K=1 << 20)
    steps = 40
    print(f"automatic shape n={w.n} K={w.K} steps={steps}", flush=True)
    auto = single_states([w], [steps])[0]
    assert len(auto) > (1 << 19)
    assert single_states([w], [steps], gate_shape=1)[0] == auto
    assert single_states([w], [steps], gate_shape=2)[0] == auto


def test_autotune_then_evolve():
    ws = small_instances(count=6, K=2000)
    b = P.batch_for(ws)
    shape, workers, grid_div, rate = b.autotune([w.dtau for w in ws], 30, 30)
    assert 0 <= shape < 9 and workers in (2, 4, 8, 16) and grid_div in (1, 2, 4, 8) and rate > 0
    steps = [2] * len(ws)
    b.evolve([w.dtau for w in ws], steps)
    ref = single_states(ws, steps)
    for i, e in enumerate(b.instances):
        assert e.state() == ref[i]
    b.close()


@pytest.mark.parametrize("shape,grid_div", [(0, 8), (1, 4), (2, 2)])
def test_grid_divisor_keeps_results(shape, grid_div):
    """A smaller gate-kernel grid (fewer workgroups taking the same tiles)
    changes no result, for every shape."""
    w = W.config2(K=4096)
    a = single_states([w], [3], gate_shape=shape)[0]
    b = single_states([w], [3], gate_shape=shape, grid_div=grid_div)[0]
    assert a == b


def test_batch_errors():
    with pytest.raises(P.ItppError):
        P.Batch([dict(n_qubits=0, threshold=1e-6, max_terms=100)])
    b = P.Batch([dict(n_qubits=8, threshold=1e-6, max_terms=100)])
    with pytest.raises(P.ItppError):
        b.set_workers(0)
    with pytest.raises(P.ItppError):
        b.evolve([0.05], [1])   # no schedule on the instance
    b.close()
