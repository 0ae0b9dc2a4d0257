"""GPU reverse sweep against the reverse-mode oracle.

The forward states are bit-identical to the oracle's, so both sides hold
the same kept sets; the per-gate dL/dtheta are sums over the state taken in
different orders (compensated on both sides), so they are compared to a
tolerance relative to the largest one.  Checkpoint intervals change only
which states are recomputed, never a result: those runs must agree exactly."""
import math

import numpy as np
import pytest

import itpp_workloads as W
from oracle import adjoint as AD
from oracle import c_oracle
from oracle import itpp as OR

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def gpu_backward(w, obs, steps, every, want_theta=True):
    e = P.engine_for(w)
    e.set_adjoint(every)
    st = e.evolve(w.dtau, steps)
    out = e.backward(*obs, want_theta=want_theta)
    return e, st, out


def check_against_oracle(w, obs, steps, every):
    e, st, (L, da, dd, dth) = gpu_backward(w, obs, steps, every)
    Lr, dar, ddr, dthr = AD.gradients(w, *obs, n_steps=steps)
    assert len(dth) == len(dthr) == st["n_gates"]
    scale = max(1e-300, max(abs(v) for v in dthr))
    err = max(abs(a - b) for a, b in zip(dth, dthr))
    assert err <= TOL * scale, (err, scale)
    assert abs(L - Lr) <= 1e-13 * max(1.0, abs(Lr))
    sa = max(1.0, max(abs(v) for v in dar))
    assert max(abs(a - b) for a, b in zip(da, dar)) <= TOL * sa
    assert abs(dd - ddr) <= TOL * max(1.0, abs(ddr))
    return e


@pytest.mark.parametrize("every", [1, 2])
def test_tfim_open_capped_matches_oracle(every):
    w = W.tfim_workload("t", 24, 1.0, 0.9, False, 2, 0.05, 0.15, 1e-6, 600)
    e = check_against_oracle(w, (w.strings, w.alphas), 3, every)
    e.close()


@pytest.mark.parametrize("n,terms,seed,K", [(12, 14, 1, 200), (64, 16, 2, 400), (100, 14, 3, 300)])
def test_random_hamiltonians_match_oracle(n, terms, seed, K):
    """Y and XZ terms, one- and two-word keys, binding cap."""
    w = W.random_two_flip_workload("r", n, terms, seed, 0.1, 2, 1e-9, K)
    obs = (w.strings[:3] + ["X" + "I" * (n - 1)], [0.7, -1.1, 0.4, 2.0])
    e = check_against_oracle(w, obs, 2, 1)
    e.close()


@pytest.mark.parametrize("n,K", [(64, 1 << 15), (100, 1 << 14)])
def test_reverse_sweep_many_tiles_matches_oracle(n, K):
    """Periodic TFIM (the adjoint benchmark's model), J = h = 1, dtau = 0.02,
    threshold 1e-6, two Trotter steps with the cap binding on every gate.
    The gate kernel's tile is 4000 merged strings for one-word keys and 2000
    for two-word keys, so an X gate's join (the whole state) spans 8 or more
    tiles: the reverse kernel's look-back positions and its gather of
    lambda' cross many tiles.  Compared with the C++ reverse sweep."""
    w = W.tfim_workload("t", n, 1.0, 1.0, True, 1, 0.02, 0.04, 1e-6, K)
    obs = (w.strings, [a / n for a in w.alphas])
    print(f"reverse sweep n={n} K={K}", flush=True)
    e, st, (L, da, dd, dth) = gpu_backward(w, obs, 2, 1)
    assert st["cap_hit"] == 1 and st["n_terms"] == K
    S = e.state()
    e.close()
    c_oracle.build(force=False)
    o = c_oracle.COracle(n)
    Lr, dar, ddr, dthr = o.gradients(w, *obs, n_steps=2)
    assert o.state() == S
    assert len(dth) == len(dthr) == st["n_gates"]
    scale = max(abs(v) for v in dthr)
    assert max(abs(a - b) for a, b in zip(dth, dthr)) <= TOL * scale
    assert abs(L - Lr) <= 1e-13 * max(1.0, abs(Lr))
    sa = max(1.0, max(abs(v) for v in dar))
    assert max(abs(a - b) for a, b in zip(da, dar)) <= TOL * sa
    assert abs(dd - ddr) <= TOL * max(1.0, abs(ddr))


def test_checkpoint_interval_does_not_change_results():
    """Checkpoint intervals and workspace sizes change only what is
    recomputed: with the default workspace every segment's states fit and
    each segment is recomputed once; a 2 MB workspace forces blocks of about
    sqrt(L) gates from sub-checkpoints (two recomputations)."""
    w = W.tfim_workload("t", 20, 1.0, 1.1, True, 1, 0.05, 0.3, 1e-6, 500)
    obs = (w.strings, w.alphas)
    ref = None
    for every, ws in ((1, 0), (2, 0), (5, 0), (100, 0), (5, 2 << 20), (100, 2 << 20)):
        e = P.engine_for(w)
        e.set_adjoint(every, ws)
        e.evolve(w.dtau, 5)
        out = e.backward(*obs, want_theta=True)
        e.close()
        if ref is None:
            ref = out
        else:
            assert out[0] == ref[0]
            assert np.array_equal(out[1], ref[1])
            assert out[2] == ref[2]
            assert np.array_equal(out[3], ref[3])


def test_state_unchanged_and_repeatable():
    w = W.tfim_workload("t", 16, 1.0, 0.8, False, 2, 0.05, 0.2, 1e-7, 300)
    e = P.engine_for(w)
    e.set_adjoint(1)
    e.evolve(w.dtau, 4)
    before = e.state()
    o1 = e.backward(w.strings, w.alphas, want_theta=True)
    assert e.state() == before
    o2 = e.backward(w.strings, w.alphas, want_theta=True)
    assert o1[0] == o2[0] and np.array_equal(o1[1], o2[1]) and np.array_equal(o1[3], o2[3])
    # the forward can continue after a reverse sweep
    e.evolve(w.dtau, 1)
    ref = e.state()
    e2 = P.engine_for(w)
    e2.evolve(w.dtau, 5)
    assert e2.state() == ref
    e.close()
    e2.close()


def test_h0_closed_form_derivatives():
    """h = 0 open chain, untruncated: <H> = -J (n-1) tanh(beta J)."""
    n, J, beta = 14, 0.9, 0.6
    w = W.tfim_workload("t", n, J, 0.0, False, 1, 0.05, beta, 0.0, 1 << 20)
    e, st, (L, da, dd, _) = gpu_backward(w, (w.strings, w.alphas), w.n_steps, 3, want_theta=False)
    nzz = n - 1
    t = math.tanh(beta * J)
    sech2 = 1.0 - t * t
    assert abs(L + J * nzz * t) < 1e-12
    assert abs(dd / w.n_steps + J * J * nzz * sech2) < 1e-11
    zz = sum(e.expect([w.strings[k]], [1.0]) for k in range(nzz))
    dJ = -zz - sum(da[k] for k in range(nzz))
    assert abs(dJ + nzz * (t + beta * J * sech2)) < 1e-11
    e.close()


def test_zero_gates_and_errors():
    w = W.tfim_workload("t", 8, 1.0, 1.0, True, 1, 0.05, 0.1, 1e-9, 100)
    e = P.engine_for(w)
    e.set_adjoint(1)
    L, da, dd, dth = e.backward(["IIIIIIII", "XIIIIIII"], [2.0, 1.0], want_theta=True)
    assert L == 2.0 and not da.any() and dd == 0.0
    e.close()
    e = P.engine_for(w)
    e.evolve(w.dtau, 1)
    with pytest.raises(P.ItppError):
        e.backward(w.strings, w.alphas)           # no checkpoints
    e.close()
    e = P.engine_for(w, precision="f32")
    with pytest.raises(P.ItppError):
        e.set_adjoint(1)                          # FP64 only
    e.close()
    e = P.engine_for(w)
    e.set_adjoint(1)
    e.evolve(w.dtau, 1)
    e.evolve(2 * w.dtau, 1)                       # two different dtau
    with pytest.raises(P.ItppError):
        e.backward(w.strings, w.alphas)
    e.close()


def test_autograd_tfim_parameters():
    """d<H>/n with respect to (J, h, beta) through torch autograd: implicit
    part from the reverse sweep, explicit part from the weights."""
    import torch

    from paper_2601_14400_amd import autograd as AG

    n, N = 10, 6
    w = W.tfim_workload("t", n, 1.0, 1.0, True, 1, 0.05, 0.05 * N, 1e-6, 400)
    nzz = n
    Jt = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    ht = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    alphas = torch.cat([-Jt.expand(nzz), -ht.expand(n)])
    eng = P.Engine(n, w.delta, w.K)
    vals = AG.expectations(eng, w.strings, alphas, w.schedule, bt / N, N, w.strings, every=2)
    E = (alphas * vals).sum() / n
    gJ, gh, gb = torch.autograd.grad(E, (Jt, ht, bt))
    # the same through the oracle
    aw = [-1.0] * nzz + [-0.7] * n
    wo = W.Workload(name="o", n=n, strings=w.strings, alphas=aw, schedule=w.schedule, dtau=0.3 / N,
                    n_steps=N, delta=w.delta, K=w.K, observables={}, meta={})
    L, da, dd, _ = AD.gradients(wo, w.strings, aw)
    a, _ = AD.forward_record(n, w.strings, aw, w.schedule, 0.3 / N, N, w.delta, w.K)
    q = [OR.expect(a, [s], [1.0]) for s in w.strings]
    assert abs(float(E.detach()) - L / n) < 1e-13
    rJ = (-sum(q[:nzz]) - sum(da[:nzz])) / n
    rh = (-sum(q[nzz:]) - sum(da[nzz:])) / n
    rb = dd / N / n
    assert abs(float(gJ) - rJ) < 1e-10 * max(1.0, abs(rJ))
    assert abs(float(gh) - rh) < 1e-10 * max(1.0, abs(rh))
    assert abs(float(gb) - rb) < 1e-10 * max(1.0, abs(rb))
    eng.close()


def test_reverse_sweep_from_a_loaded_state():
    """The first forward checkpoint is whatever state the run starts from: a
    state loaded with itpp_import gives the oracle's derivatives from that
    state."""
    w = W.tfim_workload("t", 12, 1.0, 0.9, True, 1, 0.05, 1.0, 1e-9, 2000)
    x, z, c = W.synthetic_state_words(w.n, 600, seed=51, partner=w.strings[w.schedule[0][0]])
    S0 = {}
    for i in range(len(c)):
        s = []
        for j in range(w.n):
            xb = (int(x[i][j >> 6]) >> (j & 63)) & 1
            zb = (int(z[i][j >> 6]) >> (j & 63)) & 1
            s.append("IXZY"[xb | (zb << 1)])
        S0["".join(s)] = float(c[i])
    obs = (w.strings, [a / w.n for a in w.alphas])
    e = P.engine_for(w)
    e.load(S0)
    e.set_adjoint(1)
    st = e.evolve(w.dtau, 2)
    L, da, dd, dth = e.backward(*obs, want_theta=True)
    Lr, dar, ddr, dthr = AD.gradients(w, *obs, n_steps=2, S0=S0)
    assert st["cap_hit"] == 1
    assert len(dth) == len(dthr)
    scale = max(1e-300, max(abs(v) for v in dthr))
    assert max(abs(a - b) for a, b in zip(dth, dthr)) <= TOL * scale
    assert abs(L - Lr) <= 1e-13 * max(1.0, abs(Lr))
    assert max(abs(a - b) for a, b in zip(da, dar)) <= TOL * max(1.0, max(abs(v) for v in dar))
    assert abs(dd - ddr) <= TOL * max(1.0, abs(ddr))
    e.close()
