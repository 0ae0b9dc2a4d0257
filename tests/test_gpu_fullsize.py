"""The benchmark workload at its full size: n = 64 open TFIM, Strang splitting,
dtau = 0.02, threshold 1e-6, cap K = 2^24, in the launch configuration the
benchmark times (default options, event timing on).

The oracle follows the run bit for bit through its first 130 elementary gates
(63 ZZ half-steps and 67 X gates; the threshold truncates on every gate and
the state reaches ~2.9e5 strings).  Past that the oracle cannot keep up, so
the run is carried on until the cap binds and the state is checked against
properties that hold at any size:
- exactly K strings, all distinct, the identity among them with coefficient 1 (unit trace);
- every other |c| above the threshold;
- the global spin flip prod_i X_i commutes with H, so every string has an even number of Z and Y letters;
- rho is real, so every string has an even number of Y letters.
The gate rule maps strings with both parities even to strings with both
parities even, and truncation only removes strings."""
import numpy as np
import pytest

import itpp_workloads as W
from oracle import c_oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2601_14400_amd")

PREFIX_GATES = 130


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c_oracle.build(force=False)


def full_engine(w):
    e = P.engine_for(w)
    e.set_timing(True)
    return e


def test_benchmark_workload_prefix_bitexact():
    w = W.config2()
    assert (w.n, w.K, w.delta, w.dtau) == (64, 1 << 24, 1e-6, 0.02)
    e = full_engine(w)
    st = e.evolve_gates(w.dtau, PREFIX_GATES)
    S = e.state()
    o = c_oracle.COracle(w.n)
    o.evolve(w.strings, w.alphas, w.schedule[:PREFIX_GATES], w.dtau, 1, w.delta, w.K)
    ref = o.state()
    assert len(ref) > 200000
    assert S == ref
    assert st["term_updates"] == o.term_updates()
    e.close()


def test_benchmark_workload_capped_state_properties():
    w = W.config2()
    e = full_engine(w)
    st = None
    for _ in range(40):
        st = e.evolve(w.dtau, 1)
        if st["n_terms"] == w.K:
            break
    assert st["n_terms"] == w.K and st["cap_hit"] == 1
    # two more steps with the cap binding on every gate
    st = e.evolve(w.dtau, 2)
    assert st["n_terms"] == w.K
    x, z, c = e.export()
    assert x.shape == (w.K, 1) and z.shape == (w.K, 1) and c.shape == (w.K,)
    x, z = x[:, 0], z[:, 0]  # n = 64: one x word and one z word per string
    # distinct strings: sort the (x, z) pairs and compare neighbours
    order = np.lexsort((z, x))
    xs, zs = x[order], z[order]
    assert not np.any((xs[1:] == xs[:-1]) & (zs[1:] == zs[:-1]))
    ident = (x == 0) & (z == 0)
    assert int(ident.sum()) == 1
    assert c[ident][0] == 1.0
    assert np.all(np.abs(c[~ident]) > w.delta)
    assert np.all(np.isfinite(c))
    # symmetry sectors
    assert np.all(np.bitwise_count(z) % 2 == 0)
    assert np.all(np.bitwise_count(x & z) % 2 == 0)
    e.close()
