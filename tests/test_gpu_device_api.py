"""Device-pointer entry points (itpp_expect_device, itpp_export_device) with
torch tensors: same results as the host-array entry points, and the
observable agrees with the oracle's."""
import numpy as np
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


def as_dict(x, z, c):
    return {(tuple(int(v) for v in x[i]), tuple(int(v) for v in z[i])): float(c[i]) for i in range(len(c))}


@pytest.mark.parametrize("builder,steps", [(lambda: W.config2(K=3000), 2), (lambda: W.config3(K=2000), 1)])
def test_device_variants(builder, steps):
    import torch

    w = builder()
    e = P.engine_for(w)
    e.evolve(w.dtau, steps)
    xd, zd, cd = e.export_device()
    x, z, c = e.export()
    assert xd.is_cuda and xd.dtype == torch.int64 and xd.shape == (len(c), e.W)
    dev = as_dict(xd.cpu().numpy().view(np.uint64), zd.cpu().numpy().view(np.uint64), cd.cpu().numpy())
    assert dev == as_dict(x, z, c)

    o = c_oracle.run_workload(w, n_steps=steps)
    ref = o.state()
    for name, (strings, coefs) in w.observables.items():
        xo, zo = P.strings_to_words(strings, w.n)
        xt = torch.from_numpy(xo.view(np.int64)).cuda()
        zt = torch.from_numpy(zo.view(np.int64)).cuda()
        ct = torch.tensor(coefs, dtype=torch.float64, device="cuda")
        v = e.expect_device(xt, zt, ct)
        assert v.is_cuda and v.shape == ()
        vd = float(v.item())
        assert vd == e.expect(strings, coefs), name
        assert vd == pytest.approx(OR.expect(ref, strings, coefs), rel=1e-12, abs=1e-14), name
    empty = torch.empty((0, e.W), dtype=torch.int64, device="cuda")
    assert float(e.expect_device(empty, empty, torch.empty((0,), dtype=torch.float64, device="cuda")).item()) == 0.0
    with pytest.raises(ValueError):
        e.expect_device(xt.float(), zt, ct)
    e.close()
