"""The seeded synthetic-state generator (CPU): distinct strings, the identity
first with coefficient 1, the stated magnitude set, partner pairs, and the
canonical word layout shared with the oracle (qubit j -> bit j; X, Y set x;
Z, Y set z)."""
import numpy as np
import pytest

import itpp_workloads as W
from oracle import itpp as OR


def test_string_words_match_the_oracle_canonical_key():
    rng = np.random.default_rng(0)
    for n in (1, 7, 64, 65, 100, 128):
        for _ in range(50):
            s = "".join(rng.choice(list("IXYZ"), size=n))
            x, z = W.string_words(s)
            X, Z = OR.canonical_key(s)
            assert sum(int(v) << (64 * q) for q, v in enumerate(x)) == X
            assert sum(int(v) << (64 * q) for q, v in enumerate(z)) == Z


@pytest.mark.parametrize("n,count", [(12, 2000), (64, 20000), (100, 5000)])
def test_synthetic_state(n, count):
    Q = "ZZ" + "I" * (n - 2)
    x, z, c = W.synthetic_state_words(n, count, seed=4, partner=Q)
    Wd = (n + 63) // 64
    assert x.shape == (count, Wd) and z.shape == (count, Wd) and c.shape == (count,)
    rows = {(tuple(map(int, x[i])), tuple(map(int, z[i]))) for i in range(count)}
    assert len(rows) == count
    assert not np.any(x[0]) and not np.any(z[0]) and c[0] == 1.0
    assert all(np.any(x[i]) or np.any(z[i]) for i in range(1, count))
    top = n - 64 * (Wd - 1)
    if top < 64:
        assert int(x[:, -1].max()) < (1 << top) and int(z[:, -1].max()) < (1 << top)
    mags = set(np.abs(c[1:]).tolist())
    assert mags <= {2.0 ** (-0.25 * k) for k in range(1, 77)}
    assert (c[1:] > 0).any() and (c[1:] < 0).any()
    qx, qz = W.string_words(Q)
    pairs = sum(1 for i in range(1, count)
                if (tuple(map(int, x[i] ^ qx)), tuple(map(int, z[i] ^ qz))) in rows)
    assert pairs > 0.2 * count
    x2, z2, c2 = W.synthetic_state_words(n, count, seed=4, partner=Q)
    assert np.array_equal(x, x2) and np.array_equal(z, z2) and np.array_equal(c, c2)
