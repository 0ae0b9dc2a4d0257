"""The plain C++ dictionary oracle agrees bit for bit with the Python oracle
and is pinned on its own to a closed form at a size the Python oracle does
not reach quickly.  CPU only."""
import math
import os

import numpy as np
import pytest

import itpp_workloads as W
from oracle import c_oracle, itpp


@pytest.fixture(scope="module", autouse=True)
def _built():
    c_oracle.build(force=False)


def test_config1_prefix_bitexact():
    w = W.config1()
    S, st = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 8, w.delta, w.K)
    o = c_oracle.run_workload(w, n_steps=8)
    assert o.state() == S
    assert o.term_updates() == st["term_updates"]


@pytest.mark.parametrize("seed", [0, 7])
def test_random_capped_bitexact(seed):
    w = W.random_workload("r", 12, 14, seed, 0.15, 5, 1e-10, 150)
    S, _ = itpp.run_workload(w)
    o = c_oracle.run_workload(w)
    assert len(S) == 150
    assert o.state() == S


def test_config2_shape_capped_bitexact():
    w = W.config2(K=512)
    S, _ = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, 1, w.delta, w.K)
    o = c_oracle.run_workload(w, n_steps=1)
    assert o.state() == S


def test_h0_open_closed_form_n16():
    n, J, beta = 16, 1.0, 0.5
    w = W.tfim_workload("t", n, J, 0.0, False, 1, 0.05, beta, 0.0, 1 << 40)
    o = c_oracle.run_workload(w)
    S = o.state()
    t = math.tanh(beta * J)
    assert len(S) == 2 ** (n - 1)
    for P, c in S.items():
        z = np.array([1 if a == "Z" else 0 for a in P])
        b = np.cumsum(z) % 2
        assert abs(c - t ** int(b[:-1].sum())) < 1e-14


def test_export_is_canonical_order():
    w = W.config1()
    o = c_oracle.run_workload(w, n_steps=3)
    strs, coef = o.export()
    keys = [itpp.canonical_key(s) for s in strs]
    assert keys == sorted(keys)


def _max_rel(a, b):
    scale = max(1e-300, max(abs(float(v)) for v in b))
    return max(abs(float(x) - float(y)) for x, y in zip(a, b)) / scale


@pytest.mark.parametrize("builder,steps,obs", [
    (lambda: W.tfim_workload("t", 10, 1.0, 0.9, True, 1, 0.05, 0.2, 1e-6, 300), 4, None),
    (lambda: W.tfim_workload("t", 12, 0.8, 1.1, False, 2, 0.05, 0.15, 1e-7, 200), 3, "x0"),
    (lambda: W.random_two_flip_workload("r", 12, 14, 1, 0.1, 2, 1e-9, 150), 2, None),
])
def test_reverse_sweep_matches_python_adjoint(builder, steps, obs):
    """The C++ reverse sweep (frozen support) against the pinned Python
    reverse-mode oracle: binding caps, thresholds, Y terms, Strang order."""
    from oracle import adjoint as AD

    w = builder()
    if obs is None:
        os_, oc = w.strings, [a / w.n for a in w.alphas]
    else:
        os_, oc = ["X" + "I" * (w.n - 1), w.strings[0]], [1.0, -0.5]
    Lr, dar, ddr, dthr = AD.gradients(w, os_, oc, n_steps=steps)
    o = c_oracle.COracle(w.n)
    L, da, dd, dth = o.gradients(w, os_, oc, n_steps=steps)
    assert len(dth) == len(dthr)
    assert abs(L - Lr) <= 1e-14 * max(1.0, abs(Lr))
    assert _max_rel(dth, dthr) <= 1e-13
    assert _max_rel(da, dar) <= 1e-13
    assert abs(dd - ddr) <= 1e-13 * max(1.0, abs(ddr))
    # the forward part leaves the oracle's final state
    S, _ = itpp.evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, steps, w.delta, w.K)
    assert o.state() == S


def test_reverse_sweep_h0_closed_form_n16():
    """h = 0 open chain, untruncated, 2^15 strings: <H> = -J (n-1) tanh(beta J),
    so d<H>/dbeta = -J^2 (n-1) sech^2(beta J) and the J derivative follows."""
    n, J, beta = 16, 0.9, 0.6
    w = W.tfim_workload("t", n, J, 0.0, False, 1, 0.05, beta, 0.0, 1 << 40)
    o = c_oracle.COracle(n)
    L, da, dd, _ = o.gradients(w, w.strings, w.alphas)
    nzz = n - 1
    t = math.tanh(beta * J)
    sech2 = 1.0 - t * t
    assert abs(L + J * nzz * t) < 1e-12
    assert abs(dd / w.n_steps + J * J * nzz * sech2) < 1e-11
    S = o.state()
    zz = sum(S.get(w.strings[k], 0.0) for k in range(nzz))
    dJ = -zz - sum(da[k] for k in range(nzz))
    assert abs(dJ + nzz * (t + beta * J * sech2)) < 1e-11


def test_reverse_sweep_from_loaded_state_matches_python():
    from oracle import adjoint as AD

    w = W.tfim_workload("t", 12, 1.0, 0.9, True, 1, 0.05, 1.0, 1e-9, 400)
    x, z, c = W.synthetic_state_words(w.n, 300, seed=51, partner=w.strings[w.schedule[0][0]])
    o = c_oracle.COracle(w.n)
    o.load_words(x, z, c)
    S0 = o.state()
    obs = (w.strings, [a / w.n for a in w.alphas])
    Lr, dar, ddr, dthr = AD.gradients(w, *obs, n_steps=2, S0=S0)
    L, da, dd, dth = o.gradients(w, *obs, n_steps=2)
    assert abs(L - Lr) <= 1e-14 * max(1.0, abs(Lr))
    assert _max_rel(dth, dthr) <= 1e-13
    assert abs(dd - ddr) <= 1e-13 * max(1.0, abs(ddr))


@pytest.mark.parametrize("n", [12, 64, 100])
def test_word_import_export_roundtrip(n):
    x, z, c = W.synthetic_state_words(n, 500, seed=5)
    o = c_oracle.COracle(n)
    o.load_words(x, z, c)
    S = o.state()
    assert len(S) == len(c)
    x2, z2, c2 = o.export_words(x.shape[1])
    strs, coef = o.export()
    assert np.array_equal(coef, c2)
    for i in range(len(c2)):
        assert itpp.canonical_key(strs[i]) == (sum(int(x2[i, q]) << (64 * q) for q in range(x.shape[1])),
                                               sum(int(z2[i, q]) << (64 * q) for q in range(x.shape[1])))
    # the same multiset as the input
    order = np.lexsort(tuple(z[:, q] for q in range(x.shape[1])) + tuple(x[:, q] for q in range(x.shape[1])))
    assert np.array_equal(x[order], x2) and np.array_equal(z[order], z2) and np.array_equal(c[order], c2)


def test_threshold_readings_reduce_to_algorithm_1_without_truncation():
    """The oracle's alternative threshold readings (once per Trotter step;
    every contribution before the sums) equal Algorithm 1 when the threshold
    truncates nothing, and differ from it when it does."""
    c_oracle.build(force=False)
    w = W.tfim_workload("t", 8, 1.0, 0.5, False, 1, 0.04, 0.4, 1e-300, 10 ** 9)
    ref = c_oracle.run_workload(w).state()
    for reading in (1, 2):
        o = c_oracle.COracle(w.n)
        o.set_reading(reading)
        o.evolve(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, w.delta, w.K)
        assert o.state() == ref
    states = []
    for reading in (0, 1, 2):
        o = c_oracle.COracle(w.n)
        o.set_reading(reading)
        o.evolve(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, 2.0 ** -7, w.K)
        states.append(o.state())
    assert states[0] != states[1] and states[0] != states[2]


@pytest.mark.parametrize("n,periodic,order", [(6, False, 1), (6, True, 2), (8, False, 1)])
def test_threshold_readings_match_their_definitions(n, periodic, order):
    """Both alternative readings against compositions of the Python oracle's
    steps, bit for bit, with a threshold that binds:
    1 = every gate only propagates and normalises, and the normalised state
        is thresholded once after the last gate of each Trotter step;
    2 = every contribution of Eq. ITPP_PropRules is thresholded before the
        sums, then the gate truncates and normalises as in Algorithm 1;
    3 = as 1, on the coefficients before the step's normalisation (the
        normalised ones times the product of the step's identity
        coefficients)."""
    c_oracle.build(force=False)
    w = W.tfim_workload("t", n, 1.0, 0.5, periodic, order, 0.04, 0.4, 2.0 ** -7, 10 ** 9)
    ident = "I" * n
    gates = [(w.strings[k], math.cosh(w.alphas[k] * m * w.dtau), math.sinh(w.alphas[k] * m * w.dtau))
             for k, m in w.schedule]

    S1 = {ident: 1.0}
    for _ in range(w.n_steps):
        for Q, ch, sh in gates:
            S1, _ = itpp.normalize(itpp.apply_gate(S1, Q, ch, sh), n)
        S1 = {P: c for P, c in S1.items() if P == ident or abs(c) > w.delta}

    S2 = {ident: 1.0}
    for _ in range(w.n_steps):
        for Q, ch, sh in gates:
            acc = {}
            for P, c in S2.items():
                for R, v in itpp.gate_contributions(P, c, Q, ch, sh):
                    if abs(v) > w.delta:
                        acc[R] = acc.get(R, 0.0) + v
            S2, _ = itpp.normalize(itpp.truncate(acc, w.delta, w.K), n)

    S3 = {ident: 1.0}
    for _ in range(w.n_steps):
        growth = 1.0
        for Q, ch, sh in gates:
            S3, cI = itpp.normalize(itpp.apply_gate(S3, Q, ch, sh), n)
            growth *= cI
        S3 = {P: c for P, c in S3.items() if P == ident or abs(c) * growth > w.delta}

    alg1, _ = itpp.run_workload(w)
    assert S3 != S1
    for reading, ref in ((1, S1), (2, S2), (3, S3)):
        o = c_oracle.COracle(w.n)
        o.set_reading(reading)
        o.evolve(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, w.delta, w.K)
        assert o.state() == ref, reading
        assert ref != alg1


def test_sanitized_build_runs_clean(tmp_path):
    """The C++ oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (g++, host code only) runs every entry point on a small capped chain
    without a report (oracle/c/sanitize_main.cpp)."""
    import shutil
    import subprocess

    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    here = os.path.dirname(c_oracle.SRC)
    exe = str(tmp_path / "oracle_san")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           c_oracle.SRC, os.path.join(here, "sanitize_main.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


@pytest.mark.parametrize("precision,K", [("f64", 10 ** 6), ("f64", 120), ("f32", 200)])
def test_twin_on_xxz_chain(precision, K):
    """The C++ twin equals the Python oracle bit for bit on an XXZ chain (YY
    terms flip four key bits), untruncated and with the cap binding."""
    c_oracle.build(force=False)
    n = 7
    bonds = [(i, i + 1) for i in range(n - 1)]
    strings, alphas = [], []
    for letter, a in (("X", 0.8), ("Y", 0.8), ("Z", -0.5)):
        for i, j in bonds:
            s = ["I"] * n
            s[i] = s[j] = letter
            strings.append("".join(s))
            alphas.append(a)
    sched = [(k, 1.0) for k in range(len(strings))]
    w = W.Workload("xxz", n, strings, alphas, sched, 0.05, 6, 1e-10, K, precision=precision)
    S, _ = itpp.run_workload(w)
    assert c_oracle.run_workload(w).state() == S
    assert any("Y" in P for P in S)
