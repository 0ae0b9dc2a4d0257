"""Pins of the CPU oracle against facts that do not come from the oracle:
dense Pauli matrices, matrix exponentials, exact diagonalisation, closed forms
of commuting special cases, the free-fermion solution, combinatorial counts
and brute-force enumeration.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import itpp_workloads as W
from oracle import dense, freefermion as ff, itpp

LETTERS = "IXYZ"


def all_strings(n):
    return ["".join(p) for p in itertools.product(LETTERS, repeat=n)]


# ---------------------------------------------------------------- algebra ---

def test_single_qubit_table_matches_matrices():
    for a in LETTERS:
        for b in LETTERS:
            k, r = itpp.pauli_product(a, b)
            lhs = dense.pauli_matrix(a) @ dense.pauli_matrix(b)
            rhs = (1j ** k) * dense.pauli_matrix(r)
            assert np.allclose(lhs, rhs, atol=0), (a, b)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_string_product_and_commutation_exhaustive(n):
    mats = {P: dense.pauli_matrix(P) for P in all_strings(n)}
    for P, MP in mats.items():
        for Q, MQ in mats.items():
            k, R = itpp.pauli_product(P, Q)
            assert np.array_equal(MP @ MQ, (1j ** k) * mats[R]), (P, Q)
            comm = np.array_equal(MP @ MQ, MQ @ MP)
            assert itpp.commutes(P, Q) == comm, (P, Q)


@pytest.mark.parametrize("n", [1, 2])
def test_gate_rule_matches_matrix_exponential_exhaustive(n):
    """Eq. ITPP_PropRules vs V^dagger P V with V = expm(-(theta/2) Q)."""
    rng = np.random.default_rng(5)
    for Q in all_strings(n):
        if Q == "I" * n:
            continue
        theta = float(rng.uniform(-1.5, 1.5))
        V = dense.gate_matrix(Q, theta)
        for P in all_strings(n):
            lhs = V.conj().T @ dense.pauli_matrix(P) @ V
            rhs = np.zeros_like(lhs)
            for R, v in itpp.gate_contributions(P, 1.0, Q, math.cosh(theta), math.sinh(theta)):
                rhs = rhs + v * dense.pauli_matrix(R)
            assert np.allclose(lhs, rhs, atol=1e-13), (P, Q)


def test_gate_rule_random_n3():
    rng = np.random.default_rng(11)
    strs = all_strings(3)
    for _ in range(300):
        P = strs[int(rng.integers(len(strs)))]
        Q = strs[int(rng.integers(1, len(strs)))]
        theta = float(rng.uniform(-2, 2))
        V = dense.gate_matrix(Q, theta)
        lhs = V.conj().T @ dense.pauli_matrix(P) @ V
        rhs = sum(v * dense.pauli_matrix(R) for R, v in
                  itpp.gate_contributions(P, 1.0, Q, math.cosh(theta), math.sinh(theta)))
        assert np.allclose(lhs, rhs, atol=1e-13)


# ------------------------------------------------ untruncated = Trotterized ---

def _coef_err(S, A):
    keys = set(S) | set(A)
    return max(abs(S.get(k, 0.0) - A.get(k, 0.0)) for k in keys)


@pytest.mark.parametrize("n,periodic,order", [(4, False, 1), (4, True, 1), (5, False, 2),
                                              (5, True, 2), (6, False, 1)])
def test_untruncated_equals_trotterized_dense(n, periodic, order):
    """Without truncation ITPP reproduces Eq. ThermalTrotter exactly."""
    w = W.tfim_workload("t", n, 1.0, 0.7, periodic, order, 0.05, 0.6, 0.0, 1 << 40)
    S, _ = itpp.run_workload(w)
    rho = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    A = dense.pauli_coefficients(rho, tol=1e-14)
    assert _coef_err(S, A) < 1e-12
    assert S["I" * n] == 1.0


@pytest.mark.parametrize("Lx,Ly,periodic,order", [(2, 2, False, 1), (3, 2, False, 2), (3, 3, True, 1)])
def test_untruncated_2d_lattice_equals_trotterized_dense(Lx, Ly, periodic, order):
    """A two-dimensional TFIM (square lattice) is propagated like any other
    Hamiltonian: without truncation it reproduces Eq. ThermalTrotter."""
    w = W.tfim_2d_workload("t", Lx, Ly, 1.0, 0.7, periodic, order, 0.05, 0.4, 0.0, 1 << 40)
    n = Lx * Ly
    assert len(w.strings) == (Lx * Ly * 2 if periodic else (Lx - 1) * Ly + Lx * (Ly - 1)) + n
    S, _ = itpp.run_workload(w)
    rho = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    A = dense.pauli_coefficients(rho, tol=1e-14)
    assert _coef_err(S, A) < 1e-12


def xxz_chain(n, jxy, jz, periodic):
    """XX, YY and ZZ on every bond (YY flips four key bits: the GPU path
    rejects it, the oracle takes any string)."""
    bonds = [(i, i + 1) for i in range(n - 1)] + ([(n - 1, 0)] if periodic and n > 2 else [])
    strings, alphas = [], []
    for letter, a in (("X", jxy), ("Y", jxy), ("Z", jz)):
        for i, j in bonds:
            s = ["I"] * n
            s[i] = s[j] = letter
            strings.append("".join(s))
            alphas.append(a)
    return strings, alphas, len(bonds)


@pytest.mark.parametrize("n,periodic,order,jz", [(4, False, 1, 0.6), (5, True, 2, 1.0), (6, False, 2, -0.4)])
def test_untruncated_xxz_chain_equals_trotterized_dense(n, periodic, order, jz):
    """XXZ and Heisenberg chains: without truncation the oracle reproduces
    Eq. ThermalTrotter for terms with Y letters on two sites; the Strang
    split halves the XX and YY groups around the ZZ group."""
    strings, alphas, nb = xxz_chain(n, 1.0, jz, periodic)
    xx, yy, zz = range(0, nb), range(nb, 2 * nb), range(2 * nb, 3 * nb)
    if order == 1:
        sched = [(k, 1.0) for k in range(3 * nb)]
    else:
        sched = ([(k, 0.5) for k in xx] + [(k, 0.5) for k in yy] + [(k, 1.0) for k in zz]
                 + [(k, 0.5) for k in yy] + [(k, 0.5) for k in xx])
    dtau, steps = 0.05, 8
    S, _ = itpp.evolve(n, strings, alphas, sched, dtau, steps, 0.0, 1 << 40)
    rho = dense.trotter_thermal(strings, alphas, sched, dtau, steps)
    A = dense.pauli_coefficients(rho, tol=1e-14)
    assert _coef_err(S, A) < 1e-12
    assert any("Y" in k for k in S)
    # the Trotter product commutes with the global flips (each term does)
    for P in S:
        assert sum(ch in "XY" for ch in P) % 2 == 0 and sum(ch in "ZY" for ch in P) % 2 == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_untruncated_random_hamiltonian_with_y_terms(seed):
    w = W.random_workload("r", 4, 7, seed, 0.1, 4, 0.0, 1 << 40, max_weight=3, local=False)
    assert any("Y" in s for s in w.strings)
    S, _ = itpp.run_workload(w)
    rho = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    A = dense.pauli_coefficients(rho, tol=1e-14)
    assert _coef_err(S, A) < 1e-12


def test_config1_observables_vs_dense_and_ed():
    """n=8 periodic: exact match with the dense Trotterized state; <H>/n within
    the O(dtau^2) Trotter error of exact diagonalisation."""
    w = W.config1()
    S, _ = itpp.run_workload(w)
    rho_t = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    H = dense.hamiltonian(w.strings, w.alphas)
    rho_e = dense.exact_thermal(H, w.meta["beta"])
    for name, (strs, coefs) in w.observables.items():
        O = sum(c * dense.pauli_matrix(s) for s, c in zip(strs, coefs))
        v = itpp.expect(S, strs, coefs)
        assert abs(v - dense.expectation(rho_t, O)) < 1e-12, name
    e_itpp = itpp.expect(S, *w.observables["energy_per_site"])
    e_ed = dense.expectation(rho_e, H) / w.n
    assert abs(e_itpp - e_ed) < 2e-3
    assert abs(ff.thermal_energy(8, 1.0, 1.0, 1.0, True) / 8 - e_ed) < 1e-12


# ------------------------------------------------------------ invariants ---

@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_support_size_is_central_binomial(n):
    """Saturated untruncated TFIM support has C(2n, n) strings; the paper's
    2,704,156 untruncated strings at N=12 equal C(24, 12)."""
    w = W.tfim_workload("t", n, 1.0, 0.5, False, 1, 0.04, 0.04 * 3 * n, 0.0, 1 << 40)
    S, _ = itpp.run_workload(w)
    assert len(S) == math.comb(2 * n, n)
    assert math.comb(24, 12) == 2704156


def test_invariants_every_gate():
    """a_I = 1 after every gate; even number of Y (real symmetric rho); even
    number of Z/Y letters (the TFIM commutes with prod X)."""
    w = W.tfim_workload("t", 6, 1.0, 0.9, True, 2, 0.05, 0.5, 1e-9, 300)
    seen = []

    def check(g, S, cI):
        assert S["I" * 6] == 1.0
        for P in S:
            assert P.count("Y") % 2 == 0
            assert (P.count("Z") + P.count("Y")) % 2 == 0
        assert len(S) <= 300
        seen.append(len(S))

    itpp.run_workload(w, on_gate=check)
    assert max(seen) == 300


def test_translation_invariance_periodic():
    n = 6
    w = W.tfim_workload("t", n, 1.0, 0.8, True, 1, 0.05, 0.5, 0.0, 1 << 40)
    S, _ = itpp.run_workload(w)
    # per-gate ordering breaks exact symmetry only through the Trotter error;
    # compare a symmetric quantity: <Z_i Z_{i+1}> is the same for all bonds
    # in the exact Trotterized state only up to O(dtau); check the dense twin.
    rho = dense.trotter_thermal(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps)
    for i in range(n):
        Pz = W.two_site(n, i, (i + 1) % n, "Z", "Z")
        assert abs(S.get(Pz, 0.0) - dense.expectation(rho, dense.pauli_matrix(Pz))) < 1e-12


# ----------------------------------------------------------- closed forms ---

def _bond_count_open(P):
    z = [1 if a in "ZY" else 0 for a in P]
    b = np.cumsum(z) % 2
    assert b[-1] == 0
    return int(b[:-1].sum())


def test_h0_open_closed_form():
    """h = 0: commuting ZZ terms, the Trotter product is exact and
    a_S = tanh(beta J)^{|S|} for the product of bond subset S."""
    n, J, beta = 10, 0.8, 1.2
    w = W.tfim_workload("t", n, J, 0.0, False, 1, 0.1, beta, 0.0, 1 << 40)
    S, _ = itpp.run_workload(w)
    t = math.tanh(beta * J)
    assert len(S) == 2 ** (n - 1)
    for P, c in S.items():
        assert set(P) <= {"I", "Z"}
        k = _bond_count_open(P)
        assert abs(c - t ** k) <= 1e-14 * max(1.0, t ** k) + 1e-15


def test_h0_periodic_closed_form():
    n, J, beta = 8, 1.0, 0.7
    w = W.tfim_workload("t", n, J, 0.0, True, 1, 0.07, beta, 0.0, 1 << 40)
    S, _ = itpp.run_workload(w)
    t = math.tanh(beta * J)
    assert len(S) == 2 ** (n - 1)
    for P, c in S.items():
        z = [1 if a in "ZY" else 0 for a in P]
        b = np.cumsum(z) % 2          # bond i = (i, i+1 mod n)
        k = int(b.sum())
        exact = (t ** k + t ** (n - k)) / (1 + t ** n)
        assert abs(c - exact) < 1e-14


def test_j0_closed_form():
    n, h, beta = 9, 1.3, 0.9
    w = W.tfim_workload("t", n, 0.0, h, False, 1, 0.1, beta, 0.0, 1 << 40)
    S, _ = itpp.run_workload(w)
    t = math.tanh(beta * h)
    assert len(S) == 2 ** n
    for P, c in S.items():
        k = P.count("X")
        assert abs(c - t ** k) < 1e-14


# -------------------------------------------------------------- truncation ---

def test_topk_rule_bruteforce():
    """The cap keeps exactly the subset fixed by the ordering (|c| desc,
    (X,Z) asc) plus the identity; checked over every subset of a tiny state
    with deliberate ties."""
    rng = np.random.default_rng(3)
    n = 3
    strs = all_strings(n)[1:]
    vals = [0.5, -0.5, 0.25, 0.25, -0.125, 0.5, 0.0625, -0.25, 0.125, 0.03125]
    picks = rng.choice(len(strs), size=len(vals), replace=False)
    S = {"III": 1.0}
    for v, i in zip(vals, picks):
        S[strs[int(i)]] = v
    keys = list(S)
    for K in range(1, len(S) + 1):
        got = set(itpp.truncate(S, 0.0, K))
        valid = []
        for T in itertools.combinations(keys, min(K, len(S))):
            T = set(T)
            if "III" not in T:
                continue
            ok = True
            for u in T - {"III"}:
                for v in set(keys) - T:
                    au, av = abs(S[u]), abs(S[v])
                    if not (au > av or (au == av and itpp.canonical_key(u) < itpp.canonical_key(v))):
                        ok = False
            if ok:
                valid.append(T)
        assert len(valid) == 1 and valid[0] == got, K


def test_threshold_is_strict():
    S = {"II": 1.0, "XI": 1e-6, "IX": 2e-6, "ZZ": -1e-6}
    assert set(itpp.truncate(S, 1e-6, 10)) == {"II", "IX"}


def test_canonical_key():
    assert itpp.canonical_key("XIZY") == (0b1001, 0b1100)


# ------------------------------------------------------------- free fermions ---

@pytest.mark.parametrize("periodic", [False, True])
def test_freefermion_energy_matches_ed(periodic):
    for n in (3, 4, 5, 7):
        for J, h in ((1.0, 0.5), (1.0, 1.4), (0.6, 1.0)):
            s, a, _ = W.tfim_terms(n, J, h, periodic)
            H = dense.hamiltonian(s, a)
            for beta in (0.2, 1.0, 3.0):
                E = dense.expectation(dense.exact_thermal(H, beta), H)
                assert abs(ff.thermal_energy(n, J, h, beta, periodic) - E) < 1e-10


def test_freefermion_zz_matches_ed():
    n, J, h, beta = 6, 1.0, 0.8, 1.3
    s, a, _ = W.tfim_terms(n, J, h, False)
    rho = dense.exact_thermal(dense.hamiltonian(s, a), beta)
    for r in range(1, n):
        O = dense.pauli_matrix(W.two_site(n, 0, r, "Z", "Z"))
        assert abs(ff.zz_correlation(n, J, h, beta, r) - dense.expectation(rho, O)) < 1e-10


def test_pfaffian_small():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(4, 4))
    A = A - A.T
    exp4 = A[0, 1] * A[2, 3] - A[0, 2] * A[1, 3] + A[0, 3] * A[1, 2]
    assert abs(ff.pfaffian(A) - exp4) < 1e-12
    B = rng.normal(size=(6, 6))
    B = B - B.T
    assert abs(ff.pfaffian(B) ** 2 - np.linalg.det(B)) < 1e-9


def test_ground_energy_open_matches_ed():
    n = 8
    s, a, _ = W.tfim_terms(n, 1.0, 0.5, False)
    H = dense.hamiltonian(s, a)
    assert abs(np.linalg.eigvalsh(H)[0] - ff.ground_energy(n, 1.0, 0.5, False)) < 1e-10
