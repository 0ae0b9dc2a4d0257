"""Seeded synthetic inputs for imaginary-time Pauli propagation (ITPP).

This module only *describes* workloads: Hamiltonian terms as Pauli strings
with real weights, the gate order of one Trotter step, step counts,
observables and the seeded draws that pick model parameters.  It holds none
of the method's arithmetic (no products of Pauli strings, no cosh/sinh, no
truncation), so both the CPU oracle and the GPU library can take their inputs
from here without sharing any computation.

Conventions
-----------
* A Pauli string on ``n`` qubits is a Python ``str`` of length ``n`` over the
  letters ``I X Y Z``; character ``j`` is qubit ``j``.
* The transverse-field Ising chain of the paper's Eq. (TFIM) is
  ``H = -J sum_i Z_i Z_{i+1} - h sum_i X_i``; periodic chains add the bond
  ``(n-1, 0)``.  Terms are listed as all ZZ bonds ``(0,1), (1,2), ...`` then the
  periodic bond if present, then ``X_0 .. X_{n-1}``.
* A schedule is one Trotter step: a list of ``(term_index, multiplier)``.  The
  gate for entry ``(k, m)`` has angle ``theta = alpha_k * m * dtau``.
  First order (Algorithm 1): every term once with ``m = 1`` (ZZ layer then X
  layer).  Second order (the Strang splitting of Sec. II.C): ZZ layer with
  ``m = 1/2``, X layer with ``m = 1``, ZZ layer with ``m = 1/2``; the half
  layers of consecutive steps are not merged.
* The number of steps for a target inverse temperature ``beta`` is
  ``ceil(beta/dtau - 1e-9)`` (Algorithm 1 takes the ceiling; the small offset
  absorbs floating-point noise in ``beta/dtau``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

PAULI_LETTERS = "IXYZ"


def single_site(n: int, site: int, letter: str) -> str:
    s = ["I"] * n
    s[site] = letter
    return "".join(s)


def two_site(n: int, i: int, j: int, li: str, lj: str) -> str:
    s = ["I"] * n
    s[i] = li
    s[j] = lj
    return "".join(s)


def tfim_terms(n: int, J: float, h: float, periodic: bool) -> Tuple[List[str], List[float], int]:
    """Terms of H = -J sum Z_i Z_{i+1} - h sum X_i.

    Returns ``(strings, alphas, n_zz)`` where the first ``n_zz`` terms are the
    ZZ bonds and the rest are the ``n`` single-site X terms.
    """
    if n < 2:
        raise ValueError("a chain needs at least two qubits")
    strings: List[str] = []
    alphas: List[float] = []
    for i in range(n - 1):
        strings.append(two_site(n, i, i + 1, "Z", "Z"))
        alphas.append(-float(J))
    if periodic and n > 2:
        strings.append(two_site(n, n - 1, 0, "Z", "Z"))
        alphas.append(-float(J))
    n_zz = len(strings)
    for i in range(n):
        strings.append(single_site(n, i, "X"))
        alphas.append(-float(h))
    return strings, alphas, n_zz


def tfim_schedule(n_zz: int, n_x: int, order: int) -> List[Tuple[int, float]]:
    """Gate list of one Trotter step for the term layout of ``tfim_terms``."""
    zz = list(range(n_zz))
    xx = list(range(n_zz, n_zz + n_x))
    if order == 1:
        return [(k, 1.0) for k in zz] + [(k, 1.0) for k in xx]
    if order == 2:
        return [(k, 0.5) for k in zz] + [(k, 1.0) for k in xx] + [(k, 0.5) for k in zz]
    raise ValueError("order must be 1 or 2")


def n_steps_for(beta: float, dtau: float) -> int:
    return int(math.ceil(beta / dtau - 1e-9))


def draw_uniform(seed: int, lo: float, hi: float, size: Optional[int] = None):
    rng = np.random.default_rng(seed)
    v = rng.uniform(lo, hi, size=size)
    return float(v) if size is None else v


@dataclass
class Workload:
    """One ITPP run: Hamiltonian terms, one Trotter step's gates, step size,
    number of steps, truncation threshold ``delta`` (keep ``|c| > delta``) and
    term cap ``K``."""

    name: str
    n: int
    strings: List[str]
    alphas: List[float]
    schedule: List[Tuple[int, float]]
    dtau: float
    n_steps: int
    delta: float
    K: int
    precision: str = "f64"
    observables: Dict[str, Tuple[List[str], List[float]]] = field(default_factory=dict)
    meta: Dict[str, object] = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return len(self.schedule) * self.n_steps

    @property
    def words(self) -> int:
        return (self.n + 63) // 64


def tfim_observables(n: int, J: float, h: float, periodic: bool, zz_ranges: Sequence[int] = (1,)) -> Dict[str, Tuple[List[str], List[float]]]:
    """<H>/n, <X_0>, <Z_0 Z_r> for the requested r, and M_x = sum X_i."""
    strings, alphas, _ = tfim_terms(n, J, h, periodic)
    obs: Dict[str, Tuple[List[str], List[float]]] = {}
    obs["energy_per_site"] = (strings, [a / n for a in alphas])
    obs["X0"] = ([single_site(n, 0, "X")], [1.0])
    for r in zz_ranges:
        if 0 < r < n:
            obs[f"Z0Z{r}"] = ([two_site(n, 0, r, "Z", "Z")], [1.0])
    obs["Mx"] = ([single_site(n, i, "X") for i in range(n)], [1.0] * n)
    return obs


def tfim_workload(name: str, n: int, J: float, h: float, periodic: bool, order: int,
                  dtau: float, beta: float, delta: float, K: int, precision: str = "f64",
                  zz_ranges: Sequence[int] = (1,)) -> Workload:
    strings, alphas, n_zz = tfim_terms(n, J, h, periodic)
    sched = tfim_schedule(n_zz, n, order)
    return Workload(name=name, n=n, strings=strings, alphas=alphas, schedule=sched,
                    dtau=dtau, n_steps=n_steps_for(beta, dtau), delta=delta, K=K,
                    precision=precision,
                    observables=tfim_observables(n, J, h, periodic, zz_ranges),
                    meta=dict(model="tfim", J=J, h=h, periodic=periodic, order=order, beta=beta))


# ---------------------------------------------------------------------------
# The five benchmark workloads (synthetic TFIM instances; no dataset exists).
# ---------------------------------------------------------------------------

def config1() -> Workload:
    """n=8 periodic TFIM, J=h=1, first order, dtau=0.05, beta 0->1 (20 steps),
    threshold 1e-14, cap 2^20 (never reached)."""
    return tfim_workload("tfim_n8_periodic_untruncated", 8, 1.0, 1.0, True, 1, 0.05, 1.0,
                         1e-14, 1 << 20, zz_ranges=(1, 2, 3, 4))


def config2_h(seed: int = 0) -> float:
    return draw_uniform(seed, 0.5, 1.5)


def config2(K: int = 1 << 24, beta: float = 2.0, seed: int = 0) -> Workload:
    """n=64 open TFIM, J=1, h ~ U[0.5, 1.5] (seeded), Strang, dtau=0.02,
    beta 0->2 (100 steps), threshold 1e-6, cap 2^24."""
    h = config2_h(seed)
    w = tfim_workload("tfim_n64_open_strang", 64, 1.0, h, False, 2, 0.02, beta, 1e-6, K,
                      zz_ranges=tuple(range(1, 9)))
    w.meta["seed"] = seed
    return w


def config3(K: int = 1 << 27, beta: float = 1.0, precision: str = "f32") -> Workload:
    """n=128 periodic TFIM (two words), J=h=1, dtau=0.01, beta 0->1,
    threshold 1e-7, cap 2^27."""
    return tfim_workload("tfim_n128_periodic", 128, 1.0, 1.0, True, 1, 0.01, beta, 1e-7, K,
                         precision=precision)


def config4_instances(seed: int = 1, count: int = 64, K: int = 1 << 20) -> List[Workload]:
    """64 periodic TFIM instances: n uniform in {16,24,...,128}, h ~ U[0.25,2],
    beta ~ U[0.5,2], J=1, first order, dtau=0.02, threshold 1e-6, cap 2^20."""
    rng = np.random.default_rng(seed)
    sizes = np.arange(16, 129, 8)
    ns = rng.choice(sizes, size=count)
    hs = rng.uniform(0.25, 2.0, size=count)
    betas = rng.uniform(0.5, 2.0, size=count)
    out = []
    for i in range(count):
        w = tfim_workload(f"batch_{i}", int(ns[i]), 1.0, float(hs[i]), True, 1, 0.02,
                          float(betas[i]), 1e-6, K)
        out.append(w)
    return out


def config5(K: int = 1 << 24) -> Workload:
    """n=64 periodic TFIM, J=h=1, first order, dtau=0.02, beta=1.5 (75 steps),
    threshold 1e-6, cap 2^24."""
    return tfim_workload("tfim_n64_periodic_adjoint", 64, 1.0, 1.0, True, 1, 0.02, 1.5, 1e-6, K)


def paper_validation(n: int = 10, tau: float = 20.0) -> Workload:
    """Sec. III validation run: open chain, J=1, h=0.5, dtau=0.04, no truncation."""
    return tfim_workload(f"paper_validation_n{n}", n, 1.0, 0.5, False, 1, 0.04, tau, 0.0, 1 << 62)


# ---------------------------------------------------------------------------
# Random Hamiltonians with arbitrary Pauli letters (exercise Y phases).
# ---------------------------------------------------------------------------

def random_hamiltonian(n: int, n_terms: int, seed: int, max_weight: int = 3,
                       local: bool = True) -> Tuple[List[str], List[float]]:
    """Random real-weighted Pauli terms.  ``local`` draws supports from a window
    of ``max_weight`` consecutive qubits (periodic), otherwise anywhere."""
    rng = np.random.default_rng(seed)
    strings: List[str] = []
    alphas: List[float] = []
    seen = set()
    while len(strings) < n_terms:
        w = int(rng.integers(1, max_weight + 1))
        if local:
            start = int(rng.integers(0, n))
            window = [(start + k) % n for k in range(max_weight)]
            sites = sorted(rng.choice(window, size=min(w, len(window)), replace=False).tolist())
        else:
            sites = sorted(rng.choice(n, size=w, replace=False).tolist())
        s = ["I"] * n
        for q in sites:
            s[q] = "XYZ"[int(rng.integers(0, 3))]
        key = "".join(s)
        if key in seen or key == "I" * n:
            continue
        seen.add(key)
        strings.append(key)
        alphas.append(float(rng.uniform(-1.0, 1.0)))
    return strings, alphas


def random_workload(name: str, n: int, n_terms: int, seed: int, dtau: float, n_steps: int,
                    delta: float, K: int, max_weight: int = 3, local: bool = True) -> Workload:
    strings, alphas = random_hamiltonian(n, n_terms, seed, max_weight, local)
    sched = [(k, 1.0) for k in range(n_terms)]
    obs = {"energy": (list(strings), list(alphas))}
    return Workload(name=name, n=n, strings=strings, alphas=alphas, schedule=sched, dtau=dtau,
                    n_steps=n_steps, delta=delta, K=K, observables=obs,
                    meta=dict(model="random", seed=seed))


def random_pauli_strings(n: int, count: int, seed: int, density: float = 0.5) -> List[str]:
    """Uniformly random strings (each site non-identity with probability ``density``)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = []
        for _q in range(n):
            if rng.random() < density:
                s.append("XYZ"[int(rng.integers(0, 3))])
            else:
                s.append("I")
        out.append("".join(s))
    return out


def random_two_flip_hamiltonian(n: int, n_terms: int, seed: int, span: int = 4) -> Tuple[List[str], List[float]]:
    """Random terms that flip at most two x/z bits: single-site X, Y, Z and
    two-site products of X and Z letters within ``span`` neighbouring qubits
    (periodic)."""
    rng = np.random.default_rng(seed)
    strings: List[str] = []
    alphas: List[float] = []
    seen = set()
    while len(strings) < n_terms:
        s = ["I"] * n
        i = int(rng.integers(0, n))
        if rng.random() < 0.4:
            s[i] = "XYZ"[int(rng.integers(0, 3))]
        else:
            j = (i + int(rng.integers(1, max(2, min(span, n))))) % n
            if j == i:
                continue
            s[i] = "XZ"[int(rng.integers(0, 2))]
            s[j] = "XZ"[int(rng.integers(0, 2))]
        key = "".join(s)
        if key in seen:
            continue
        seen.add(key)
        strings.append(key)
        alphas.append(float(rng.uniform(-1.0, 1.0)))
    return strings, alphas


def random_two_flip_workload(name: str, n: int, n_terms: int, seed: int, dtau: float, n_steps: int,
                             delta: float, K: int) -> Workload:
    strings, alphas = random_two_flip_hamiltonian(n, n_terms, seed)
    sched = [(k, 1.0) for k in range(n_terms)]
    return Workload(name=name, n=n, strings=strings, alphas=alphas, schedule=sched, dtau=dtau,
                    n_steps=n_steps, delta=delta, K=K, observables={"energy": (list(strings), list(alphas))},
                    meta=dict(model="random_two_flip", seed=seed))


# ---------------------------------------------------------------------------
# Synthetic states (inputs for loading a state directly, e.g. at full size).
# ---------------------------------------------------------------------------

def string_words(P: str) -> Tuple[np.ndarray, np.ndarray]:
    """Canonical x/z words of one string (qubit j -> bit j of word j // 64;
    X and Y set the x bit, Z and Y the z bit)."""
    n = len(P)
    W = (n + 63) // 64
    x = np.zeros(W, dtype=np.uint64)
    z = np.zeros(W, dtype=np.uint64)
    for j, a in enumerate(P):
        bit = np.uint64(1) << np.uint64(j & 63)
        if a in "XY":
            x[j >> 6] |= bit
        if a in "ZY":
            z[j >> 6] |= bit
    return x, z


def synthetic_state_words(n: int, count: int, seed: int, partner: Optional[str] = None,
                          partner_frac: float = 0.3, levels: int = 76,
                          step: float = 0.25) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """A seeded state of ``count`` distinct strings on ``n`` qubits as canonical
    words ``x, z`` (shape ``(count, W)``) and coefficients.

    * Row 0 is the identity with coefficient 1.
    * The other strings are uniformly random; about ``partner_frac`` of them
      also appear flipped by ``partner``'s bits (so a gate with that string
      meets partner pairs).
    * Magnitudes are ``2**(-k*step)`` for integer ``k`` uniform in
      ``[1, levels]`` with random signs: a few dozen distinct values, so a cap
      cuts through large groups of equal magnitudes.
    """
    if count < 1:
        raise ValueError("count must be >= 1")
    rng = np.random.default_rng(seed)
    W = (n + 63) // 64
    masks = np.array([np.uint64((1 << min(64, n - 64 * q)) - 1) if n - 64 * q < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
                      for q in range(W)], dtype=np.uint64)
    m = count - 1
    # a margin over the expected count; the surplus is cut after removing repeats
    base = int(1.05 * m / (1.0 + partner_frac)) + 64 if partner is not None else m + 64
    xs = rng.integers(0, 2**63, size=(base, W), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(base, W), dtype=np.uint64)
    zs = rng.integers(0, 2**63, size=(base, W), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(base, W), dtype=np.uint64)
    xs &= masks
    zs &= masks
    if partner is not None:
        qx, qz = string_words(partner)
        pick = rng.random(base) < partner_frac
        xs = np.concatenate([xs, xs[pick] ^ qx])
        zs = np.concatenate([zs, zs[pick] ^ qz])
    # distinct, non-identity, in random order, exactly m of them
    rows = np.concatenate([xs, zs], axis=1)
    rows = rows[np.any(rows != 0, axis=1)]
    order = np.lexsort(tuple(rows[:, i] for i in reversed(range(rows.shape[1]))))  # stable
    srt = rows[order]
    repeat = np.concatenate([[False], np.all(srt[1:] == srt[:-1], axis=1)])
    rows = rows[np.sort(order[~repeat])]
    if rows.shape[0] < m:
        raise ValueError("not enough distinct strings; lower partner_frac or raise n")
    rows = rows[rng.permutation(rows.shape[0])[:m]]
    x = np.concatenate([np.zeros((1, W), dtype=np.uint64), rows[:, :W]])
    z = np.concatenate([np.zeros((1, W), dtype=np.uint64), rows[:, W:]])
    k = rng.integers(1, levels + 1, size=m)
    sign = np.where(rng.random(m) < 0.5, -1.0, 1.0)
    coef = np.concatenate([[1.0], sign * np.exp2(-step * k.astype(np.float64))])
    return x, z, coef


# ---------------------------------------------------------------------------
# Two-dimensional transverse-field Ising model (a general lattice Hamiltonian).
# ---------------------------------------------------------------------------

def tfim_2d_terms(Lx: int, Ly: int, J: float, h: float, periodic: bool = False) -> Tuple[List[str], List[float], int]:
    """H = -J sum_<ij> Z_i Z_j - h sum_i X_i on an Lx x Ly square lattice,
    site (x, y) -> qubit x + Lx * y; horizontal bonds, then vertical bonds,
    then the X terms.  Returns (strings, weights, number of ZZ terms)."""
    n = Lx * Ly
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            if x + 1 < Lx or (periodic and Lx > 2):
                bonds.append((x + Lx * y, (x + 1) % Lx + Lx * y))
    for y in range(Ly):
        for x in range(Lx):
            if y + 1 < Ly or (periodic and Ly > 2):
                bonds.append((x + Lx * y, x + Lx * ((y + 1) % Ly)))
    strings = [two_site(n, min(i, j), max(i, j), "Z", "Z") for i, j in bonds]
    alphas = [-J] * len(bonds)
    strings += [single_site(n, i, "X") for i in range(n)]
    alphas += [-h] * n
    return strings, alphas, len(bonds)


def tfim_2d_workload(name: str, Lx: int, Ly: int, J: float, h: float, periodic: bool, order: int,
                     dtau: float, beta: float, delta: float, K: int, precision: str = "f64") -> Workload:
    strings, alphas, n_zz = tfim_2d_terms(Lx, Ly, J, h, periodic)
    n = Lx * Ly
    sched = tfim_schedule(n_zz, n, order)
    obs = {"energy_per_site": (list(strings), [a / n for a in alphas]),
           "X0": ([single_site(n, 0, "X")], [1.0])}
    return Workload(name=name, n=n, strings=strings, alphas=alphas, schedule=sched, dtau=dtau,
                    n_steps=n_steps_for(beta, dtau), delta=delta, K=K, precision=precision, observables=obs,
                    meta=dict(model="tfim_2d", Lx=Lx, Ly=Ly, J=J, h=h, periodic=periodic, order=order, beta=beta))
