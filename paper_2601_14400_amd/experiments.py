"""Drivers for the paper's numerical experiments (Sec. III) on the GPU engine.

- ``threshold_sweep``: one chain, coefficient thresholds 2^-k and the
  untruncated case (Sec. III.B, Fig. PP_ITE_12_THERMAL, up to beta = 3;
  Sec. III.C, Fig. PP_ITE_12_GS, up to tau = 20).
- ``fixed_k_size_scan``: the cap fixed, the chain length scanned
  (Sec. III.C, Fig. PP_ITE_fixedK).
- ``k_scan`` and ``min_k_for_error``: energies at several inverse
  temperatures for caps K = 2^9 .. 2^24, and the smallest cap whose relative
  error is at most eps0 (Sec. III.B, Fig. thermal_scalability).

The model is the transverse-field Ising chain of Eq. TFIM,
H = -J sum_i Z_i Z_{i+1} - h sum_i X_i.  One Trotter step applies every ZZ
bond, then every X term (first order, Algorithm 1), or ZZ at half weight, X,
ZZ at half weight (Strang).  beta = n_steps * dtau.

Every run starts from rho = I and returns ITPP results only: energies per
site and retained-string counts along the run.  Exact references (free
fermions) are the caller's; ``min_k_for_error`` takes them as an argument.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Optional, Sequence, Tuple

from ._native import Engine


def tfim_hamiltonian(n: int, J: float, h: float, periodic: bool) -> Tuple[List[str], List[float], int]:
    """Terms of Eq. TFIM: the ZZ bonds (0,1), (1,2), ... (and (n-1, 0) when
    periodic) with weight -J, then X_0 .. X_{n-1} with weight -h.  Returns
    (strings, weights, number of ZZ terms)."""
    if n < 2:
        raise ValueError("the chain needs at least two sites")
    strings: List[str] = []
    alphas: List[float] = []
    bonds = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        bonds.append((n - 1, 0))
    for i, j in bonds:
        s = ["I"] * n
        s[i] = "Z"
        s[j] = "Z"
        strings.append("".join(s))
        alphas.append(-J)
    for i in range(n):
        s = ["I"] * n
        s[i] = "X"
        strings.append("".join(s))
        alphas.append(-h)
    return strings, alphas, len(bonds)


def tfim_schedule(n_zz: int, n_x: int, order: int) -> List[Tuple[int, float]]:
    """One Trotter step as (term, multiplier) pairs."""
    zz = list(range(n_zz))
    xs = list(range(n_zz, n_zz + n_x))
    if order == 1:
        return [(k, 1.0) for k in zz + xs]
    if order == 2:
        return [(k, 0.5) for k in zz] + [(k, 1.0) for k in xs] + [(k, 0.5) for k in zz]
    raise ValueError("order must be 1 or 2")


def n_steps_for(beta: float, dtau: float) -> int:
    """Algorithm 1's ceiling of beta / dtau (a tiny offset absorbs rounding noise)."""
    return max(0, math.ceil(beta / dtau - 1e-9))


def tfim_run(n: int, J: float, h: float, dtau: float, beta: float, delta: float, K: int,
             periodic: bool = False, order: int = 1, record_betas: Optional[Sequence[float]] = None,
             precision: str = "f64") -> Dict:
    """One ITPP run of the TFIM from rho = I to ``beta``.

    The energy per site and the number of retained strings are recorded
    after every Trotter step, or only at the steps of ``record_betas``.
    """
    strings, alphas, n_zz = tfim_hamiltonian(n, J, h, periodic)
    sched = tfim_schedule(n_zz, n, order)
    obs = [a / n for a in alphas]
    steps = n_steps_for(beta, dtau)
    at = None if record_betas is None else sorted({n_steps_for(b, dtau) for b in record_betas})
    e = Engine(n, delta, K, precision=precision)
    try:
        e.set_hamiltonian(strings, alphas)
        e.set_schedule(sched)
        out = {"n": n, "J": J, "h": h, "dtau": dtau, "delta": delta, "K": K, "periodic": periodic,
               "order": order, "beta": [], "energy_per_site": [], "n_terms": [], "term_updates": 0.0,
               "cap_hit": 0}
        t0 = time.perf_counter()
        done = 0
        targets = list(range(1, steps + 1)) if at is None else [s for s in at if 0 < s <= steps]
        for s in targets:
            st = e.evolve(dtau, s - done)
            done = s
            out["term_updates"] += st["term_updates"]
            out["cap_hit"] |= st["cap_hit"]
            out["beta"].append(s * dtau)
            out["energy_per_site"].append(e.expect(strings, obs))
            out["n_terms"].append(st["n_terms"])
        if done < steps:
            st = e.evolve(dtau, steps - done)
            out["term_updates"] += st["term_updates"]
            out["cap_hit"] |= st["cap_hit"]
        out["seconds"] = time.perf_counter() - t0
        out["max_terms"] = max(out["n_terms"]) if out["n_terms"] else 1
        return out
    finally:
        e.close()


def threshold_sweep(n: int = 12, J: float = 1.0, h: float = 0.5, dtau: float = 0.04, beta: float = 3.0,
                    ks: Sequence[int] = tuple(range(5, 20)), untruncated: bool = True, K: int = 1 << 24,
                    periodic: bool = False, order: int = 1,
                    record_betas: Optional[Sequence[float]] = None) -> List[Dict]:
    """Runs at thresholds 2^-k (and 0, the untruncated case), one chain."""
    deltas = ([0.0] if untruncated else []) + [2.0 ** (-k) for k in ks]
    return [tfim_run(n, J, h, dtau, beta, d, K, periodic, order, record_betas) for d in deltas]


def fixed_k_size_scan(ns: Sequence[int] = tuple(range(12, 52, 2)), K: int = 2704156, J: float = 1.0,
                      h: float = 0.5, dtau: float = 0.04, beta: float = 20.0, delta: float = 0.0,
                      periodic: bool = False, order: int = 1) -> List[Dict]:
    """The cap fixed (by default the untruncated support of 12 sites), the
    chain length scanned; energies at the final beta."""
    return [tfim_run(n, J, h, dtau, beta, delta, K, periodic, order, record_betas=[beta]) for n in ns]


def k_scan(n: int, betas: Sequence[float], Ks: Sequence[int] = tuple(1 << k for k in range(9, 25)),
           J: float = 1.0, h: float = 0.5, dtau: float = 0.04, delta: float = 0.0, periodic: bool = False,
           order: int = 1) -> List[Dict]:
    """For every cap K, one run to max(betas) recording the energy at each beta."""
    return [tfim_run(n, J, h, dtau, max(betas), delta, K, periodic, order, record_betas=betas) for K in Ks]


def min_k_for_error(runs: Sequence[Dict], beta: float, reference: float, eps0: float = 1e-2) -> Optional[int]:
    """Smallest cap K among ``runs`` (from ``k_scan``) whose energy at ``beta``
    is within relative error eps0 of ``reference``; None if none is."""
    best = None
    for r in runs:
        for b, E in zip(r["beta"], r["energy_per_site"]):
            if abs(b - beta) < 1e-9 and abs(E - reference) <= eps0 * abs(reference):
                best = r["K"] if best is None else min(best, r["K"])
    return best
