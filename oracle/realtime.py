"""Real-time Pauli propagation rule (test infrastructure only).

Sec. II.B: under U_Q(theta) = exp(-i theta Q / 2), a string P that commutes
with Q is unchanged and one that anticommutes becomes
cos(theta) P + i sin(theta) Q P.  For anticommuting Hermitian strings
Q P = i^k R with k odd, so i Q P = i^(k+1) R is real: -R for k = 1, +R for
k = 3.  The identity commutes with every Q, so its coefficient stays 1 and
trace normalisation is not needed.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

from .itpp import OracleError, commutes, identity, pauli_product, truncate


def gate_contributions_real(P: str, c: float, Q: str, cs: float, sn: float) -> List[Tuple[str, float]]:
    """Image of ``c P`` under ``U_Q(theta)^dagger (.) U_Q(theta)``."""
    if commutes(P, Q):
        return [(P, c)]
    k, R = pauli_product(Q, P)  # Q P = i^k R
    if k % 2 == 0:
        raise OracleError("anticommuting strings gave a real phase")
    s = -1.0 if k == 1 else 1.0
    return [(P, cs * c), (R, s * sn * c)]


def apply_gate_real(S: Dict[str, float], Q: str, cs: float, sn: float) -> Dict[str, float]:
    out: Dict[str, float] = {}
    for P, c in S.items():
        for R, v in gate_contributions_real(P, c, Q, cs, sn):
            out[R] = out.get(R, 0.0) + v
    return out


def evolve_real(S0: Dict[str, float], strings: Sequence[str], alphas: Sequence[float],
                schedule: Sequence[Tuple[int, float]], dt: float, n_steps: int, delta: float,
                K: int, max_weight=None) -> Tuple[Dict[str, float], float]:
    """First-order (or any scheduled) Trotter steps of real-time propagation
    from S0 with angle theta = alpha_k * m * dt per gate, truncated after
    every gate like the imaginary-time oracle (threshold, optional Pauli
    weight cutoff, cap: both truncation rules of Sec. II.B are stated for
    real-time propagation).  Returns (S, term updates)."""
    S = dict(S0)
    n = len(next(iter(S)))
    updates = 0.0
    for _ in range(n_steps):
        for k, m in schedule:
            Q = strings[k]
            if Q == identity(n):
                continue
            th = alphas[k] * m * dt
            updates += len(S)
            S = truncate(apply_gate_real(S, Q, math.cos(th), math.sin(th)), delta, K, max_weight)
    return S, updates
