"""Dictionary-of-strings ITPP oracle (test infrastructure only).

Plain, slow and meant to be checked by eye against the paper
(arXiv 2601.14400, "Pauli Propagation for Imaginary-Time Evolution"):

* The state is a dict ``{pauli_string: coefficient}`` with
  ``rho = 2^-n sum_P a_P P``; it starts as ``{"I"*n: 1.0}`` because
  propagating the identity instead of ``I/2^n`` gives the same normalised
  state (Sec. II.C, the paragraph after Eq. ThermalTrotter).
* One elementary gate ``V_Q = exp(-(theta/2) Q)`` maps every string by
  Eq. (ITPP_PropRules), derived in Appendix A:
  anticommuting ``P`` stays ``P``; commuting ``P`` becomes
  ``cosh(theta) P - sinh(theta) Q P``.  Here ``theta = alpha_k * m * dtau``
  for term ``alpha_k Q_k`` and schedule multiplier ``m`` (Algorithm 1 uses
  ``m = 1``: the gate is ``exp(-(dtau/2) h_k Q_k)``).
* After each gate the contributions are accumulated in the Pauli basis, the
  result is truncated (keep ``|c| > delta`` as in the coefficient-threshold
  rule of Sec. II.B; if more than ``K`` strings remain keep the identity and
  the ``K-1`` largest ``|c|`` as in the K-truncation paragraph of Sec. II.C)
  and then divided by the identity coefficient, which is the trace
  normalisation of Algorithm 1 done after every elementary step as Sec. II.C
  prescribes.

Optional Pauli-weight cutoff (``max_weight``, the second truncation rule of
Sec. II.B): a string of weight (number of non-identity letters) above the
cutoff is dropped.  Reading: it is applied with the coefficient threshold
after every gate, before the cap selection, so the K kept strings are the
largest of those within the cutoff; the identity (weight 0) always passes.

Readings fixed here where the paper leaves a choice open:
* ``Q P`` multiplies with ``Q`` on the left, using ``XY = iZ``, ``YZ = iX``,
  ``ZX = iY``; for commuting strings ``Q P = sign * R`` with ``sign = +-1``.
* truncation uses the value before normalisation (Algorithm 1 writes
  ``T(rho') / Tr T(rho')``);
* equal magnitudes at the cap are broken by the smaller canonical key
  ``(X, Z)``, where ``X = sum_j x_j 2^j`` and ``Z = sum_j z_j 2^j`` are the
  integers of the x- and z-bits (``X``: letters X, Y; ``Z``: letters Z, Y),
  compared as the pair ``(X, Z)``;
* a gate whose string is the identity is skipped (after normalisation it
  would only rescale every coefficient by the same factor);
* ``cosh`` and ``sinh`` are evaluated once per gate with the C library
  (Python's ``math``), and each new coefficient is ``ch*c`` (or ``c`` for an
  anticommuting string) plus at most one branch term ``-sh*sign*c'``.

Single-precision form (``precision="f32"``): coefficients are stored and
propagated as IEEE binary32; ``ch`` and ``sh`` are the double values rounded
to binary32; every product and sum of Eq. (ITPP_PropRules) is rounded to
binary32; the threshold compares the binary32 magnitude (exactly widened) with
the double ``delta``; normalisation divides in double and rounds the quotient
to binary32; observables sum in double.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

# Single-qubit products a*b = i^k * r as (k mod 4, r): Pauli algebra.
_MUL: Dict[Tuple[str, str], Tuple[int, str]] = {}
for _a in "IXYZ":
    _MUL[("I", _a)] = (0, _a)
    _MUL[(_a, "I")] = (0, _a)
for _a in "XYZ":
    _MUL[(_a, _a)] = (0, "I")
for _a, _b, _c in (("X", "Y", "Z"), ("Y", "Z", "X"), ("Z", "X", "Y")):
    _MUL[(_a, _b)] = (1, _c)   # a b =  i c
    _MUL[(_b, _a)] = (3, _c)   # b a = -i c


class OracleError(RuntimeError):
    pass


def identity(n: int) -> str:
    return "I" * n


def pauli_product(P: str, Q: str) -> Tuple[int, str]:
    """``P Q = i^k R``; returns ``(k mod 4, R)``."""
    if len(P) != len(Q):
        raise ValueError("length mismatch")
    k = 0
    out = []
    for a, b in zip(P, Q):
        ph, r = _MUL[(a, b)]
        k += ph
        out.append(r)
    return k % 4, "".join(out)


def anticommuting_sites(P: str, Q: str) -> int:
    """Number of qubits where both letters are non-identity and differ."""
    return sum(1 for a, b in zip(P, Q) if a != "I" and b != "I" and a != b)


def commutes(P: str, Q: str) -> bool:
    return anticommuting_sites(P, Q) % 2 == 0


def canonical_key(P: str) -> Tuple[int, int]:
    """``(X, Z)`` integers of the string's x- and z-bits (qubit j -> bit j)."""
    X = 0
    Z = 0
    for j, a in enumerate(P):
        if a in "XY":
            X |= 1 << j
        if a in "ZY":
            Z |= 1 << j
    return X, Z


def gate_contributions(P: str, c: float, Q: str, ch: float, sh: float) -> List[Tuple[str, float]]:
    """Image of ``c P`` under ``V_Q^dagger (.) V_Q`` (Eq. ITPP_PropRules)."""
    if not commutes(P, Q):
        return [(P, c)]
    k, R = pauli_product(Q, P)          # Q P = i^k R
    if k % 2:
        raise OracleError("commuting strings gave an imaginary phase")
    sign = 1.0 if k == 0 else -1.0
    return [(P, ch * c), (R, -sh * sign * c)]


def apply_gate(S: Dict[str, float], Q: str, ch: float, sh: float) -> Dict[str, float]:
    """Propagate every term and accumulate in the Pauli basis (rho')."""
    out: Dict[str, float] = {}
    for P, c in S.items():
        for R, v in gate_contributions(P, c, Q, ch, sh):
            out[R] = out.get(R, 0.0) + v
    return out


def apply_gate_f32(S: Dict[str, np.float32], Q: str, ch: float, sh: float) -> Dict[str, np.float32]:
    """Single-precision twin of ``apply_gate`` (binary32 products and sums)."""
    ch32 = np.float32(ch)
    sh32 = np.float32(sh)
    out: Dict[str, np.float32] = {}
    for P, c in S.items():
        if not commutes(P, Q):
            contribs = [(P, c)]
        else:
            k, R = pauli_product(Q, P)
            if k % 2:
                raise OracleError("commuting strings gave an imaginary phase")
            t = np.float32(sh32 * c)
            contribs = [(P, np.float32(ch32 * c)), (R, -t if k == 0 else t)]
        for R, v in contribs:
            out[R] = np.float32(out[R] + v) if R in out else np.float32(v)
    return out


def pauli_weight(P: str) -> int:
    """Number of non-identity letters (Sec. II.B)."""
    return sum(1 for a in P if a != "I")


def truncate(S: Dict[str, float], delta: float, K: int, max_weight: Optional[int] = None) -> Dict[str, float]:
    """Keep ``|c| > delta`` (and, with a cutoff, Pauli weight <= max_weight);
    if more than ``K`` remain keep the identity and the ``K-1`` other strings
    of largest ``|c|`` (ties: smaller (X, Z))."""
    kept = {P: c for P, c in S.items()
            if abs(float(c)) > delta and (max_weight is None or pauli_weight(P) <= max_weight)}
    if len(kept) <= K:
        return kept
    n = len(next(iter(kept)))
    ident = identity(n)
    if ident not in kept:
        raise OracleError("identity coefficient was truncated")
    others = [(P, c) for P, c in kept.items() if P != ident]
    others.sort(key=lambda t: (-abs(float(t[1])), canonical_key(t[0])))
    out = {ident: kept[ident]}
    for P, c in others[: K - 1]:
        out[P] = c
    return out


def normalize(S: Dict[str, float], n: int) -> Tuple[Dict[str, float], float]:
    """Divide every coefficient by the identity coefficient (unit trace)."""
    cI = S.get(identity(n))
    if cI is None or not math.isfinite(cI) or cI <= 0.0:
        raise OracleError(f"bad identity coefficient {cI!r}")
    return {P: c / cI for P, c in S.items()}, cI


def normalize_f32(S: Dict[str, np.float32], n: int) -> Tuple[Dict[str, np.float32], float]:
    """Divide in double by the identity coefficient, round to binary32."""
    cI = S.get(identity(n))
    if cI is None or not math.isfinite(float(cI)) or float(cI) <= 0.0:
        raise OracleError(f"bad identity coefficient {cI!r}")
    d = float(cI)
    return {P: np.float32(float(c) / d) for P, c in S.items()}, d


def gate_angle(alpha: float, mult: float, dtau: float) -> float:
    return alpha * mult * dtau


def evolve(n: int, strings: Sequence[str], alphas: Sequence[float],
           schedule: Sequence[Tuple[int, float]], dtau: float, n_steps: int,
           delta: float, K: int, S0: Optional[Dict[str, float]] = None,
           on_gate: Optional[Callable[[int, Dict[str, float], float], None]] = None,
           precision: str = "f64", max_weight: Optional[int] = None) -> Tuple[Dict[str, float], Dict[str, float]]:
    """Algorithm 1 with per-gate truncation and normalisation.

    Returns ``(S, stats)`` with ``stats['term_updates']`` = sum over gates of
    the number of strings entering the gate.
    """
    f32 = precision == "f32"
    S = dict(S0) if S0 is not None else {identity(n): (np.float32(1.0) if f32 else 1.0)}
    if f32:
        S = {P: np.float32(c) for P, c in S.items()}
    ident = identity(n)
    updates = 0
    g = 0
    for _step in range(n_steps):
        for k, m in schedule:
            Q = strings[k]
            if len(Q) != n:
                raise ValueError("term length differs from n")
            if Q == ident:
                continue
            theta = gate_angle(alphas[k], m, dtau)
            ch = math.cosh(theta)
            sh = math.sinh(theta)
            updates += len(S)
            if f32:
                Sp = apply_gate_f32(S, Q, ch, sh)
                St = truncate(Sp, delta, K, max_weight)
                S, cI = normalize_f32(St, n)
            else:
                Sp = apply_gate(S, Q, ch, sh)
                St = truncate(Sp, delta, K, max_weight)
                S, cI = normalize(St, n)
            if on_gate is not None:
                on_gate(g, S, cI)
            g += 1
    return S, {"term_updates": float(updates), "n_gates": float(g)}


def expect(S: Dict[str, float], strings: Iterable[str], coefs: Iterable[float]) -> float:
    """<O> = sum_j o_j a_{P_j} for O = sum_j o_j P_j (absent strings count 0)."""
    return math.fsum(o * float(S.get(P, 0.0)) for P, o in zip(strings, coefs))


def run_workload(w, **kw):
    """Convenience wrapper for an ``itpp_workloads.Workload``."""
    kw.setdefault("precision", w.precision)
    return evolve(w.n, w.strings, w.alphas, w.schedule, w.dtau, w.n_steps, w.delta, w.K, **kw)
