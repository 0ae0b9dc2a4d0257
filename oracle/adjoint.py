"""Reverse-mode derivatives of an ITPP observable (test infrastructure only).

The quantity is ``L = sum_j o_j a[P_j]`` for the state ``a`` left by
Algorithm 1 of arXiv 2601.14400 (every gate followed by truncation and the
division by the identity coefficient, Sec. II.C).  Truncation is not
differentiable, so the derivative is the one of the map in which every gate
keeps exactly the strings the forward run kept ("frozen support"): a change
of the parameters changes the retained coefficients, never the retained set.

One gate ``g`` with string ``Q`` and angle ``theta`` maps the normalised input
``a`` to ``u = G(theta) a`` by Eq. (ITPP_PropRules), keeps the set ``S_g``
(``b = u`` on ``S_g``) and normalises ``a' = b / b_I``.  Given
``lam' = dL/da'`` the reverse sweep is, in plain calculus:

* normalisation: ``dL/db_P = lam'_P / b_I`` and, for the identity only,
  ``- (sum_R lam'_R a'_R) / b_I`` (the derivative of ``b_P / b_I`` with respect
  to ``b_I``);
* support: that vector restricted to ``S_g`` (zero elsewhere), ``lam_u``;
* gate: a commuting ``P`` with ``Q P = sigma R`` sent ``ch a_P`` to ``P`` and
  ``-sigma sh a_P`` to ``R``, so ``lam_P = ch lam_u[P] - sigma sh lam_u[R]``;
  an anticommuting ``P`` passed through, ``lam_P = lam_u[P]``;
* angle: ``d ch/d theta = sh`` and ``d sh/d theta = ch`` give
  ``dL/dtheta_g = sum_{P commuting} a_P (sh lam_u[P] - sigma ch lam_u[R])``.

With ``theta_g = alpha_k m_g dtau`` (Algorithm 1 with schedule multipliers)
the chain rule gives ``dL/dalpha_k = sum_{g of term k} m_g dtau dL/dtheta_g``
and ``dL/ddtau = sum_g alpha_k m_g dL/dtheta_g``.  Every long sum is taken
with ``math.fsum``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

from . import itpp


@dataclass
class GateRecord:
    term: int
    mult: float
    theta: float
    a_in: Dict[str, float]     # normalised input of the gate
    kept: frozenset            # strings kept after truncation
    b_I: float                 # identity coefficient before normalisation


def forward_record(n: int, strings: Sequence[str], alphas: Sequence[float],
                   schedule: Sequence[Tuple[int, float]], dtau: float, n_steps: int,
                   delta: float, K: int,
                   S0: Optional[Dict[str, float]] = None) -> Tuple[Dict[str, float], List[GateRecord]]:
    """Algorithm 1 exactly as ``itpp.evolve``, keeping what the reverse sweep
    needs for every gate; from ``S0`` (normalised, a_I = 1) instead of
    rho = I when given."""
    ident = itpp.identity(n)
    S = {ident: 1.0} if S0 is None else dict(S0)
    recs: List[GateRecord] = []
    for _ in range(n_steps):
        for k, m in schedule:
            Q = strings[k]
            if Q == ident:
                continue
            theta = itpp.gate_angle(alphas[k], m, dtau)
            u = itpp.apply_gate(S, Q, math.cosh(theta), math.sinh(theta))
            b = itpp.truncate(u, delta, K)
            a_out, bI = itpp.normalize(b, n)
            recs.append(GateRecord(k, m, theta, S, frozenset(b), bI))
            S = a_out
    return S, recs


def forward_frozen(n: int, strings: Sequence[str], recs: Sequence[GateRecord],
                   alphas: Sequence[float], dtau: float) -> Dict[str, float]:
    """The same gate sequence with new parameters, each gate keeping the
    recorded support (used for finite differences)."""
    ident = itpp.identity(n)
    S = {ident: 1.0}
    for r in recs:
        theta = itpp.gate_angle(alphas[r.term], r.mult, dtau)
        u = itpp.apply_gate(S, strings[r.term], math.cosh(theta), math.sinh(theta))
        b = {P: u.get(P, 0.0) for P in r.kept}
        S, _ = itpp.normalize(b, n)
    return S


def backward(n: int, strings: Sequence[str], recs: Sequence[GateRecord], a_final: Dict[str, float],
             obs_strings: Sequence[str], obs_coefs: Sequence[float]
             ) -> Tuple[float, List[float], Dict[str, float]]:
    """Returns ``(L, dL/dtheta per gate, dL/d a_initial)``."""
    ident = itpp.identity(n)
    lam: Dict[str, float] = {}
    for P, o in zip(obs_strings, obs_coefs):
        if P in a_final:
            lam[P] = lam.get(P, 0.0) + o
    L = itpp.expect(a_final, obs_strings, obs_coefs)
    a_out = a_final
    s = math.fsum(v * a_out[P] for P, v in lam.items())
    dtheta = [0.0] * len(recs)
    for g in range(len(recs) - 1, -1, -1):
        r = recs[g]
        Q = strings[r.term]
        ch, sh = math.cosh(r.theta), math.sinh(r.theta)
        lam_u = {P: lam.get(P, 0.0) / r.b_I for P in r.kept}
        lam_u[ident] = lam_u.get(ident, 0.0) - s / r.b_I
        lam_in: Dict[str, float] = {}
        terms = []
        for P, aP in r.a_in.items():
            lp = lam_u.get(P, 0.0)
            if not itpp.commutes(P, Q):
                lam_in[P] = lp
                continue
            k, R = itpp.pauli_product(Q, P)
            sigma = 1.0 if k == 0 else -1.0
            lr = lam_u.get(R, 0.0)
            lam_in[P] = ch * lp - sigma * sh * lr
            terms.append(aP * (sh * lp - sigma * ch * lr))
        dtheta[g] = math.fsum(terms)
        s = math.fsum(lam_in[P] * aP for P, aP in r.a_in.items())
        lam = lam_in
    return L, dtheta, lam


def parameter_gradients(strings: Sequence[str], alphas: Sequence[float], recs: Sequence[GateRecord],
                        dtheta: Sequence[float], dtau: float) -> Tuple[List[float], float]:
    """Chain rule from per-gate angles to (alpha_k, dtau)."""
    per_term: List[List[float]] = [[] for _ in strings]
    per_dtau: List[float] = []
    for r, d in zip(recs, dtheta):
        per_term[r.term].append(r.mult * dtau * d)
        per_dtau.append(alphas[r.term] * r.mult * d)
    return [math.fsum(t) for t in per_term], math.fsum(per_dtau)


def gradients(w, obs_strings: Sequence[str], obs_coefs: Sequence[float],
              n_steps: Optional[int] = None, S0: Optional[Dict[str, float]] = None):
    """``(L, dL/dalpha, dL/ddtau, dL/dtheta per gate)`` for a workload, from
    ``S0`` when given (the parameters do not act on it)."""
    steps = w.n_steps if n_steps is None else n_steps
    a, recs = forward_record(w.n, w.strings, w.alphas, w.schedule, w.dtau, steps, w.delta, w.K, S0)
    L, dth, _ = backward(w.n, w.strings, recs, a, obs_strings, obs_coefs)
    da, dd = parameter_gradients(w.strings, w.alphas, recs, dth, w.dtau)
    return L, da, dd, dth
