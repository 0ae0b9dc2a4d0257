"""Squared-state observables (test infrastructure only).

Sec. II.C gives <O>_{2 tau} ~= Tr[(O rho) rho] / Tr[rho^2] for the ITPP state
rho at imaginary time tau, evaluated without forming rho^2: expand O rho and
take its overlap with rho; the denominator is the purity, the l2 norm of the
Pauli coefficients.

With rho = 2^-n sum_P a_P P (a_I = 1, Tr rho = 1) and O = sum_j o_j Q_j:
* Tr[rho^2] = 2^-n * sum_P a_P^2, so ``purity = sum_P a_P^2``;
* Tr[(O rho) rho] = 2^-n * sum_j o_j sum_P a_P a_R Re(i^k), where Q_j P = i^k R.
  A string P that commutes with Q_j gives k = 0 or 2 (a sign +-1); one that
  anticommutes gives an imaginary term that cancels against the term of R,
  so only commuting strings are summed: ``num``.
* <O>_{2 tau} = num / purity.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

from .itpp import OracleError, commutes, pauli_product


def squared_expectation(S: Dict[str, float], strings: Sequence[str], coefs: Sequence[float]) -> Tuple[float, float]:
    """``(num, purity)`` of the squared state for O = sum_j coefs[j] strings[j]."""
    terms = []
    for Q, o in zip(strings, coefs):
        for P, a in S.items():
            if not commutes(P, Q):
                continue
            k, R = pauli_product(Q, P)  # Q P = i^k R
            if k % 2:
                raise OracleError("commuting strings gave an imaginary phase")
            aR = S.get(R)
            if aR is None:
                continue
            s = 1.0 if k == 0 else -1.0
            terms.append(o * (a * aR) * s)
    num = math.fsum(terms)
    purity = math.fsum(float(a) * float(a) for a in S.values())
    return num, purity
