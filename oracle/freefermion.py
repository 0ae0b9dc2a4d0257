"""Free-fermion (Bogoliubov-de Gennes) thermal values of the TFIM chain
``H = -J sum Z_i Z_{i+1} - h sum X_i`` (Eq. TFIM; test infrastructure only).

Jordan-Wigner with the field axis as parity: ``g_{2i} = (prod_{j<i} X_j) Z_i``,
``g_{2i+1} = (prod_{j<i} X_j) Y_i``.  Then ``X_i = i g_{2i} g_{2i+1}`` and
``Z_i Z_{i+1} = i g_{2i+1} g_{2i+2}``, so ``H = (i/4) g^T M g`` with a real
antisymmetric ``M`` (``M[2i,2i+1] = -2h``, ``M[2i+1,2i+2] = -2J``).  The
periodic bond equals ``-i P g_{2n-1} g_0`` with the parity ``P = prod X_j``,
so each parity sector ``p`` is a quadratic ``H_p`` with
``M[2n-1,0] = 2 J p`` and ``Z = sum_p Tr[(1 + p P)/2 exp(-beta H_p)]``.
For the quadratic ``H_p`` with single-particle energies ``e_k >= 0``:
``Tr exp(-beta H_p) = prod 2 cosh(beta e_k / 2)`` and
``Tr P exp(-beta H_p) = (-1)^n sgn Pf(M_p) prod 2 sinh(beta e_k / 2)``.
These closed forms are checked against exact diagonalisation in the tests.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np


def majorana_matrix(n: int, J: float, h: float, periodic: bool, parity: int = 1) -> np.ndarray:
    M = np.zeros((2 * n, 2 * n))
    for i in range(n):
        M[2 * i, 2 * i + 1] = -2.0 * h
    for i in range(n - 1):
        M[2 * i + 1, 2 * i + 2] = -2.0 * J
    if periodic:
        M[2 * n - 1, 0] = 2.0 * J * parity
    return M - M.T


def pfaffian(A: np.ndarray) -> float:
    """Pfaffian of a real antisymmetric matrix (Parlett-Reid elimination with
    pivoting)."""
    A = np.array(A, dtype=float, copy=True)
    m = A.shape[0]
    if m % 2:
        return 0.0
    pf = 1.0
    for k in range(0, m - 1, 2):
        kp = k + 1 + int(np.argmax(np.abs(A[k + 1:, k])))
        if kp != k + 1:
            A[[k + 1, kp], :] = A[[kp, k + 1], :]
            A[:, [k + 1, kp]] = A[:, [kp, k + 1]]
            pf = -pf
        if A[k + 1, k] == 0.0:
            return 0.0
        pf *= A[k, k + 1]
        if k + 2 < m:
            tau = A[k, k + 2:] / A[k, k + 1]
            col = A[k + 2:, k + 1].copy()
            A[k + 2:, k + 2:] += np.outer(tau, col) - np.outer(col, tau)
    return pf


def single_particle_energies(M: np.ndarray) -> np.ndarray:
    """Non-negative ``e_k`` with ``iM`` having eigenvalues ``+-e_k``."""
    ev = np.linalg.eigvalsh(1j * M)
    ev = np.sort(np.abs(ev))
    return ev[::2]  # each |e| appears twice


def _cosh_sinh_terms(e: np.ndarray, beta: float) -> Tuple[float, float, float, float]:
    """log|prod 2cosh|, d/dbeta of it, and the same for prod 2sinh (or -inf)."""
    x = beta * e / 2.0
    logc = float(np.sum(np.logaddexp(x, -x)))
    dlogc = float(np.sum(e / 2.0 * np.tanh(x)))
    if np.any(x == 0.0):
        return logc, dlogc, -math.inf, 0.0
    logs = float(np.sum(np.log(2.0 * np.sinh(x)) if np.all(x < 300) else x + np.log1p(-np.exp(-2 * x))))
    dlogs = float(np.sum(e / 2.0 / np.tanh(x)))
    return logc, dlogc, logs, dlogs


def thermal_energy(n: int, J: float, h: float, beta: float, periodic: bool) -> float:
    """``<H>`` of ``exp(-beta H)/Z`` for the TFIM chain."""
    if not periodic:
        e = single_particle_energies(majorana_matrix(n, J, h, False))
        return float(-np.sum(e / 2.0 * np.tanh(beta * e / 2.0)))
    # four-term parity-projected partition function
    logs = []
    for p in (1, -1):
        M = majorana_matrix(n, J, h, True, p)
        e = single_particle_energies(M)
        sgn = np.sign(pfaffian(M)) * (-1) ** n
        lc, dc, ls, ds = _cosh_sinh_terms(e, beta)
        logs.append((lc, dc, 1.0))
        if ls > -math.inf and sgn != 0:
            logs.append((ls, ds, float(p * sgn)))
    ref = max(l for l, _, _ in logs)
    Z = sum(s * math.exp(l - ref) for l, _, s in logs)
    dZ = sum(s * d * math.exp(l - ref) for l, d, s in logs)
    return float(-dZ / Z)


def ground_energy(n: int, J: float, h: float, periodic: bool) -> float:
    """Ground-state energy (open chain: BdG vacuum)."""
    if periodic:
        raise NotImplementedError("periodic ground state needs the parity analysis")
    e = single_particle_energies(majorana_matrix(n, J, h, False))
    return float(-np.sum(e) / 2.0)


def covariance(n: int, J: float, h: float, beta: float) -> np.ndarray:
    """``G[a,b] = (i/2) <[g_a, g_b]>`` of the open-chain thermal state,
    ``G = i tanh(beta (iM) / 2)``."""
    M = majorana_matrix(n, J, h, False)
    w, U = np.linalg.eigh(1j * M)
    T = (U * np.tanh(beta * w / 2.0)) @ U.conj().T
    G = 1j * T
    return np.real(G)


def zz_correlation(n: int, J: float, h: float, beta: float, r: int, start: int = 0) -> float:
    """``<Z_s Z_{s+r}>`` (open chain) = Pf of the covariance block of
    Majoranas ``2s+1 .. 2(s+r)`` (``Z_s Z_{s+r} = i^r g_{2s+1} ... g_{2s+2r}``)."""
    G = covariance(n, J, h, beta)
    idx = list(range(2 * start + 1, 2 * (start + r) + 1))
    return float(pfaffian(G[np.ix_(idx, idx)]))
