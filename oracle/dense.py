"""Dense-matrix references for small systems (test infrastructure only).

Tensor order: qubit 0 is the leftmost Kronecker factor, so basis index
``b = sum_j bit_j * 2^(n-1-j)``.
"""
from __future__ import annotations

from functools import reduce
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

_P1 = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def pauli_matrix(P: str) -> np.ndarray:
    return reduce(np.kron, [_P1[a] for a in P])


def hamiltonian(strings: Sequence[str], alphas: Sequence[float]) -> np.ndarray:
    H = None
    for s, a in zip(strings, alphas):
        M = a * pauli_matrix(s)
        H = M if H is None else H + M
    return H


def gate_matrix(Q: str, theta: float) -> np.ndarray:
    """``V_Q = exp(-(theta/2) Q)`` by the matrix exponential (not the
    cosh/sinh closed form, so it checks that form independently)."""
    return sla.expm(-(theta / 2.0) * pauli_matrix(Q))


def exact_thermal(H: np.ndarray, beta: float) -> np.ndarray:
    """``exp(-beta H) / Tr`` via the eigendecomposition."""
    w, U = np.linalg.eigh(H)
    wb = np.exp(-beta * (w - w.min()))
    rho = (U * wb) @ U.conj().T
    return rho / np.trace(rho).real


def trotter_operator(strings: Sequence[str], alphas: Sequence[float],
                     schedule: Sequence[Tuple[int, float]], dtau: float, n_steps: int) -> np.ndarray:
    """``U = V_1 V_2 ... V_G`` over all gates in application order.

    ITPP maps rho -> V^dagger rho V gate by gate, so after all gates
    rho = U^dagger rho0 U (Eq. ThermalTrotter with rho0 proportional to I)."""
    n = len(strings[0])
    step = np.eye(2 ** n, dtype=complex)
    for k, m in schedule:
        if strings[k] == "I" * n:
            continue
        step = step @ gate_matrix(strings[k], alphas[k] * m * dtau)
    return np.linalg.matrix_power(step, n_steps)


def trotter_thermal(strings, alphas, schedule, dtau, n_steps) -> np.ndarray:
    U = trotter_operator(strings, alphas, schedule, dtau, n_steps)
    rho = U.conj().T @ U
    return rho / np.trace(rho).real


def pauli_coefficients(rho: np.ndarray, tol: float = 0.0) -> Dict[str, float]:
    """All ``a_P = Tr(P rho)`` (so ``rho = 2^-n sum a_P P`` when Tr rho = 1).

    For ``P = i^{x.z} X^x Z^z``: ``Tr(X^x Z^z rho) = sum_m (-1)^{z.m}
    rho[m, m xor x]``; the sum over ``m`` for every ``z`` is a Walsh-Hadamard
    transform of the diagonal-offset vector ``rho[m, m xor x]``."""
    dim = rho.shape[0]
    n = dim.bit_length() - 1
    m = np.arange(dim)
    out: Dict[str, float] = {}
    for xb in range(dim):
        f = rho[m, m ^ xb].astype(complex)
        # fast Walsh-Hadamard transform: F[zb] = sum_m (-1)^{popcount(zb & m)} f[m]
        F = f.copy()
        h = 1
        while h < dim:
            F = F.reshape(-1, 2, h)
            a = F[:, 0, :].copy()
            b = F[:, 1, :].copy()
            F[:, 0, :] = a + b
            F[:, 1, :] = a - b
            F = F.reshape(dim)
            h *= 2
        for zb in range(dim):
            val = F[zb]
            ny = bin(xb & zb).count("1")
            val = val * (1j ** ny)
            if abs(val) > tol:
                letters = []
                for j in range(n):
                    bit = 1 << (n - 1 - j)
                    xj = bool(xb & bit)
                    zj = bool(zb & bit)
                    letters.append("I" if not xj and not zj else "X" if xj and not zj else "Z" if zj and not xj else "Y")
                if abs(val.imag) > 1e-9 * max(1.0, abs(val.real)):
                    raise ValueError("non-Hermitian input: imaginary Pauli coefficient")
                out["".join(letters)] = float(val.real)
    return out


def expectation(rho: np.ndarray, O: np.ndarray) -> float:
    return float(np.real(np.trace(O @ rho)))


def weight_projected_trotter(strings: Sequence[str], alphas: Sequence[float],
                             schedule: Sequence[Tuple[int, float]], dtau: float, n_steps: int,
                             max_weight: int) -> Dict[str, float]:
    """Trotter product applied gate by gate to rho = I with the Pauli-weight
    cutoff of Sec. II.B after every gate, as a linear projection: rho ->
    V rho V (V = exp(-(theta/2) Q) by the matrix exponential), then
    rho -> 2^-n sum over P of weight <= max_weight of Tr(P rho) P.  Returns
    the coefficients a_P = Tr(P rho) / Tr(rho) of the final state (the
    projection is linear, so normalising once at the end equals normalising
    after every gate)."""
    n = len(strings[0])
    dim = 2 ** n
    letters = "IXYZ"
    basis = []
    for idx in range(4 ** n):
        P = "".join(letters[(idx >> (2 * j)) & 3] for j in range(n))
        if sum(1 for a in P if a != "I") <= max_weight:
            basis.append((P, pauli_matrix(P)))
    rho = np.eye(dim, dtype=complex)
    for _ in range(n_steps):
        for k, m in schedule:
            Q = strings[k]
            if Q == "I" * n:
                continue
            V = gate_matrix(Q, alphas[k] * m * dtau)
            rho = V @ rho @ V
            proj = np.zeros_like(rho)
            for P, M in basis:
                proj += (np.trace(M @ rho) / dim) * M
            rho = proj
    tr = np.trace(rho).real
    out: Dict[str, float] = {}
    for P, M in basis:
        a = np.trace(M @ rho) / tr
        if abs(a.imag) > 1e-9:
            raise ValueError("imaginary Pauli coefficient")
        out[P] = float(a.real)
    return out
