"""ctypes wrapper of the plain C++ dictionary oracle in ``oracle/c``
(test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "itpp_oracle.cpp")
LIB = os.path.join(_HERE, "c", "libitpp_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", SRC, "-o", LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        lib = ctypes.CDLL(LIB)
        lib.itpp_oracle_new.restype = ctypes.c_void_p
        lib.itpp_oracle_new.argtypes = [ctypes.c_int]
        lib.itpp_oracle_new32.restype = ctypes.c_void_p
        lib.itpp_oracle_new32.argtypes = [ctypes.c_int]
        lib.itpp_oracle_free.argtypes = [ctypes.c_void_p]
        lib.itpp_oracle_error.restype = ctypes.c_char_p
        lib.itpp_oracle_error.argtypes = [ctypes.c_void_p]
        lib.itpp_oracle_evolve.restype = ctypes.c_int
        lib.itpp_oracle_evolve.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p,
                                           ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.c_longlong,
                                           ctypes.c_double, ctypes.c_longlong]
        lib.itpp_oracle_set_reading.restype = None
        lib.itpp_oracle_set_reading.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.itpp_oracle_set_max_weight.restype = None
        lib.itpp_oracle_set_max_weight.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.itpp_oracle_size.restype = ctypes.c_longlong
        lib.itpp_oracle_size.argtypes = [ctypes.c_void_p]
        lib.itpp_oracle_term_updates.restype = ctypes.c_double
        lib.itpp_oracle_term_updates.argtypes = [ctypes.c_void_p]
        lib.itpp_oracle_export.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.itpp_oracle_import.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_char_p,
                                           ctypes.c_void_p]
        lib.itpp_oracle_gradients.restype = ctypes.c_int
        lib.itpp_oracle_gradients.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p,
                                              ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_double, ctypes.c_longlong,
                                              ctypes.c_double, ctypes.c_longlong, ctypes.c_int,
                                              ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                                              ctypes.c_void_p]
        lib.itpp_oracle_import_words.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.itpp_oracle_export_words.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


class COracle:
    def __init__(self, n: int, precision: str = "f64"):
        self.n = n
        self._lib = _load()
        self._h = self._lib.itpp_oracle_new32(n) if precision == "f32" else self._lib.itpp_oracle_new(n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.itpp_oracle_free(h)
            self._h = None

    def evolve(self, strings: Sequence[str], alphas: Sequence[float],
               schedule: Sequence[Tuple[int, float]], dtau: float, n_steps: int,
               delta: float, K: int) -> None:
        buf = "".join(strings).encode("ascii")
        a = np.ascontiguousarray(alphas, dtype=np.float64)
        ti = np.ascontiguousarray([k for k, _ in schedule], dtype=np.int32)
        mu = np.ascontiguousarray([m for _, m in schedule], dtype=np.float64)
        rc = self._lib.itpp_oracle_evolve(self._h, len(strings), buf, a.ctypes.data, len(schedule),
                                          ti.ctypes.data, mu.ctypes.data, float(dtau),
                                          int(n_steps), float(delta), int(K))
        if rc != 0:
            raise RuntimeError(self._lib.itpp_oracle_error(self._h).decode())

    def set_reading(self, reading: int) -> None:
        """Where the threshold applies: 0 Algorithm 1 (after every gate),
        1 once per Trotter step, 2 on every contribution before the sums,
        3 once per Trotter step on the coefficients before the step's
        normalisation."""
        self._lib.itpp_oracle_set_reading(self._h, int(reading))

    def set_max_weight(self, max_weight: int) -> None:
        """Pauli-weight cutoff of the following gates (0: none)."""
        self._lib.itpp_oracle_set_max_weight(self._h, int(max_weight))

    def size(self) -> int:
        return int(self._lib.itpp_oracle_size(self._h))

    def term_updates(self) -> float:
        return float(self._lib.itpp_oracle_term_updates(self._h))

    def export(self) -> Tuple[list, np.ndarray]:
        m = self.size()
        sbuf = ctypes.create_string_buffer(m * self.n + 1)
        coef = np.empty(m, dtype=np.float64)
        self._lib.itpp_oracle_export(self._h, sbuf, coef.ctypes.data)
        raw = sbuf.raw[: m * self.n].decode("ascii")
        strings = [raw[i * self.n:(i + 1) * self.n] for i in range(m)]
        return strings, coef

    def state(self) -> Dict[str, float]:
        s, c = self.export()
        return dict(zip(s, c.tolist()))

    def load(self, S: Dict[str, float]) -> None:
        keys = list(S)
        buf = "".join(keys).encode("ascii")
        coef = np.ascontiguousarray([S[k] for k in keys], dtype=np.float64)
        self._lib.itpp_oracle_import(self._h, len(keys), buf, coef.ctypes.data)


    def load_words(self, x: np.ndarray, z: np.ndarray, coef: np.ndarray) -> None:
        """Replace the state by strings given as canonical words, shape (m, W)."""
        x = np.ascontiguousarray(x, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint64)
        c = np.ascontiguousarray(coef, dtype=np.float64)
        self._lib.itpp_oracle_import_words(self._h, len(c), x.shape[1], x.ctypes.data, z.ctypes.data,
                                           c.ctypes.data)

    def export_words(self, W: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """The state as canonical words in ascending (X, Z) order."""
        m = self.size()
        x = np.zeros((m, W), dtype=np.uint64)
        z = np.zeros((m, W), dtype=np.uint64)
        c = np.zeros(m, dtype=np.float64)
        self._lib.itpp_oracle_export_words(self._h, W, x.ctypes.data, z.ctypes.data, c.ctypes.data)
        return x, z, c

    def gradients(self, w, obs_strings: Sequence[str], obs_coefs: Sequence[float],
                  n_steps: Optional[int] = None):
        """Reverse-mode derivatives from the current state (the steps of
        ``oracle.adjoint``): ``(L, dL/dalpha, dL/ddtau, dL/dtheta per gate)``.
        The state becomes the forward run's final state."""
        steps = w.n_steps if n_steps is None else n_steps
        ident = "I" * w.n
        G = steps * sum(1 for k, _ in w.schedule if w.strings[k] != ident)
        buf = "".join(w.strings).encode("ascii")
        a = np.ascontiguousarray(w.alphas, dtype=np.float64)
        ti = np.ascontiguousarray([k for k, _ in w.schedule], dtype=np.int32)
        mu = np.ascontiguousarray([m for _, m in w.schedule], dtype=np.float64)
        ob = "".join(obs_strings).encode("ascii")
        oc = np.ascontiguousarray(obs_coefs, dtype=np.float64)
        L = ctypes.c_double(0.0)
        dd = ctypes.c_double(0.0)
        dth = np.zeros(max(G, 1), dtype=np.float64)
        da = np.zeros(len(w.strings), dtype=np.float64)
        rc = self._lib.itpp_oracle_gradients(self._h, len(w.strings), buf, a.ctypes.data, len(w.schedule),
                                             ti.ctypes.data, mu.ctypes.data, float(w.dtau), int(steps),
                                             float(w.delta), int(w.K), len(oc), ob, oc.ctypes.data,
                                             ctypes.byref(L), dth.ctypes.data, G, da.ctypes.data,
                                             ctypes.byref(dd))
        if rc != 0:
            raise RuntimeError(self._lib.itpp_oracle_error(self._h).decode())
        return L.value, da, dd.value, dth[:G]


def run_workload(w, n_steps=None, K=None, precision=None, max_weight=0) -> COracle:
    o = COracle(w.n, precision or w.precision)
    if max_weight:
        o.set_max_weight(max_weight)
    o.evolve(w.strings, w.alphas, w.schedule, w.dtau, w.n_steps if n_steps is None else n_steps,
             w.delta, w.K if K is None else K)
    return o
