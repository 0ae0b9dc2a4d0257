"""ctypes binding of ``libitpp.so`` (argument marshalling only).

Every step of the propagation runs in the library's HIP kernels; this module
converts Python strings and lists to the packed words and arrays the C ABI
takes and turns status codes into exceptions.  There is no fallback: if the
library is missing, importing the engine fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libitpp.so")

STATUS = {0: "ITPP_OK", 1: "ITPP_ERR_ARG", 2: "ITPP_ERR_OOM", 3: "ITPP_ERR_CAP",
          4: "ITPP_ERR_NUMERIC", 5: "ITPP_ERR_DEVICE", 6: "ITPP_ERR_STATE"}

# Every entry point declared in include/itpp.h.
EXPORTED = ["itpp_create", "itpp_destroy", "itpp_set_hamiltonian", "itpp_set_schedule",
            "itpp_reset", "itpp_import", "itpp_evolve", "itpp_evolve_gates", "itpp_expect", "itpp_num_terms", "itpp_export",
            "itpp_expect_device", "itpp_export_device", "itpp_expect_squared", "itpp_expect_squared_noalloc",
            "itpp_set_adjoint", "itpp_backward", "itpp_num_gates", "itpp_set_option", "itpp_set_timing", "itpp_get_timing",
            "itpp_batch_create", "itpp_batch_destroy", "itpp_batch_instance", "itpp_batch_set_workers",
            "itpp_batch_evolve", "itpp_batch_autotune", "itpp_batch_last_error",
            "itpp_last_error", "itpp_version"]


class ItppConfig(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("threshold", ctypes.c_double), ("max_terms", ctypes.c_int64),
                ("cap_policy", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("device_bytes_limit", ctypes.c_int64)]


class ItppStats(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int64), ("n_gates", ctypes.c_int64),
                ("term_updates", ctypes.c_double), ("c_identity", ctypes.c_double),
                ("cap_hit", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("alg_bytes", ctypes.c_double), ("spec_gates", ctypes.c_int64),
                ("spec_retries", ctypes.c_int64), ("written", ctypes.c_double),
                ("c_I_min", ctypes.c_double), ("c_I_max", ctypes.c_double),
                ("kth_abs_min", ctypes.c_double), ("graph_steps", ctypes.c_int64)]


class ItppTiming(ctypes.Structure):
    _fields_ = [("gate_ms", ctypes.c_double), ("select_ms", ctypes.c_double),
                ("gate_launches", ctypes.c_int64), ("alg_bytes", ctypes.c_double)]


class ItppError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None):
    """Load libitpp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with paper_2601_14400_amd.build.build()")
    # One HIP runtime per process: load PyTorch's first so that the library's
    # libamdhip64.so.7 dependency binds to the runtime torch already uses (a
    # stream or device pointer from torch is then valid in the library).
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.itpp_create.argtypes = [ctypes.POINTER(ItppConfig), ctypes.POINTER(vp)]
    lib.itpp_destroy.argtypes = [vp]
    lib.itpp_set_hamiltonian.argtypes = [vp, i32, vp, vp, vp]
    lib.itpp_set_schedule.argtypes = [vp, i32, vp, vp]
    lib.itpp_reset.argtypes = [vp]
    lib.itpp_import.argtypes = [vp, i64, vp, vp, vp]
    lib.itpp_evolve.argtypes = [vp, dbl, i64, ctypes.POINTER(ItppStats)]
    lib.itpp_evolve_gates.argtypes = [vp, dbl, i64, ctypes.POINTER(ItppStats)]
    lib.itpp_expect.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(dbl)]
    lib.itpp_num_terms.argtypes = [vp, ctypes.POINTER(i64)]
    lib.itpp_export.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(i64)]
    lib.itpp_expect_device.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.itpp_expect_squared.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.itpp_expect_squared_noalloc.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.itpp_export_device.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(i64)]
    lib.itpp_set_adjoint.argtypes = [vp, i32, i64]
    lib.itpp_backward.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(dbl), vp, ctypes.POINTER(dbl), vp, i64]
    lib.itpp_num_gates.argtypes = [vp, ctypes.POINTER(i64)]
    lib.itpp_set_option.argtypes = [vp, i32, dbl]
    lib.itpp_set_timing.argtypes = [vp, i32]
    lib.itpp_get_timing.argtypes = [vp, ctypes.POINTER(ItppTiming)]
    lib.itpp_batch_create.argtypes = [i32, ctypes.POINTER(ItppConfig), ctypes.POINTER(vp)]
    lib.itpp_batch_destroy.argtypes = [vp]
    lib.itpp_batch_instance.argtypes = [vp, i32]
    lib.itpp_batch_set_workers.argtypes = [vp, i32]
    lib.itpp_batch_evolve.argtypes = [vp, vp, vp, vp]
    lib.itpp_batch_autotune.argtypes = [vp, vp, i64, i64, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.itpp_batch_last_error.argtypes = [vp]
    lib.itpp_batch_last_error.restype = ctypes.c_char_p
    lib.itpp_last_error.argtypes = [vp]
    lib.itpp_last_error.restype = ctypes.c_char_p
    lib.itpp_version.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("itpp_last_error", "itpp_version", "itpp_batch_last_error", "itpp_batch_instance"):
            getattr(lib, name).restype = ctypes.c_int
    lib.itpp_batch_instance.restype = vp
    if path is None:
        _lib = lib
    return lib


def strings_to_words(strings: Sequence[str], n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Pack 'IXYZ' strings (character j = qubit j) into x/z words."""
    W = (n + 63) // 64
    x = np.zeros((len(strings), W), dtype=np.uint64)
    z = np.zeros((len(strings), W), dtype=np.uint64)
    for s, P in enumerate(strings):
        if len(P) != n:
            raise ValueError(f"string length {len(P)} != n_qubits {n}")
        for j, a in enumerate(P):
            if a == "I":
                continue
            bit = np.uint64(1) << np.uint64(j & 63)
            if a in "XY":
                x[s, j >> 6] |= bit
            if a in "ZY":
                z[s, j >> 6] |= bit
            if a not in "XYZ":
                raise ValueError(f"bad Pauli letter {a!r}")
    return x, z


def words_to_strings(x: np.ndarray, z: np.ndarray, n: int) -> List[str]:
    """Unpack x/z words into 'IXYZ' strings (character j = qubit j)."""
    out: List[str] = []
    if n <= 0:
        return [""] * x.shape[0]
    j = np.arange(n)
    word = j >> 6
    shift = (j & 63).astype(np.uint64)
    lut = np.frombuffer(b"IXZY", dtype=np.uint8)
    one = np.uint64(1)
    for r0 in range(0, x.shape[0], 1 << 16):
        xs = np.asarray(x[r0:r0 + (1 << 16)], dtype=np.uint64)
        zs = np.asarray(z[r0:r0 + (1 << 16)], dtype=np.uint64)
        code = ((xs[:, word] >> shift) & one) | (((zs[:, word] >> shift) & one) << one)
        chars = np.ascontiguousarray(lut[code.astype(np.uint8)])
        out.extend(b.decode("ascii") for b in chars.view(f"S{n}").ravel())
    return out


def _current_stream():
    try:
        import torch

        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(None)


class Engine:
    """One ITPP state on the current HIP device (see include/itpp.h)."""

    def __init__(self, n_qubits: int, threshold: float, max_terms: int, precision: str = "f64",
                 cap_policy: str = "topk", stream=None, device_bytes_limit: int = 0):
        self._lib = load_library()
        self.n = int(n_qubits)
        self.W = (self.n + 63) // 64
        self.n_terms = 0
        cfg = ItppConfig()
        cfg.n_qubits = self.n
        cfg.precision = {"f64": 0, "f32": 1}[precision]
        cfg.threshold = float(threshold)
        cfg.max_terms = int(max_terms)
        cfg.cap_policy = {"topk": 0, "fail": 1}[cap_policy]
        cfg.stream = stream if stream is not None else _current_stream()
        cfg.device_bytes_limit = int(device_bytes_limit)
        h = ctypes.c_void_p()
        rc = self._lib.itpp_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            msg = self._lib.itpp_last_error(None)
            raise ItppError(rc, "itpp_create: " + (msg.decode() if msg else ""))
        self._h = h

    def _check(self, rc: int):
        if rc != 0:
            msg = self._lib.itpp_last_error(self._h)
            raise ItppError(rc, msg.decode() if msg else "")

    @classmethod
    def _borrowed(cls, lib, handle, n_qubits: int):
        """An Engine view of a context owned by a Batch (not destroyed here)."""
        e = cls.__new__(cls)
        e._lib = lib
        e.n = int(n_qubits)
        e.W = (e.n + 63) // 64
        e.n_terms = 0
        e._h = handle
        e._owned = False
        return e

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                self._lib.itpp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_hamiltonian(self, strings: Sequence[str], alphas: Sequence[float]):
        self.n_terms = len(strings)
        x, z = strings_to_words(strings, self.n)
        a = np.ascontiguousarray(alphas, dtype=np.float64)
        self._check(self._lib.itpp_set_hamiltonian(self._h, len(strings), x.ctypes.data,
                                                   z.ctypes.data, a.ctypes.data))

    def set_schedule(self, schedule: Sequence[Tuple[int, float]]):
        ti = np.ascontiguousarray([k for k, _ in schedule], dtype=np.int32)
        mu = np.ascontiguousarray([m for _, m in schedule], dtype=np.float64)
        self._check(self._lib.itpp_set_schedule(self._h, len(schedule), ti.ctypes.data, mu.ctypes.data))

    def reset(self):
        self._check(self._lib.itpp_reset(self._h))

    def import_words(self, x: np.ndarray, z: np.ndarray, coef: np.ndarray):
        """Replace the state by sum_j coef[j] P_j (canonical x/z words, the
        layout export() returns); normalised by the identity's coefficient."""
        x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, self.W)
        z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, self.W)
        coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1)
        if not (x.shape[0] == z.shape[0] == coef.shape[0]):
            raise ValueError("x, z and coef must describe the same number of strings")
        self._check(self._lib.itpp_import(self._h, ctypes.c_int64(coef.shape[0]), x.ctypes.data, z.ctypes.data,
                                          coef.ctypes.data))

    def load(self, S: Dict[str, float]):
        """Replace the state by the strings and coefficients of S."""
        keys = list(S)
        x, z = strings_to_words(keys, self.n)
        self.import_words(x, z, np.array([S[k] for k in keys], dtype=np.float64))

    def evolve(self, dtau: float, n_steps: int, log: Optional[List[Dict[str, float]]] = None) -> Dict[str, float]:
        """n_steps Trotter steps of dtau; returns the call's statistics.  With
        ``log`` (a list) the steps run one call each and every step's
        statistics are appended to it (a per-step metrics log: strings kept,
        c_I, whether the cap bound, the smallest K-th magnitude, redone
        gates, ...); the summed statistics are returned as without it."""
        if log is None:
            st = ItppStats()
            self._check(self._lib.itpp_evolve(self._h, float(dtau), int(n_steps), ctypes.byref(st)))
            return self._stats(st)
        tot: Optional[Dict[str, float]] = None
        for _ in range(int(n_steps)):
            st = ItppStats()
            self._check(self._lib.itpp_evolve(self._h, float(dtau), 1, ctypes.byref(st)))
            d = self._stats(st)
            log.append(d)
            if tot is None:
                tot = dict(d)
            else:
                for k in ("n_gates", "term_updates", "alg_bytes", "spec_gates", "spec_retries", "written",
                          "graph_steps"):
                    tot[k] += d[k]
                for k in ("n_terms", "c_identity"):
                    tot[k] = d[k]
                tot["cap_hit"] = max(tot["cap_hit"], d["cap_hit"])
                tot["c_I_min"] = min(tot["c_I_min"], d["c_I_min"])
                tot["c_I_max"] = max(tot["c_I_max"], d["c_I_max"])
                tot["kth_abs_min"] = min(tot["kth_abs_min"], d["kth_abs_min"])
        if tot is None:
            return self.evolve(dtau, 0)
        return tot

    def evolve_gates(self, dtau: float, n_gates: int) -> Dict[str, float]:
        st = ItppStats()
        self._check(self._lib.itpp_evolve_gates(self._h, float(dtau), int(n_gates), ctypes.byref(st)))
        return self._stats(st)

    def set_adjoint(self, every_steps: int, workspace_bytes: int = 0):
        """Store forward checkpoints every ``every_steps`` Trotter steps so
        that ``backward`` can run (takes effect from the next reset)."""
        self._check(self._lib.itpp_set_adjoint(self._h, int(every_steps), int(workspace_bytes)))

    def backward(self, strings: Sequence[str], coefs: Sequence[float], want_theta: bool = False):
        """``L = sum_j coefs[j] a[strings[j]]`` and its derivatives with the
        truncation support held fixed: ``(L, dL/dalpha per term, dL/ddtau,
        dL/dtheta per gate or None)``."""
        x, z = strings_to_words(strings, self.n)
        c = np.ascontiguousarray(coefs, dtype=np.float64)
        val = ctypes.c_double()
        dd = ctypes.c_double()
        da = np.zeros(max(self.n_terms, 1), dtype=np.float64)
        ng = self.num_gates()
        dth = np.zeros(max(ng, 1), dtype=np.float64) if want_theta else None
        self._check(self._lib.itpp_backward(self._h, len(strings), x.ctypes.data, z.ctypes.data, c.ctypes.data,
                                            ctypes.byref(val), da.ctypes.data, ctypes.byref(dd),
                                            dth.ctypes.data if dth is not None else None,
                                            len(dth) if dth is not None else 0))
        return (float(val.value), da[: self.n_terms], float(dd.value),
                dth[:ng] if dth is not None else None)

    def num_gates(self) -> int:
        """Elementary gates applied since the last reset or load."""
        v = ctypes.c_int64(0)
        self._check(self._lib.itpp_num_gates(self._h, ctypes.byref(v)))
        return int(v.value)

    @staticmethod
    def _stats(st):
        return {"n_terms": st.n_terms, "n_gates": st.n_gates, "term_updates": st.term_updates,
                "c_identity": st.c_identity, "cap_hit": st.cap_hit, "alg_bytes": st.alg_bytes,
                "spec_gates": st.spec_gates, "spec_retries": st.spec_retries, "written": st.written,
                "c_I_min": st.c_I_min, "c_I_max": st.c_I_max, "kth_abs_min": st.kth_abs_min,
                "graph_steps": st.graph_steps}

    def set_option(self, name: str, value: float):
        opt = {"speculation": 1, "spec_margin": 2, "gate_shape": 3, "real_time": 4, "graphs": 5,
               "grid_div": 6, "max_weight": 7}[name]
        self._check(self._lib.itpp_set_option(self._h, opt, float(value)))

    def set_timing(self, enable: bool = True):
        self._check(self._lib.itpp_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> Dict[str, float]:
        t = ItppTiming()
        self._check(self._lib.itpp_get_timing(self._h, ctypes.byref(t)))
        return {"gate_ms": t.gate_ms, "select_ms": t.select_ms, "gate_launches": t.gate_launches,
                "alg_bytes": t.alg_bytes}

    def expect(self, strings: Sequence[str], coefs: Sequence[float]) -> float:
        x, z = strings_to_words(strings, self.n)
        c = np.ascontiguousarray(coefs, dtype=np.float64)
        out = ctypes.c_double()
        self._check(self._lib.itpp_expect(self._h, len(strings), x.ctypes.data, z.ctypes.data,
                                          c.ctypes.data, ctypes.byref(out)))
        return float(out.value)

    def num_terms(self) -> int:
        v = ctypes.c_int64()
        self._check(self._lib.itpp_num_terms(self._h, ctypes.byref(v)))
        return int(v.value)

    def export(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        m = self.num_terms()
        x = np.zeros((max(m, 1), self.W), dtype=np.uint64)
        z = np.zeros((max(m, 1), self.W), dtype=np.uint64)
        c = np.zeros(max(m, 1), dtype=np.float64)
        n_out = ctypes.c_int64()
        self._check(self._lib.itpp_export(self._h, m, x.ctypes.data, z.ctypes.data, c.ctypes.data,
                                          ctypes.byref(n_out)))
        k = int(n_out.value)
        return x[:k], z[:k], c[:k]

    def expect_squared(self, strings: Sequence[str], coefs: Sequence[float],
                       noalloc: bool = False) -> Tuple[float, float]:
        """(<O>_{2 tau}, purity) of the squared state, O = sum_j coefs[j] strings[j]
        (Tr[(O rho) rho] / Tr[rho^2] and sum_P a_P^2).  noalloc: through
        itpp_expect_squared_noalloc (no allocation; library scratch)."""
        x, z = strings_to_words(strings, self.n)
        c = np.ascontiguousarray(coefs, dtype=np.float64)
        v = ctypes.c_double()
        p = ctypes.c_double()
        fn = self._lib.itpp_expect_squared_noalloc if noalloc else self._lib.itpp_expect_squared
        self._check(fn(self._h, len(strings), x.ctypes.data, z.ctypes.data, c.ctypes.data,
                       ctypes.byref(v), ctypes.byref(p)))
        return float(v.value), float(p.value)

    def expect_device(self, x, z, coef, out=None):
        """<O> for observables held in torch device tensors: x, z int64 (the
        bit patterns of the canonical words, shape (m, W)), coef float64 (m,).
        Enqueued on the engine's stream (the torch stream current when the
        engine was created); returns a 0-dim float64 device tensor."""
        import torch

        x = x.contiguous()
        z = z.contiguous()
        coef = coef.contiguous()
        m = coef.shape[0]
        for t, dt in ((x, torch.int64), (z, torch.int64), (coef, torch.float64)):
            if t.dtype != dt or not t.is_cuda:
                raise ValueError("expect_device takes int64 x, z and float64 coef device tensors")
        if x.shape != (m, self.W) or z.shape != (m, self.W):
            raise ValueError(f"x and z must have shape ({m}, {self.W})")
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=coef.device)
        self._check(self._lib.itpp_expect_device(self._h, m, x.data_ptr(), z.data_ptr(), coef.data_ptr(),
                                                 out.data_ptr()))
        return out

    def export_device(self):
        """The surviving strings as torch device tensors (x, z int64 bit
        patterns of shape (m, W), normalised float64 coefficients), in storage
        order."""
        import torch

        m = self.num_terms()
        dev = torch.device("cuda", torch.cuda.current_device())
        x = torch.empty((max(m, 1), self.W), dtype=torch.int64, device=dev)
        z = torch.empty((max(m, 1), self.W), dtype=torch.int64, device=dev)
        c = torch.empty((max(m, 1),), dtype=torch.float64, device=dev)
        n_out = ctypes.c_int64()
        self._check(self._lib.itpp_export_device(self._h, m, x.data_ptr(), z.data_ptr(), c.data_ptr(),
                                                 ctypes.byref(n_out)))
        k = int(n_out.value)
        return x[:k], z[:k], c[:k]

    def state(self) -> Dict[str, float]:
        x, z, c = self.export()
        return dict(zip(words_to_strings(x, z, self.n), c.tolist()))


def version() -> str:
    return load_library().itpp_version().decode()


class Batch:
    """Independent instances in one device arena, evolved concurrently
    (see itpp_batch_* in include/itpp.h).  ``instances[i]`` is an Engine
    view of instance i for the single-instance calls."""

    def __init__(self, instance_configs: Sequence[Dict]):
        self._lib = load_library()
        n = len(instance_configs)
        arr = (ItppConfig * n)()
        for i, c in enumerate(instance_configs):
            arr[i].n_qubits = int(c["n_qubits"])
            arr[i].precision = {"f64": 0, "f32": 1}[c.get("precision", "f64")]
            arr[i].threshold = float(c["threshold"])
            arr[i].max_terms = int(c["max_terms"])
            arr[i].cap_policy = {"topk": 0, "fail": 1}[c.get("cap_policy", "topk")]
            arr[i].stream = None
            arr[i].device_bytes_limit = int(c.get("device_bytes_limit", 0))
        h = ctypes.c_void_p()
        rc = self._lib.itpp_batch_create(n, arr, ctypes.byref(h))
        if rc != 0:
            msg = self._lib.itpp_batch_last_error(None)
            raise ItppError(rc, "itpp_batch_create: " + (msg.decode() if msg else ""))
        self._h = h
        self.instances = [Engine._borrowed(self._lib, ctypes.c_void_p(self._lib.itpp_batch_instance(h, i)),
                                           instance_configs[i]["n_qubits"]) for i in range(n)]

    def _check(self, rc: int):
        if rc != 0:
            msg = self._lib.itpp_batch_last_error(self._h)
            raise ItppError(rc, msg.decode() if msg else "")

    def set_workers(self, workers: int):
        self._check(self._lib.itpp_batch_set_workers(self._h, int(workers)))

    def evolve(self, dtaus: Sequence[float], n_steps: Sequence[int]) -> List[Dict[str, float]]:
        n = len(self.instances)
        d = np.ascontiguousarray(dtaus, dtype=np.float64)
        k = np.ascontiguousarray(n_steps, dtype=np.int64)
        st = (ItppStats * n)()
        self._check(self._lib.itpp_batch_evolve(self._h, d.ctypes.data, k.ctypes.data, st))
        out = []
        for i in range(n):
            out.append(Engine._stats(st[i]))
        return out

    def autotune(self, dtaus: Sequence[float], warm_gates: int, probe_gates: int) -> Tuple[int, int, int, float]:
        """(shape code = shape for n <= 64 + 3 * shape for n > 64, workers,
        grid divisor, probe rate); the setting is left applied."""
        d = np.ascontiguousarray(dtaus, dtype=np.float64)
        sh, wk, gd, rate = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(self._lib.itpp_batch_autotune(self._h, d.ctypes.data, int(warm_gates), int(probe_gates),
                                                  ctypes.byref(sh), ctypes.byref(wk), ctypes.byref(gd),
                                                  ctypes.byref(rate)))
        return int(sh.value), int(wk.value), int(gd.value), float(rate.value)

    def close(self):
        if getattr(self, "_h", None):
            for e in self.instances:
                e._h = None
            self._lib.itpp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
