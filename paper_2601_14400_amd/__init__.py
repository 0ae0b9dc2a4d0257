"""MI355X-native imaginary-time Pauli propagation (arXiv 2601.14400).

The engine (``Engine``) is a thin binding of the C ABI in ``include/itpp.h``
implemented by ``libitpp.so`` (hand-written HIP for gfx950).  There is no
CPU path: without the built library, creating an engine raises.
"""
from ._native import Batch, Engine, ItppError, load_library, strings_to_words, version, words_to_strings

__all__ = ["Batch", "Engine", "ItppError", "load_library", "strings_to_words", "words_to_strings", "version",
           "engine_for", "run_workload"]


def engine_for(w, **kw) -> Engine:
    """Engine configured with a workload's Hamiltonian, schedule, threshold and cap."""
    kw.setdefault("precision", w.precision)
    e = Engine(w.n, w.delta, w.K, **kw)
    e.set_hamiltonian(w.strings, w.alphas)
    e.set_schedule(w.schedule)
    return e


def run_workload(w, n_steps=None, **kw):
    e = engine_for(w, **kw)
    st = e.evolve(w.dtau, w.n_steps if n_steps is None else n_steps)
    return e, st


def batch_for(workloads, **kw):
    """Batch with one instance per workload (Hamiltonian, schedule, cap set)."""
    b = Batch([dict(n_qubits=w.n, threshold=w.delta, max_terms=w.K, precision=w.precision, **kw)
               for w in workloads])
    for e, w in zip(b.instances, workloads):
        e.set_hamiltonian(w.strings, w.alphas)
        e.set_schedule(w.schedule)
    return b
