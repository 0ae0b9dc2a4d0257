"""CPU oracle for imaginary-time Pauli propagation (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import anything here.  The GPU library never calls into this package and the
two share no code: the oracle keeps Pauli strings as character strings over
``I X Y Z`` and multiplies them letter by letter with the single-qubit table,
while the library works on packed bit words.

Modules
-------
``itpp``        dictionary-of-strings ITPP (Algorithm 1) in plain Python.
``dense``       dense-matrix references for small ``n``: Pauli matrices, exact
                and Trotterized thermal states, Pauli decomposition.
``freefermion`` Bogoliubov-de Gennes thermal energy of the TFIM chain.
``c_oracle``    ctypes wrapper of the plain C++ twin of ``itpp`` (``c/``).
"""
