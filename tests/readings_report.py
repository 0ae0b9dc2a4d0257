"""Report of threshold readings for the paper's ground-state count at
threshold 2^-7 (not a test; CPU only, C++ oracle).

Sec. III.C quotes 42,466 strings at threshold 2^-7 for the open N = 12 TFIM
(J = 1, h = 0.5, dtau = 0.04, tau = 20), with relative energy error ~1e-2.
Algorithm 1 (threshold after every gate) keeps far fewer there.  This runs
the oracle under the readings of where the threshold applies:
0 = after every gate (Algorithm 1), 1 = once per Trotter step on the
normalised state, 2 = on every contribution before the accumulation (then on
the sums), 3 = once per Trotter step on the coefficients before the step's
normalisation, each with the printed gate angle h dtau and with the doubled angle
of beta = 2 tau, and prints the strings kept at the end and the energy error
against the free-fermion ground state.

Usage (from the repository root):
    python tests/readings_report.py [cases as reading:angle_multiplier:exponent[:order], e.g. 1:1:7]
order (default 1): 1 = first order, ZZ gates then X gates; 3 = first order,
X gates then ZZ gates; 2 = Strang (half ZZ, X, half ZZ).
(no cases: every reading, both angles, thresholds 2^-6, 2^-7, 2^-8; the runs
go to a process pool, one per core, and the table prints in case order).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import itpp_workloads as W  # noqa: E402
from oracle import c_oracle  # noqa: E402
from oracle import freefermion as FF  # noqa: E402
from oracle import itpp as OR  # noqa: E402


def run(n, reading, delta, angle_mult, order=1, steps=500, dtau=0.04, J=1.0, h=0.5):
    strings, alphas, _ = W.tfim_terms(n, J, h, False)
    if order == 3:
        sched = [(k, 1.0) for k in range(n - 1, 2 * n - 1)] + [(k, 1.0) for k in range(n - 1)]
    else:
        sched = W.tfim_schedule(n - 1, n, order)
    o = c_oracle.COracle(n)
    o.set_reading(reading)
    t0 = time.perf_counter()
    o.evolve(strings, alphas, [(k, m * angle_mult) for k, m in sched], dtau, steps, delta, 1 << 40)
    S = o.state()
    e = OR.expect(S, strings, alphas) / n
    return len(S), e, time.perf_counter() - t0


def one(case):
    reading, mult, ex, order = case
    cnt, e, dt = run(12, reading, 2.0 ** -ex, mult, order)
    return case, cnt, e, dt


def main():
    from concurrent.futures import ProcessPoolExecutor

    n = 12
    if len(sys.argv) > 1:
        cases = [tuple(int(v) if i != 1 else float(v) for i, v in enumerate(a.split(":"))) for a in sys.argv[1:]]
        cases = [c + (1,) if len(c) == 3 else c for c in cases]
    else:
        cases = [(r, m, ex, 1) for r in (0, 1, 2) for m in (1.0, 2.0) for ex in (6, 7, 8)]
    exact = FF.ground_energy(n, 1.0, 0.5, False) / n
    print(f"# Threshold readings, open TFIM N = {n}, J = 1, h = 0.5, dtau = 0.04, 500 steps\n")
    print("Command (repository root, CPU): `python tests/readings_report.py " + " ".join(sys.argv[1:]) + "`\n")
    print(f"Free-fermion ground-state energy per site: {exact:.10f}.  The paper quotes 42,466 strings at 2^-7.\n")
    print("| reading | gate order | gate angle | threshold | strings at the end | energy per site | relative error | seconds |")
    print("|---|---|---|---|---:|---:|---:|---:|")
    names = {0: "after every gate (Algorithm 1)", 1: "once per Trotter step", 2: "every contribution, then sums",
             3: "once per Trotter step, before normalising"}
    orders = {1: "ZZ then X", 3: "X then ZZ", 2: "Strang"}
    with ProcessPoolExecutor(max_workers=min(len(cases), os.cpu_count() or 1)) as ex:
        for (reading, mult, e2, order), cnt, e, dt in ex.map(one, cases):
            aname = "h dtau" if mult == 1.0 else f"{mult:g} h dtau"
            print(f"| {names[reading]} | {orders[order]} | {aname} | 2^-{e2} | {cnt} | {e:.10f} | "
                  f"{abs(e - exact) / abs(exact):.3e} | {dt:.1f} |", flush=True)


if __name__ == "__main__":
    main()
