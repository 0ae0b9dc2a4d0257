"""The paper's TFIM experiments (Sec. III) on the GPU engine, with exact
free-fermion references from the oracle; prints markdown tables.

    python tests/experiments_report.py [--quick]

Ordered-phase chain J = 1, h = 0.5, open boundaries, first-order Trotter
steps of dtau = 0.04 (the paper's settings):
1. ground state, N = 12, tau = 20: thresholds 2^-19 .. 2^-5 and none;
2. thermal, N = 12, beta = 3: the same thresholds;
3. fixed cap K = 2,704,156 (the untruncated 12-site support), tau = 20, N = 12 .. 48;
4. K(N, eps0): the smallest cap 2^9 .. 2^24 with relative energy error <= 1e-2
   at beta = 0.08, 0.24, 0.8;
5. readings of the paper's ground-state count at threshold 2^-7 (N = 12,
   500 steps): first order or Strang, gate angle h dtau (Algorithm 1) or
   2 h dtau (beta = 2 tau), open or periodic chain.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import freefermion as FF  # noqa: E402
from paper_2601_14400_amd import experiments as X  # noqa: E402

J, H, DTAU = 1.0, 0.5, 0.04
T0 = time.time()


def log(msg):
    print(f"[report {time.time() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def rel(a, b):
    return abs(a - b) / abs(b)


def sweep_table(title, n, beta, ref, ks):
    print(f"\n### {title}\n")
    print("| threshold | energy per site | relative error | strings at the end | most strings | seconds |")
    print("|---|---:|---:|---:|---:|---:|")
    for d_k in [None] + list(ks):
        delta = 0.0 if d_k is None else 2.0 ** (-d_k)
        r = X.tfim_run(n, J, H, DTAU, beta, delta, 1 << 23, record_betas=[beta])
        E = r["energy_per_site"][-1]
        name = "0 (none)" if d_k is None else f"2^-{d_k}"
        print(f"| {name} | {E:.10f} | {rel(E, ref):.3e} | {r['n_terms'][-1]} | {r['max_terms']} | {r['seconds']:.2f} |",
              flush=True)
        log(f"{title}: threshold {name} done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer sizes and caps")
    args = ap.parse_args()
    ks = list(range(5, 20, 2)) if args.quick else list(range(5, 20))
    print("## TFIM experiments (J = 1, h = 0.5, open, first order, dtau = 0.04)")

    n = 12
    e0 = FF.ground_energy(n, J, H, False) / n
    print(f"\nExact ground-state energy per site (free fermions), N = 12: {e0:.10f}")
    sweep_table("Ground state, N = 12, tau = 20", n, 20.0, e0, ks)
    eth = FF.thermal_energy(n, J, H, 3.0, False) / n
    print(f"\nExact thermal energy per site, N = 12, beta = 3: {eth:.10f}")
    sweep_table("Thermal state, N = 12, beta = 3", n, 3.0, eth, ks)

    K = 2704156
    ns = [12, 20, 28, 36, 44] if args.quick else list(range(12, 52, 2))
    print(f"\n### Fixed cap K = {K}, tau = 20\n")
    print("| N | energy per site | exact | relative error | cap reached | seconds |")
    print("|---:|---:|---:|---:|---|---:|")
    for N in ns:
        [r] = X.fixed_k_size_scan(ns=[N], K=K)
        E = r["energy_per_site"][-1]
        ref = FF.ground_energy(N, J, H, False) / N
        print(f"| {N} | {E:.10f} | {ref:.10f} | {rel(E, ref):.3e} | {'yes' if r['cap_hit'] else 'no'} | "
              f"{r['seconds']:.2f} |", flush=True)
        log(f"fixed K: N = {N} done")

    betas = [0.08, 0.24, 0.8]
    Ks = [1 << k for k in range(9, 25, 2 if args.quick else 1)]
    ns = [8, 16, 24, 32] if args.quick else [8, 12, 16, 20, 24, 32, 40, 48]
    print("\n### K(N, eps0 = 1e-2): smallest cap with relative energy error <= 1e-2\n")
    print("| N | beta = 0.08 | beta = 0.24 | beta = 0.8 |")
    print("|---:|---:|---:|---:|")
    for N in ns:
        runs = X.k_scan(N, betas, Ks)
        cells = []
        for beta in betas:
            k = X.min_k_for_error(runs, beta, FF.thermal_energy(N, J, H, beta, False) / N, 1e-2)
            cells.append(f"2^{k.bit_length() - 1}" if k else f"> 2^{Ks[-1].bit_length() - 1}")
        print(f"| {N} | " + " | ".join(cells) + " |", flush=True)
        log(f"K scan: N = {N} done")

    print("\n### Readings of the ground-state count at threshold 2^-7 (N = 12, 500 steps)\n")
    print("| order | gate angle | boundary | strings at the end | energy |")
    print("|---|---|---|---:|---:|")
    for order in (1, 2):
        for scale in (1, 2):
            for periodic in (False, True):
                r = X.tfim_run(12, J, H, DTAU * scale, 500 * DTAU * scale, 2.0 ** -7, 1 << 23, periodic, order,
                               record_betas=[500 * DTAU * scale])
                angle = "h dtau (Algorithm 1)" if scale == 1 else "2 h dtau (beta = 2 tau)"
                print(f"| {'first' if order == 1 else 'Strang'} | {angle} | {'periodic' if periodic else 'open'} | "
                      f"{r['n_terms'][-1]} | {12 * r['energy_per_site'][-1]:.3f} |", flush=True)
    log("readings done")


if __name__ == "__main__":
    main()
