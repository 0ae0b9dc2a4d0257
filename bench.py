"""Benchmark of the ITPP layer update on one MI355X.

A step is one pass of the whole hot path on the benchmark workload: reset to
rho = I, all Trotter steps of the schedule (every elementary gate with its
merge, truncation and normalisation), and the observables read from the
final state.  The workload is the n=64 open TFIM chain, h ~ U[0.5, 1.5]
(seed 0), second-order Trotter with dtau = 0.02 to beta = 2 (100 steps,
19,000 gates), threshold 1e-6 and cap 2^24, FP64 coefficients.

Printed metric: Pauli-term updates per second (one update = one string
entering one elementary gate, summed over all gates of the step).  The
roofline object reports the gate kernel's algorithmic bytes per launch
((strings in + strings out) * 24 B) over its average launch time, measured
with HIP events on the engine's stream; the CPU baseline is the plain C++
dictionary oracle on a bounded prefix of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--K", type=int, default=1 << 24, help="term cap (default 2^24)")
    ap.add_argument("--beta", type=float, default=2.0, help="final inverse temperature (default 2)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(w, budget_s: float):
    """The C++ dictionary oracle, single-threaded, on the first Trotter steps
    of the same workload until the time budget is used."""
    from oracle import c_oracle

    c_oracle.build(force=False)
    o = c_oracle.COracle(w.n)
    t0 = time.perf_counter()
    steps = 0
    while steps < w.n_steps and time.perf_counter() - t0 < budget_s:
        o.evolve(w.strings, w.alphas, w.schedule, w.dtau, 1, w.delta, w.K)
        steps += 1
    dt = time.perf_counter() - t0
    tu = o.term_updates()
    return {"value": tu / dt, "unit": "term-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"C++ dict oracle, Trotter steps 1-{steps} of the same workload "
                      f"({tu:.3e} term updates in {dt:.1f} s, {o.size()} strings at the end); "
                      f"host {platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()}"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this engine runs one state on one GPU; multi-GPU runs are not part of it "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    torch.cuda.set_device(0)
    w = W.config2(K=args.K, beta=args.beta)
    eng = P.engine_for(w)
    obs = w.observables

    def one_step():
        eng.reset()
        st = eng.evolve(w.dtau, w.n_steps)
        vals = {k: eng.expect(s, c) for k, (s, c) in obs.items() if k in ("energy_per_site", "Z0Z1", "Z0Z8")}
        return st, vals

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    eng.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_updates = 0.0
    last = None
    for _ in range(args.steps):
        st, vals = one_step()
        tot_updates += st["term_updates"]
        last = (st, vals)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = eng.timing()
    eng.set_timing(False)
    launches = max(1, tim["gate_launches"])
    avg_ms = tim["gate_ms"] / launches
    bytes_per_launch = tim["alg_bytes"] / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    st, vals = last
    out = {
        "metric": "pauli_term_updates_per_sec",
        "value": tot_updates / dt,
        "unit": "term-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"tfim_n{w.n}_open_strang_dtau{w.dtau}_beta{args.beta}_delta1e-6_K{args.K}",
                   "n_qubits": w.n, "K": args.K, "delta": w.delta, "dtau": w.dtau,
                   "trotter_steps": w.n_steps, "gates_per_step": st["n_gates"],
                   "h": w.meta["h"], "seed": w.meta["seed"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "gate_kernel", "avg_launch_ms": avg_ms,
                     "alg_bytes_per_launch": bytes_per_launch, "launches": tim["gate_launches"]},
        "detail": {"term_updates_per_step": st["term_updates"], "final_terms": st["n_terms"],
                   "gate_ms_total": tim["gate_ms"], "select_ms_total": tim["select_ms"],
                   "observables": vals},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
