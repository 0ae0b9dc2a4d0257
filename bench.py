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

--form selects one of the method's forms instead, each against the plain
FP64 form on the same GPU (one step = one whole run of its workload):
  fp32     n=128 periodic TFIM, dtau 0.01, beta 1, threshold 1e-7, cap 2^27,
           binary32 coefficients; error of every observable vs FP64;
  batched  64 periodic TFIM instances (n in {16..128}, h, beta drawn from
           seed 1), cap 2^20 each: one batch vs a loop of single runs;
  adjoint  n=64 periodic TFIM, beta 1.5, cap 2^24: forward with checkpoints
           every 10 Trotter steps plus the reverse sweep of <H>, vs the plain
           forward; d<H>/dJ, d<H>/dh, d<H>/dbeta;
  squared  the benchmark chain at cap 2^20 after beta = 2: <H>/n and <Z0 Z1>
           at 2 beta from the squared state (Tr[(O rho) rho] / Tr[rho^2]),
           in stored strings x observable strings per second;
  realtime a synthetic state of 2^24 strings on the benchmark chain, one
           Trotter step of real-time gates (Sec. II.B rule), cap 2^24.
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
# the sources the gate kernel is built from (its traffic record is keyed by them)
KERNEL_SOURCES = ("paper_2601_14400_amd/csrc/itpp_gate.hip", "paper_2601_14400_amd/csrc/itpp_device.h",
                  "paper_2601_14400_amd/csrc/itpp_internal.h")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "gate_kernel_traffic_tfim_n64_open_K2e24.json")
COPY_BYTES = 256 << 20



# Every form but the small state runs the 512-thread gate kernel (gate shape
# 1) at every state size: it is the kernel their roofline and rocprofv3
# summaries cover.  The library's automatic default would run gates on states
# of at most 2^19 strings on the layer kernel instead (faster there).
GATE_SHAPE = 1

def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per gate-kernel launch from the committed counter record, if
    it was taken on the current kernel source (else None)."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return rec


def summarize_pmc(fetch_csv: str, write_csv: str):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the gate kernel, each
    scaled by bytes / counter of the device copies of known size."""
    import csv

    def read(path):
        rows = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                d = int(r["Dispatch_Id"])
                rows.setdefault(d, [r["Kernel_Name"], 0.0])
                rows[d][1] += float(r["Counter_Value"])
        return rows

    out = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = read(path)
        items = sorted(rows.items())
        gate_ids = [d for d, (k, _) in items if "gate_kernel" in k and "true" not in k]
        # a gate redone after a failed speculation leaves the rest of its
        # host batch as launches that return at once: they read and write
        # (almost) nothing and are not gates, so the bytes of every launch
        # are summed and divided by the launches that did work
        vals = sorted(rows[d][1] for d in gate_ids)
        floor = 0.01 * vals[len(vals) // 2] if vals else 0.0
        gate = [rows[d][1] for d in gate_ids]
        worked = sum(1 for v in gate if v > floor)
        # the copy dispatches after the last gate launch are the calibration:
        # three copies of COPY_BYTES
        tail = [v for d, (k, v) in items if "copyBuffer" in k and d > gate_ids[-1]]
        per_copy_kib = sum(tail) / 3.0
        factor = (COPY_BYTES / 1024.0) / per_copy_kib
        out[name] = {"launches": worked, "empty_launches": len(gate) - worked,
                     "mean_kib_per_launch": sum(gate) / max(1, worked),
                     "copy_kib_per_256MiB": per_copy_kib, "factor": factor}
    bpl = (out["fetch"]["mean_kib_per_launch"] * out["fetch"]["factor"] +
           out["write"]["mean_kib_per_launch"] * out["write"]["factor"]) * 1024.0
    rec = {"kernel": "gate_kernel", "workload": "tfim_n64_open_strang_dtau0.02_beta2.0_delta1e-6_K16777216",
           "kernel_source_sha256": kernel_source_hash(), "bytes_per_launch": bpl, "counters": out,
           "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- "
                        "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --calibration-copy --progress",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- "
                        "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --calibration-copy --progress"]}
    with open(TRAFFIC_RECORD, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 2; 1 for --form)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 1; 0 for --form)")
    ap.add_argument("--K", type=int, default=1 << 24, help="term cap (default 2^24)")
    ap.add_argument("--beta", type=float, default=2.0, help="final inverse temperature (default 2)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", choices=["fp64", "fp32", "batched", "adjoint", "squared", "realtime", "small"],
                    default="fp64")
    ap.add_argument("--progress", action="store_true", help="print a line after every tenth of the Trotter steps")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with three 256 MiB device copies (the byte counters' calibration in a --pmc run)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn the counter_collection.csv of a FETCH_SIZE and a WRITE_SIZE run of this "
                         "benchmark (with --calibration-copy) into the traffic record under profiles/")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 2 if args.form == "fp64" else 1
    if args.warmup is None:
        args.warmup = 1 if args.form == "fp64" else 0
    return args


def cpu_baseline(w, budget_s: float):
    """The C++ dictionary oracle, single-threaded, gate by gate from rho = I
    along the same workload until the time budget is used."""
    from oracle import c_oracle

    c_oracle.build(force=False)
    o = c_oracle.COracle(w.n, w.precision)
    t0 = time.perf_counter()
    gates = 0
    total = w.n_steps * len(w.schedule)
    while gates < total and time.perf_counter() - t0 < budget_s:
        k, m = w.schedule[gates % len(w.schedule)]
        o.evolve(w.strings, w.alphas, [(k, m)], w.dtau, 1, w.delta, w.K)
        gates += 1
    dt = time.perf_counter() - t0
    tu = o.term_updates()
    return {"value": tu / dt, "unit": "term-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"C++ dict oracle, the first {gates} elementary gates of the same workload from rho = I "
                      f"({tu:.3e} term updates in {dt:.1f} s, {o.size()} strings at the end); "
                      f"host {platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()}"}


def roofline_of(tim, peak=HBM_PEAK_GBS):
    launches = max(1, tim["gate_launches"])
    avg_ms = tim["gate_ms"] / launches
    bpl = tim["alg_bytes"] / launches
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s", "frac": achieved / peak,
            "traffic": None, "kernel": "gate_kernel", "avg_launch_ms": avg_ms, "alg_bytes_per_launch": bpl,
            "launches": tim["gate_launches"]}


_T0 = time.perf_counter()


def progress(msg):
    print(f"[bench {time.perf_counter() - _T0:8.1f}s] {msg}", file=sys.stderr, flush=True)


def base_line(args, metric_value, ms, dtype, config):
    return {"metric": "pauli_term_updates_per_sec", "value": metric_value, "unit": "term-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def run_form_fp32(args):
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    K = args.K if args.K != (1 << 24) else (1 << 27)
    out = {}
    vals = {}
    for prec in ("f32", "f64"):
        w = W.config3(K=K, beta=args.beta if args.beta != 2.0 else 1.0, precision=prec)
        eng = P.engine_for(w)
        eng.set_option("gate_shape", GATE_SHAPE)
        obs = w.observables
        for _ in range(args.warmup):
            eng.reset()
            eng.evolve(w.dtau, w.n_steps)
        torch.cuda.synchronize()
        eng.set_timing(True)
        t0 = time.perf_counter()
        tu = 0.0
        for _ in range(args.steps):
            eng.reset()
            for s in range(w.n_steps):
                st = eng.evolve(w.dtau, 1)
                tu += st["term_updates"]
                if s % 10 == 9:
                    progress(f"{prec} step {s + 1}/{w.n_steps} terms {st['n_terms']}")
            vals[prec] = {k: eng.expect(a, b) for k, (a, b) in obs.items()}
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[prec] = {"value": tu / dt, "ms": dt * 1e3 / args.steps, "roofline": roofline_of(eng.timing()),
                     "final_terms": st["n_terms"], "w": w}
        eng.close()
    w = out["f32"]["w"]
    line = base_line(args, out["f32"]["value"], out["f32"]["ms"], "f32",
                     {"workload": f"tfim_n{w.n}_periodic_first_order_dtau{w.dtau}_beta{w.n_steps * w.dtau:g}"
                                  f"_delta{w.delta:g}_K{K}", "form": "fp32", "n_qubits": w.n, "K": K,
                      "trotter_steps": w.n_steps})
    line["roofline"] = out["f32"]["roofline"]
    line["form"] = {"fp64_value": out["f64"]["value"], "fp32_over_fp64": out["f32"]["value"] / out["f64"]["value"],
                    "fp64_roofline_frac": out["f64"]["roofline"]["frac"],
                    "observables_fp32": vals["f32"], "observables_fp64": vals["f64"],
                    "abs_error_vs_fp64": {k: abs(vals["f32"][k] - vals["f64"][k]) for k in vals["f32"]}}
    return line, w


def run_form_small(args):
    """The 8-qubit untruncated workload (12,870 strings, 16 gates a step,
    320 gates a run): every gate is a chain of small dependent kernels, so
    the wall time is set by launches or by the latency of that chain, not by
    bandwidth.  Whole runs (reset + 20 steps) are timed with step graphs (the
    default) and with one launch per kernel; a separate event-timed run gives
    the kernels' own time, and the line says which of the two bounds it."""
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    w = W.config1()
    reps = 100 * args.steps
    res = {}
    for mode in ("graphs", "direct"):
        eng = P.engine_for(w)
        eng.set_option("graphs", 1 if mode == "graphs" else 0)
        for _ in range(max(1, args.warmup) * 5):
            eng.reset()
            eng.evolve(w.dtau, w.n_steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tu = 0.0
        gsteps = 0
        for _ in range(reps):
            eng.reset()
            st = eng.evolve(w.dtau, w.n_steps)
            tu += st["term_updates"]
            gsteps += st["graph_steps"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[mode] = {"value": tu / dt, "ms_per_run": dt * 1e3 / reps, "us_per_gate": dt * 1e6 / reps / st["n_gates"],
                     "graph_steps_per_run": gsteps / reps, "terms": st["n_terms"]}
        if mode == "graphs":
            vals = {k: eng.expect(a, b) for k, (a, b) in w.observables.items()}
        eng.close()
        progress(f"{mode}: {res[mode]['ms_per_run']:.3f} ms per run")
    eng = P.engine_for(w)
    eng.set_timing(True)
    eng.reset()
    st = eng.evolve(w.dtau, w.n_steps)
    tim = eng.timing()
    eng.close()
    kern_us = (tim["gate_ms"] + tim["select_ms"]) * 1e3 / max(1, tim["gate_launches"])
    line = base_line(args, res["graphs"]["value"], res["graphs"]["ms_per_run"], "f64",
                     {"workload": f"tfim_n{w.n}_periodic_first_order_dtau{w.dtau}_beta{w.n_steps * w.dtau:g}"
                                  f"_delta{w.delta:g}_untruncated", "form": "small", "n_qubits": w.n,
                      "trotter_steps": w.n_steps, "gates_per_run": st["n_gates"], "runs_timed": reps})
    line["roofline"] = roofline_of(tim)
    share = kern_us / res["graphs"]["us_per_gate"]
    # launch-bound if launches and host waits take most of the wall time;
    # otherwise the per-gate chain of small kernels (their latency) does
    line["form"] = {"bound": "launches" if share < 0.5 else "kernel latency", "graphs": res["graphs"],
                    "direct": res["direct"],
                    "graphs_over_direct": res["graphs"]["value"] / res["direct"]["value"],
                    "kernel_us_per_gate": kern_us,
                    "kernel_share_of_wall_graphs": kern_us / res["graphs"]["us_per_gate"],
                    "observables": vals}
    return line, w


def run_form_batched(args):
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    K = args.K if args.K != (1 << 24) else (1 << 20)
    ws = W.config4_instances(seed=1, count=64, K=K)
    dts = [w.dtau for w in ws]
    steps = [w.n_steps for w in ws]
    # single runs, one after another
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tu_seq = 0.0
    for i, w in enumerate(ws):
        e = P.engine_for(w)
        e.set_option("gate_shape", GATE_SHAPE)
        tu_seq += e.evolve(w.dtau, w.n_steps)["term_updates"]
        e.close()
        if i % 8 == 7:
            progress(f"sequential {i + 1}/64")
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    b = P.batch_for(ws)
    progress("autotune: shape pairs, then workers, then grid divisor (200 warm + 100 timed gates per probe)")
    shape, workers, grid_div, rate = b.autotune(dts, 200, 100)
    progress(f"autotune: shapes {shape % 3} (n <= 64) and {shape // 3} (n > 64), workers {workers}, "
             f"grid divisor {grid_div}, probe rate {rate:.3e}")
    for _ in range(args.warmup):
        for e in b.instances:
            e.reset()
        b.evolve(dts, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tu = 0.0
    for _ in range(args.steps):
        for e in b.instances:
            e.reset()
        st = b.evolve(dts, steps)
        tu += sum(x["term_updates"] for x in st)
        progress("batch done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # gate-kernel roofline of one instance of the largest size, timed alone
    big = max(ws, key=lambda w: w.n * w.n_steps)
    progress(f"roofline run: n={big.n}, {big.n_steps} steps")
    e = P.engine_for(big)
    e.set_option("gate_shape", shape // 3 if big.n > 64 else shape % 3)
    e.set_timing(True)
    e.evolve(big.dtau, big.n_steps)
    roof = roofline_of(e.timing())
    e.close()
    line = base_line(args, tu / dt, dt * 1e3 / args.steps, "f64",
                     {"workload": f"tfim_batch64_periodic_n16-128_dtau0.02_delta1e-6_K{K}_seed1", "form": "batched",
                      "instances": 64, "K": K, "gates": int(sum(2 * w.n * w.n_steps for w in ws))})
    line["roofline"] = roof
    line["form"] = {"sequential_value": tu_seq / t_seq, "sequential_s": t_seq, "batched_s": dt / args.steps,
                    "batched_over_sequential": (tu / dt) / (tu_seq / t_seq),
                    "autotune_shape_small": shape % 3, "autotune_shape_large": shape // 3,
                    "autotune_workers": workers, "autotune_grid_div": grid_div}
    return line, big


def run_form_adjoint(args):
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    K = args.K
    w = W.config5(K=K)
    nzz = w.n
    H = (w.strings, w.alphas)
    # plain forward
    e = P.engine_for(w)
    e.set_option("gate_shape", GATE_SHAPE)
    e.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = e.evolve(w.dtau, w.n_steps)
    E_plain = e.expect(*H)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    roof = roofline_of(e.timing())
    e.close()
    progress(f"plain forward {t_fwd:.2f} s")
    # forward with checkpoints + reverse sweep
    e = P.engine_for(w)
    e.set_adjoint(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st2 = e.evolve(w.dtau, w.n_steps)
    torch.cuda.synchronize()
    t_fwd_ck = time.perf_counter() - t0
    progress(f"checkpointed forward {t_fwd_ck:.2f} s")
    t0 = time.perf_counter()
    L, da, dd, _ = e.backward(*H)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    progress(f"reverse sweep {t_bwd:.2f} s")
    zz = sum(e.expect([w.strings[k]], [1.0]) for k in range(nzz))
    xx = sum(e.expect([w.strings[k]], [1.0]) for k in range(nzz, 2 * nzz))
    e.close()
    # the same sweep with checkpoints every step: each segment's states fit
    # in device memory, so every segment is recomputed once instead of twice
    e = P.engine_for(w)
    e.set_adjoint(1)
    e.evolve(w.dtau, w.n_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L1, _, dd1, _ = e.backward(*H)
    torch.cuda.synchronize()
    t_bwd1 = time.perf_counter() - t0
    e.close()
    progress(f"reverse sweep, checkpoints every step {t_bwd1:.2f} s")
    beta = w.dtau * w.n_steps
    dE_dJ = -zz - float(sum(da[:nzz]))
    dE_dh = -xx - float(sum(da[nzz:]))
    dE_db = dd / w.n_steps
    line = base_line(args, st2["term_updates"] / (t_fwd_ck + t_bwd), (t_fwd_ck + t_bwd) * 1e3, "f64",
                     {"workload": f"tfim_n64_periodic_first_order_dtau0.02_beta1.5_delta1e-6_K{K}", "form": "adjoint",
                      "n_qubits": w.n, "K": K, "trotter_steps": w.n_steps, "checkpoint_every_steps": 10})
    line["roofline"] = roof
    line["form"] = {"plain_forward_s": t_fwd, "plain_forward_value": st["term_updates"] / t_fwd,
                    "checkpointed_forward_s": t_fwd_ck, "reverse_sweep_s": t_bwd,
                    "backward_over_forward": t_bwd / t_fwd, "energy": L, "energy_plain_forward": E_plain,
                    "dE_dJ": dE_dJ, "dE_dh": dE_dh, "dE_dbeta": dE_db, "specific_heat": -beta * beta * dE_db,
                    "reverse_sweep_every_step_s": t_bwd1, "backward_over_forward_every_step": t_bwd1 / t_fwd,
                    "every_step_same_result": L1 == L and dd1 == dd}
    return line, w


def run_form_squared(args):
    """Squared-state observables (<O>_{2 beta} from the state at beta) on the
    benchmark chain at a 2^20 cap, after the whole run to beta = 2."""
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    K = 1 << 20
    w = W.config2(K=K)
    e = P.engine_for(w)
    e.set_option("gate_shape", GATE_SHAPE)
    st = e.evolve(w.dtau, w.n_steps)
    torch.cuda.synchronize()
    N = st["n_terms"]
    progress(f"state at beta = 2: {N} strings")
    obs = {k: w.observables[k] for k in ("energy_per_site", "Z0Z1")}
    res = {}
    for name, (strings, coefs) in obs.items():
        best = None
        for _ in range(3):
            t0 = time.perf_counter()
            val, pur = e.expect_squared(strings, coefs)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        res[name] = {"value_at_2beta": val, "purity": pur, "strings": len(strings), "seconds": best,
                     "value_at_beta": e.expect(strings, coefs)}
        progress(f"{name}: {best * 1e3:.1f} ms")
    e.close()
    m = len(obs["energy_per_site"][0])
    t = res["energy_per_site"]["seconds"]
    elem = 16 * ((w.n + 63) // 64) + 8
    alg = N * elem * (1 + m)
    line = base_line(args, N * m / t, t * 1e3, "f64",
                     {"workload": f"tfim_n64_open_strang_dtau0.02_beta2.0_delta1e-6_K{K}_squared_energy",
                      "form": "squared", "n_qubits": w.n, "K": K, "stored_strings": N, "observable_strings": m})
    line["metric"] = "squared_string_pairs_per_sec"
    line["unit"] = "string-pairs/s"
    line["roofline"] = {"bound": "hbm", "achieved": alg / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": alg / t / 1e9 / HBM_PEAK_GBS, "traffic": None, "kernel": "squared_kernel",
                        "alg_bytes": alg}
    line["form"] = res
    return line, w


def run_form_realtime(args):
    """Real-time gates (Sec. II.B rule) on the benchmark chain at cap 2^24:
    a synthetic state of 2^24 strings is loaded, one Trotter step is timed."""
    import torch

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    K = args.K
    w = W.config2(K=K)
    # about 1e6 distinct magnitudes in [2^-19.5, 1): ties at the cap stay small
    x, z, c = W.synthetic_state_words(w.n, K, seed=41, partner=w.strings[w.schedule[0][0]], levels=1 << 20,
                                      step=19.5 / (1 << 20))
    progress("synthetic state generated")
    e = P.engine_for(w)
    e.set_option("gate_shape", GATE_SHAPE)
    e.import_words(x, z, c)
    e.set_option("real_time", 1)
    e.evolve(w.dtau, 1)  # warm-up: one step, so every schedule position has its K-th value ratio
    e.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = e.evolve(w.dtau, 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    roof = roofline_of(e.timing())
    e.close()
    progress(f"one real-time Trotter step: {dt:.3f} s")
    line = base_line(args, st["term_updates"] / dt, dt * 1e3, "f64",
                     {"workload": f"tfim_n64_open_strang_dtau0.02_K{K}_realtime_synthetic_state", "form": "realtime",
                      "n_qubits": w.n, "K": K, "gates": st["n_gates"], "cap_hit": st["cap_hit"]})
    line["roofline"] = roof
    line["form"] = {"term_updates": st["term_updates"], "final_terms": st["n_terms"], "seconds": dt}
    return line, w


def cpu_baseline_realtime(w, budget_s: float):
    """The real-time oracle (pure Python), gate by gate on a synthetic state of
    2^15 strings of the same chain, until the time budget is used."""
    import math as _m

    import itpp_workloads as W
    from oracle import realtime as RT

    x, z, c = W.synthetic_state_words(w.n, 1 << 15, seed=41, partner=w.strings[w.schedule[0][0]])
    from paper_2601_14400_amd import words_to_strings  # marshalling only

    S = dict(zip(words_to_strings(x, z, w.n), c.tolist()))
    t0 = time.perf_counter()
    gates, updates = 0, 0.0
    while time.perf_counter() - t0 < budget_s:
        k, mlt = w.schedule[gates % len(w.schedule)]
        th = w.alphas[k] * mlt * w.dtau
        updates += len(S)
        S = RT.truncate(RT.apply_gate_real(S, w.strings[k], _m.cos(th), _m.sin(th)), w.delta, w.K)
        gates += 1
    dt = time.perf_counter() - t0
    return {"value": updates / dt, "unit": "term-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"Python dict real-time oracle, {gates} gates of the same chain on a synthetic state of "
                      f"{1 << 15} strings ({updates:.3e} term updates in {dt:.1f} s); "
                      f"host {platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()}"}


def cpu_baseline_squared(w, budget_s: float):
    """The oracle's squared-state energy on the C++ oracle's own state after
    the first gates of the same workload, grown until the evaluation covers
    about 8e4 string pairs per second of budget (the pure-Python oracle makes
    about 1e5 pair evaluations per second)."""
    from oracle import c_oracle
    from oracle import squared as SQ

    c_oracle.build(force=False)
    strings, coefs = w.observables["energy_per_site"]
    target = 8e4 * budget_s
    o = c_oracle.COracle(w.n, w.precision)
    gates = 0
    while o.size() * len(strings) < target and gates < len(w.schedule) * w.n_steps:
        k, mlt = w.schedule[gates % len(w.schedule)]
        o.evolve(w.strings, w.alphas, [(k, mlt)], w.dtau, 1, w.delta, w.K)
        gates += 1
    S = o.state()
    t0 = time.perf_counter()
    SQ.squared_expectation(S, strings, coefs)
    dt = time.perf_counter() - t0
    return {"value": len(S) * len(strings) / dt, "unit": "string-pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"Python dict oracle, squared-state energy ({len(strings)} strings) on the C++ oracle's state "
                      f"after the first {gates} gates of the same workload ({len(S)} strings) in {dt:.1f} s; "
                      f"host {platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()}"}


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this engine runs one state on one GPU; multi-GPU runs are not part of it "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.form != "fp64":
        torch.cuda.set_device(0)
        line, w = {"fp32": run_form_fp32, "batched": run_form_batched, "adjoint": run_form_adjoint,
                   "squared": run_form_squared, "realtime": run_form_realtime,
                   "small": run_form_small}[args.form](args)
        if not args.no_cpu_baseline:
            progress("cpu baseline")
            base = {"squared": cpu_baseline_squared, "realtime": cpu_baseline_realtime}.get(args.form, cpu_baseline)
            line["cpu_baseline"] = base(w, args.cpu_seconds)
        print(json.dumps(line), flush=True)
        return

    import itpp_workloads as W
    import paper_2601_14400_amd as P

    torch.cuda.set_device(0)
    w = W.config2(K=args.K, beta=args.beta)
    eng = P.engine_for(w)
    eng.set_option("gate_shape", GATE_SHAPE)
    obs = w.observables

    def one_step():
        eng.reset()
        if args.progress:
            # ten calls of a tenth of the steps, with a line after each
            tot = None
            for k in range(10):
                n = w.n_steps * (k + 1) // 10 - w.n_steps * k // 10
                sk = eng.evolve(w.dtau, n)
                if tot is None:
                    tot = dict(sk)
                else:
                    for key in ("n_gates", "term_updates", "alg_bytes", "spec_gates", "spec_retries", "written"):
                        tot[key] += sk[key]
                    for key in ("n_terms", "c_identity", "cap_hit"):
                        tot[key] = sk[key]
                    tot["c_I_min"] = min(tot["c_I_min"], sk["c_I_min"])
                    tot["c_I_max"] = max(tot["c_I_max"], sk["c_I_max"])
                    tot["kth_abs_min"] = min(tot["kth_abs_min"], sk["kth_abs_min"])
                progress(f"trotter steps {w.n_steps * (k + 1) // 10}/{w.n_steps}")
            st = tot
        else:
            st = eng.evolve(w.dtau, w.n_steps)
        vals = {k: eng.expect(s, c) for k, (s, c) in obs.items() if k == "energy_per_site" or k.startswith("Z0Z")}
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
                   "h": w.meta["h"], "seed": w.meta["seed"], "gate_shape": GATE_SHAPE},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "gate_kernel", "avg_launch_ms": avg_ms,
                     "alg_bytes_per_launch": bytes_per_launch, "launches": tim["gate_launches"]},
        "detail": {"term_updates_per_step": st["term_updates"], "final_terms": st["n_terms"],
                   "gate_ms_total": tim["gate_ms"], "select_ms_total": tim["select_ms"],
                   "spec_gates": st["spec_gates"], "spec_retries": st["spec_retries"],
                   "written_per_gate_over_K": st["written"] / max(1, st["n_gates"]) / args.K,
                   "c_I_range": [st["c_I_min"], st["c_I_max"]], "kth_abs_min": st["kth_abs_min"],
                   "observables": vals},
    }
    rec = measured_traffic()
    if rec is not None and args.K == (1 << 24) and args.beta == 2.0:
        out["roofline"]["traffic"] = rec["bytes_per_launch"]
        out["roofline"]["traffic_over_alg"] = rec["bytes_per_launch"] / bytes_per_launch
        # measured HBM bytes over this run's event-timed launch average
        out["roofline"]["traffic_GBps"] = rec["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        out["roofline"]["traffic_frac"] = out["roofline"]["traffic_GBps"] / HBM_PEAK_GBS
    if args.calibration_copy:
        x = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
