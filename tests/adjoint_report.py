"""Report of the adjoint form at the adjoint benchmark's size (not a test).

Model: 1D TFIM, n = 64 periodic, J = h = 1, first-order Trotter, dtau = 0.02,
beta = 1.5 (75 steps), threshold 1e-6, cap K = 2^24, FP64, forward
checkpoints every 10 Trotter steps.  On one GPU it measures
- the plain forward, the checkpointed forward and the reverse sweeps
  (one seeded with H, one with M_x = sum_i X_i) and their times;
- d<H>/dJ, d<H>/dh, d<H>/dbeta and d<M_x>/dh from the reverse sweep
  (truncation support held fixed), and the specific heat
  C = -beta^2 d<H>/dbeta;
- the same derivatives by central finite differences (step 1e-5) of whole
  GPU runs, each truncating anew (so the kept sets differ between the runs);
- the free-fermion values (exact thermal state of the periodic chain with
  the parity projection) of <H> and its derivatives, the derivatives by
  central differences of the closed form.
ITPP at this cap is far from the exact thermal state (the string budget
is exhausted long before beta = 1.5), so the free-fermion columns measure
the method's truncation error, not the implementation.

Usage (from the repository root, on a GPU):
    python tests/adjoint_report.py [K] > profiles/adjoint_form_tfim_n64_periodic_K2e24.md
"""
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

import itpp_workloads as W  # noqa: E402
import paper_2601_14400_amd as P  # noqa: E402
from oracle import freefermion as FF  # noqa: E402

EPS = 1e-5


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(K, J=1.0, h=1.0, beta=1.5):
    w = W.tfim_workload("c5", 64, J, h, True, 1, 0.02, 1.5, 1e-6, K)
    # beta = N dtau with the step count N = 75 fixed
    return dataclasses.replace(w, dtau=beta / w.n_steps)


def forward(w, every=0):
    e = P.engine_for(w)
    if every:
        e.set_adjoint(every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = e.evolve(w.dtau, w.n_steps)
    torch.cuda.synchronize()
    return e, st, time.perf_counter() - t0


def energy_and_mx(e, w):
    n = w.n
    E = e.expect(w.strings, w.alphas)
    Mx = e.expect(w.strings[n:], [1.0] * n)
    return E, Mx


def main():
    K = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 24
    torch.cuda.set_device(0)
    w = workload(K)
    n, N, beta = w.n, w.n_steps, 1.5
    zz_idx, x_idx = range(n), range(n, 2 * n)
    e, st, t_plain = forward(w)
    E0, M0 = energy_and_mx(e, w)
    e.close()
    log(f"plain forward {t_plain:.2f} s, E = {E0}")
    e, st_ck, t_ck = forward(w, every=10)
    log(f"checkpointed forward {t_ck:.2f} s")
    t0 = time.perf_counter()
    LH, daH, ddH, _ = e.backward(w.strings, w.alphas)
    torch.cuda.synchronize()
    t_bH = time.perf_counter() - t0
    log(f"reverse sweep <H> {t_bH:.2f} s")
    t0 = time.perf_counter()
    LM, daM, ddM, _ = e.backward(w.strings[n:], [1.0] * n)
    torch.cuda.synchronize()
    t_bM = time.perf_counter() - t0
    log(f"reverse sweep M_x {t_bM:.2f} s")
    zz = sum(e.expect([w.strings[k]], [1.0]) for k in zz_idx)
    xx = sum(e.expect([w.strings[k]], [1.0]) for k in x_idx)
    e.close()
    adj = {
        # alpha_ZZ = -J, alpha_X = -h; explicit parts -<sum ZZ>, -<sum X>
        "dE_dJ": -zz - float(sum(daH[k] for k in zz_idx)),
        "dE_dh": -xx - float(sum(daH[k] for k in x_idx)),
        "dE_dbeta": ddH / N,
        "dMx_dh": -float(sum(daM[k] for k in x_idx)),
        "dMx_dJ": -float(sum(daM[k] for k in zz_idx)),
        "dMx_dbeta": ddM / N,
    }
    # central differences of whole runs (each run truncates anew)
    fd = {}
    for name, kw in (("J", "J"), ("h", "h"), ("beta", "beta")):
        vals = []
        for s in (+1, -1):
            args = {"J": 1.0, "h": 1.0, "beta": beta}
            args[kw] += s * EPS
            ww = workload(K, **args)
            ee, _, _ = forward(ww)
            vals.append(energy_and_mx(ee, ww))
            ee.close()
        fd[f"dE_d{name}"] = (vals[0][0] - vals[1][0]) / (2 * EPS)
        fd[f"dMx_d{name}"] = (vals[0][1] - vals[1][1]) / (2 * EPS)
        log(f"finite differences in {name} done")
    # free fermions (closed form), derivatives by central differences of it
    def ff(J=1.0, h=1.0, b=beta):
        return FF.thermal_energy(n, J, h, b, True)

    ffd = {"E": ff(),
           "dE_dJ": (ff(J=1 + EPS) - ff(J=1 - EPS)) / (2 * EPS),
           "dE_dh": (ff(h=1 + EPS) - ff(h=1 - EPS)) / (2 * EPS),
           "dE_dbeta": (ff(b=beta + EPS) - ff(b=beta - EPS)) / (2 * EPS)}
    rows = [("d<H>/dJ", adj["dE_dJ"], fd["dE_dJ"], ffd["dE_dJ"]),
            ("d<H>/dh", adj["dE_dh"], fd["dE_dh"], ffd["dE_dh"]),
            ("d<H>/dbeta", adj["dE_dbeta"], fd["dE_dbeta"], ffd["dE_dbeta"]),
            ("d<M_x>/dh (transverse susceptibility)", adj["dMx_dh"], fd["dMx_dh"], None),
            ("d<M_x>/dJ", adj["dMx_dJ"], fd["dMx_dJ"], None),
            ("d<M_x>/dbeta", adj["dMx_dbeta"], fd["dMx_dbeta"], None)]
    out = []
    out.append("# Adjoint form: TFIM n = 64 periodic, K = 2^24 (derivatives, checks, timing)\n")
    out.append("Command (repository root, one MI355X, after `python -c \"import __graft_entry__ as g; g.build()\"`):\n")
    out.append(f"```\npython tests/adjoint_report.py {K}\n```\n")
    out.append("Model: H = -J sum Z_i Z_{i+1} - h sum X_i, n = 64 periodic, J = h = 1, first-order Trotter, "
               f"dtau = 0.02, beta = 1.5 (75 steps, 9600 gates), threshold 1e-6, cap K = {K}, FP64, "
               "forward checkpoints every 10 Trotter steps.  beta varies with the step count fixed (dtau = beta / 75).\n")
    out.append("| quantity | reverse sweep (support fixed) | central differences, eps = 1e-5 (re-truncated) | "
               "difference | free fermions (exact thermal state) |")
    out.append("|---|---:|---:|---:|---:|")
    for name, a, f, x in rows:
        xs = f"{x:.6f}" if x is not None else "-"
        out.append(f"| {name} | {a:.6f} | {f:.6f} | {a - f:.2e} | {xs} |")
    C_adj, C_ff = -beta ** 2 * adj["dE_dbeta"], -beta ** 2 * ffd["dE_dbeta"]
    out.append("")
    out.append(f"<H> = {E0:.6f} (ITPP) against {ffd['E']:.6f} (free fermions); <M_x> = {M0:.6f}.  "
               f"Specific heat C = -beta^2 d<H>/dbeta = {C_adj:.6f} (reverse sweep), {C_ff:.6f} (free fermions); "
               f"per site {C_adj / n:.6f} and {C_ff / n:.6f}.\n")
    out.append(f"The reverse sweep and the observables agree: L = {LH:.12f} for <H> and {LM:.12f} for <M_x>, "
               f"equal to the forward readouts {E0:.12f} and {M0:.12f}.\n")
    out.append("| run | seconds |\n|---|---:|")
    out.append(f"| plain forward (speculation on) | {t_plain:.2f} |")
    out.append(f"| forward with checkpoints (no speculation) | {t_ck:.2f} |")
    out.append(f"| reverse sweep of <H> | {t_bH:.2f} |")
    out.append(f"| reverse sweep of <M_x> | {t_bM:.2f} |")
    out.append(f"\nReverse sweep over plain forward: {t_bH / t_plain:.2f}; checkpointed forward plus reverse sweep "
               f"over plain forward: {(t_ck + t_bH) / t_plain:.2f}.\n")
    out.append("The differences between the reverse sweep and the central differences are the derivative of "
               "the truncation itself: each finite-difference run keeps its own set of strings, while the "
               "reverse sweep differentiates the map with the kept sets of the base run (frozen support; "
               "the frozen-support derivatives are checked against the reverse-mode oracle in "
               "`tests/test_gpu_adjoint.py`).  The free-fermion columns are the exact thermal state: at this "
               "cap ITPP's <H> is far from it (the truncation error of Sec. III), so these columns are an "
               "accuracy report, not a check of the implementation.\n")
    out.append("```\n" + json.dumps({"adjoint": adj, "finite_differences": fd, "free_fermions": ffd,
                                     "E": E0, "Mx": M0, "times_s": {"plain": t_plain, "checkpointed": t_ck,
                                                                  "reverse_H": t_bH, "reverse_Mx": t_bM}}) + "\n```")
    print("\n".join(out))


if __name__ == "__main__":
    main()
