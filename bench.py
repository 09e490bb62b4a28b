#!/usr/bin/env python
"""Benchmark of the generalized-Neumann-kernel solver on one MI355X.

One step = the whole hot path on the 17-component bounded workload (unit
circle + 16 seeded ellipses, n = 1024 nodes per component, N = 17408
unknowns, A = eta, gamma = -log|eta|): FBIE (right-hand side y, GMRES solve of
(2I + diag(B1) - B) mu = -y to relative residual 1e-12, and h) followed by
FBIEad (GMRES solve of (diag(e) + B^T + Phat) mu = gamma), all on the GPU with
the inputs resident in HBM.

value = Cauchy pair evaluations per second over the step (pair x column,
        counted from the launches the library actually made), in Gpair/s.
roofline = the dominant kernel (single-column FP64 Cauchy sum), timed with
        HIP events on the stream it runs on, against the FP64 vector peak.
cpu_baseline = the CPU oracle's pair evaluation (dense kernel-matrix rows)
        on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N/M matvec Gpair/s (% FP64 peak) + solve time to 1e-10, mixed/batched vs plain"
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, AMD public figure
FLOPS_PER_PAIR = 16.0            # one column: 2 sub, |d|^2 (3), reciprocal (1), q (2), complex FMA (8)


def cpu_baseline(dom, budget_s=10.0):
    """Oracle kernel-matrix rows (complex FP64, NumPy) of the same workload."""
    import numpy as np
    from oracle import nystrom as orc
    rng = np.random.default_rng(0)
    x = rng.normal(size=dom.N)
    block = 512
    pairs = 0
    rows_done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and rows_done < dom.N:
        sl = slice(rows_done, min(dom.N, rows_done + block))
        K = orc.kernel_rows(dom.eta, dom.etap, dom.A, dom.n, sl)
        _ = K.imag @ x
        pairs += K.shape[0] * dom.N
        rows_done += K.shape[0]
    dt = time.perf_counter() - t0
    return {"value": round(pairs / dt / 1e9, 5), "unit": "Gpair/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle kernel rows 0..{rows_done} x {dom.N} sources of the N={dom.N} workload "
                      f"(K_ij assembly + one product), {dt:.1f} s, NumPy single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the solver has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl
    from paper_1308_5351_amd import gnk

    dom, gam = wl.config1()
    ctx = gnk.Context(0)
    dd = gnk.DeviceDomain.from_host(dom, "cuda:0")
    g = torch.from_numpy(gam[:, 0].copy()).to("cuda:0")
    opts = dict(restart=25, maxit=40, tol=1e-12)

    def step():
        mu, h, inf, st = ctx.fbie(dd, g, **opts)
        mua, infa, sta = ctx.fbie_ad(dd, g, **opts)
        if st != 0 or sta != 0:
            raise RuntimeError(f"solve did not converge: {inf} {infa}")
        return inf[0], infa[0]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    # per-phase solve times (one extra pair of solves, outside the timed region)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)

    ta = time.perf_counter()
    ctx.fbie(dd, g, **opts)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ctx.fbie_ad(dd, g, **opts)
    torch.cuda.synchronize()
    tc = time.perf_counter()

    ms_step = (t1 - t0) * 1e3 / args.steps
    value = prof["pair_cols"] / (t1 - t0) / 1e9
    pairs1 = prof["pairs1"] / max(1, prof["launches1"])
    avg1_ms = prof["ms1"] / max(1, prof["launches1"])
    achieved = FLOPS_PER_PAIR * pairs1 / (avg1_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bounded 17-component domain: unit circle + 16 seeded ellipses, n=1024, "
                               "N=17408, A=eta, gamma=-log|eta|; step = FBIE (mu, h) + FBIEad, GMRES "
                               "restart 25, tol 1e-12",
                   "N": dom.N, "m1": dom.m1, "n": dom.n, "precision": "fp64"},
        "matvec": {"kernel": "k_cauchy_fp64<1>", "avg_ms": round(avg1_ms, 5),
                   "gpair_s": round(pairs1 / (avg1_ms * 1e-3) / 1e9, 2),
                   "frac_fp64_peak": round(achieved / FP64_PEAK_TFLOPS, 4),
                   "launches_per_step": prof["launches"] / args.steps},
        "solve_ms": {"fbie": round((tb - ta) * 1e3, 3), "fbie_ad": round((tc - tb) * 1e3, 3)},
        "gmres_iters": {"fbie": infos[-1][0]["inner_it"], "fbie_ad": infos[-1][1]["inner_it"]},
        "true_relres": {"fbie": infos[-1][0]["true_relres"], "fbie_ad": infos[-1][1]["true_relres"]},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dom)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
