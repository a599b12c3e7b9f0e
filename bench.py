#!/usr/bin/env python3
"""Benchmark of the chiral rank-k multigrid hot path on one MI355X.

Workload (anisotropic 16^3x32 lattice, xi = 3.5): smoothed random SU(3) links
exp(i 0.2 H) + 3 APE-like projections, m0 placed just above the critical mass
found by the oracle (tests/golden/m0_tuned.json), m' = 48 test vectors with 60 MR
sweeps in FP32, 4^4 blocks, chiral SVD truncation to k = 24 per chirality
(FP64), Galerkin coarse operator (FP64), then an MG-preconditioned GCR solve of
10 Gaussian right-hand sides to a true relative residual of 1e-10 (FP64 outer
GCR, FP32 K-cycle with 8 MR post-smoothing steps).

One step = one full setup + one 10-RHS solve, inputs resident in device memory.
The JSON line reports the MG setup seconds (value), the dslash HBM bandwidth
of the smoother's launches, solve throughput and latency percentiles, the same
workload in the plain FP64 form, the kernel's roofline position and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

DIMS = [16, 16, 16, 32]
XI, EPS, N_APE, CONFIG = 3.5, 0.2, 3, 2
M_PRIME, K, BLOCK, N_SMOOTH, NRHS = 48, 24, [4, 4, 4, 4], 60, 10
SOLVE = dict(nu_post=8, tau=0.1, restart=16, max_iter=500)
HBM_PEAK_GBPS = 8000.0
METRIC = "MG setup s & dslash GB/s; solves/s, p50/p99 at 1e-10 vs plain FP64 form"


def tuned_m0():
    path = os.path.join(ROOT, "tests", "golden", "m0_tuned.json")
    with open(path) as f:
        return float(json.load(f)["ensembles"]["aniso_xi3.5_eps0.2"]["m0"])


def dslash_bytes(V, nrhs, form):
    """Algorithmic HBM bytes of one multi-RHS dslash launch: every input spinor read
    once, every output written once, every link read once."""
    spinor = {0: 192, 1: 96, 2: 52}[form]       # 12 complex, FP64 / FP32 / FP16+scale
    link = {0: 576, 1: 288, 2: 144}[form]       # 4 forward links + 4 backward links per site, 9 complex each
    return V * (2 * spinor * nrhs + link)


def cpu_baseline(U, m0, V):
    """Time the oracle on a bounded sample of one setup and scale to a full setup."""
    from oracle import chiral, galerkin, mr
    from oracle.wilson import WilsonOp
    op = WilsonOp(U, DIMS, m0, XI)
    v = synth.gaussian_vectors(M_PRIME, V, 12, config=CONFIG, level=0)
    cols = np.ascontiguousarray(np.transpose(v, (1, 2, 0)))
    t0 = time.perf_counter()
    q = op.apply(cols)                                  # one sweep's operator application, all 48 vectors
    a = mr.cdot(q, cols) / mr.cdot(q, q).real
    cols = cols + a * cols
    t_sweep = time.perf_counter() - t0
    psi = mr.normalize_columns(cols)
    A = chiral.chiral_blocks(psi, DIMS, BLOCK)
    nsvd = 16
    t0 = time.perf_counter()
    Pb, _ = chiral.prolongator_blocks(A[:nsvd // 2], K)  # 16 (block, chirality) SVDs
    t_svd = (time.perf_counter() - t0) / nsvd
    Pfull = np.zeros((A.shape[0], 2, A.shape[2], K), dtype=np.complex128)
    Pfull[:nsvd // 2] = Pb
    t0 = time.perf_counter()
    galerkin.galerkin(op, Pfull, BLOCK, blocks=[0])      # one coarse site
    t_gal = time.perf_counter() - t0
    nblocks = A.shape[0]
    est = (N_SMOOTH + 1) * t_sweep + 2 * nblocks * t_svd + nblocks * t_gal
    sample = (f"oracle FP64: 1 of {N_SMOOTH + 1} smoother operator passes over all {M_PRIME} vectors, "
              f"{nsvd} of {2 * nblocks} block SVDs, 1 of {nblocks} Galerkin coarse sites; "
              f"scaled to one full setup")
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle", "sample": sample,
            "sample_seconds": t_sweep + nsvd * t_svd + t_gal,
            "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU domain "
                                   "decomposition is a design (DESIGN.md) and is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2502_03091_amd as crk

    dev = torch.device("cuda", 0)
    V = int(np.prod(DIMS))
    m0 = tuned_m0()
    U = synth.gauge_field(DIMS, EPS, N_APE, config=CONFIG)
    lat = crk.Lattice(DIMS, m0, XI)
    lat.load_gauge(U)
    b_host = synth.gaussian_rhs(NRHS, V, config=CONFIG)
    b = torch.from_numpy(b_host.view(np.float64)).to(dev)
    x = torch.empty_like(b)
    torch.cuda.synchronize()

    def step(setup_form, solve_form, m_prime=M_PRIME, k=K):
        t0 = time.perf_counter()
        H = crk.Hierarchy(lat, m_prime=[m_prime], k=[k], block=[BLOCK], n_smooth=[N_SMOOTH],
                          setup_form=setup_form, seed=0x2502030910)
        t1 = time.perf_counter()
        info = H.solve_dev(b, x, NRHS, form=solve_form, raise_on_noconv=False, **SOLVE)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tim = H.timing(0)
        H.close()
        return t1 - t0, t2 - t1, info, tim

    for _ in range(args.warmup):
        step(crk.FORM_FP32, crk.FORM_FP32)

    torch.cuda.synchronize()
    setups, solves, infos, tims = [], [], [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        s, v, info, tim = step(crk.FORM_FP32, crk.FORM_FP32)
        setups.append(s)
        solves.append(v)
        infos.append(info)
        tims.append(tim)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start

    dslash_avg = float(np.mean([t["dslash_avg"] for t in tims]))
    alg = dslash_bytes(V, M_PRIME, 1)
    achieved = alg / dslash_avg / 1e9
    result = {
        "metric": METRIC,
        "value": float(np.mean(setups)),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "16^3x32 xi=3.5 smoothed random SU(3) (eps=0.2, 3 APE), m0 = m_c + 0.01 "
                        "(oracle-located critical mass); chiral rank-k setup m'=48 -> k=24, 4^4 blocks, "
                        "60 FP32 MR sweeps, FP64 SVD+Galerkin; two-level MG-GCR solve of 10 RHS to 1e-10 "
                        "(FP32 K-cycle, FP64 outer GCR)",
            "m0": m0, "global_batch": NRHS, "lattice": DIMS, "parallelism": "none (1 GPU)",
        },
        "setup_s": float(np.mean(setups)),
        "setup_device_s": float(np.mean([t["total"] for t in tims])),
        "setup_stages_s": {k_: float(np.mean([t[k_] for t in tims])) for k_ in ("smoother", "svd", "galerkin")},
        "dslash_GBps": achieved,
        "dslash_launch_ms": 1e3 * dslash_avg,
        "solve_s": float(np.mean(solves)),
        "solves_per_s": NRHS / float(np.mean(solves)),
        "solve_p50_s": float(np.percentile(solves, 50)),
        "solve_p99_s": float(np.percentile(solves, 99)),
        "solve_iters": infos[-1]["iters"],
        "solve_level_iters": infos[-1]["level_iters"],
        "true_rel_resid": max(i["true_rel_resid"] for i in infos),
        "converged": all(i["converged"] for i in infos),
        "roofline": {
            "kernel": "wilson_kernel<FP32, 4 RHS/thread> (48 RHS, 16^3x32)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
            "algorithmic_bytes_per_launch": alg,
        },
    }
    if not args.no_fp64:
        s, v, info, tim = step(crk.FORM_FP64, crk.FORM_FP64)
        result["fp64_plain"] = {"setup_s": s, "solve_s": v, "solves_per_s": NRHS / v, "iters": info["iters"],
                                "level_iters": info["level_iters"], "true_rel_resid": info["true_rel_resid"],
                                "converged": info["converged"],
                                "dslash_GBps": dslash_bytes(V, M_PRIME, 0) / tim["dslash_avg"] / 1e9}
        s, v, info, tim = step(crk.FORM_FP32, crk.FORM_FP32, m_prime=K, k=K)
        result["conventional_m24"] = {"setup_s": s, "solve_s": v, "iters": info["iters"],
                                      "level_iters": info["level_iters"], "true_rel_resid": info["true_rel_resid"],
                                      "converged": info["converged"]}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(U, m0, V)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
