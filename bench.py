"""Benchmark of the Wilson-Dirac hot path on one MI355X.

Workload (the lattice of the paper's CG benchmark is unspecified; this is the
multi-RHS mixed-precision case): 32^3 x 64 lattice, plain Wilson, kappa = 0.12,
periodic space / antiperiodic time, synthetic SU(3) links (seed 0), the 12
spin-colour point sources at the origin.  One step = one solve of
S^H S x_e = b_e for all 12 sources to a 1e-10 FP64 true relative residual,
with FP16-storage CG (FP32 arithmetic, 12-RHS batched hop) inside FP64 defect
correction.  Reported value: effective GB/s of the FP16 12-RHS hop kernel
(algorithmic bytes / HIP-event kernel time over the timed steps); also the
time per source against plain FP64 CG (one source, 18-real links) and the
FP64 CPU oracle on the machine's host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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

METRIC = "Dslash GB/s (% HBM peak); CG time-to-1e-10 residual, mixed/multi-RHS vs FP64"
HBM_PEAK_GBS = 8000.0
DIMS = (32, 32, 32, 64)
KAPPA = 0.12
TOL = 1e-10


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(U, b, budget_s=12.0):
    """The FP64 oracle's full-lattice hop on the same lattice, timed on host cores."""
    import oracle

    from paper_2302_00850_amd.synth import bc_phases
    bc = bc_phases((0, 0, 0, np.pi))
    V = int(np.prod(DIMS))
    oracle.hop(U, b, bc)  # warm (page in)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.hop(U, b, bc)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 20:
            break
    per = el / n
    return {"value": V * 1536 / per / 1e9, "unit": "GB/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} FP64 full-lattice hops D psi on {DIMS[0]}^3x{DIMS[3]} (1 rhs), "
                      f"{per:.3f} s each; bytes counted as the GPU FP64 18-real hop "
                      f"(1536 B per output site)"}


def hop_mode(args):
    """Time the half-lattice hop alone: one JSON line per (precision, nrhs) case."""
    import torch

    from paper_2302_00850_amd import cola
    from paper_2302_00850_amd.synth import Synth, bc_phases

    dims = tuple(int(v) for v in args.lattice.split(","))
    s = Synth(0, device="cuda")
    U = s.gauge(dims)
    bc = bc_phases((0, 0, 0, np.pi))
    for prec in [int(p) for p in args.prec.split(",")]:
        for nrhs in [int(r) for r in args.nrhs.split(",")]:
            lat = cola.Lattice(dims, KAPPA, bc, 0.0, cola.COLA_FLAG_TIMING)
            lat.set_gauge(U)
            if args.tune:
                cola.cola_set_tuning(lat.h, 1)
            psi = s.gaussian_spinor(dims, nrhs)
            pin = lat.pack(psi, prec, 1)
            del psi
            out = lat.empty_packed(prec, nrhs, 0)
            for _ in range(3):
                lat.dslash(out, pin, cola.COLA_OP_HOP, 0, prec, nrhs)
            torch.cuda.synchronize()
            lat.reset_stats()
            t0 = time.perf_counter()
            for _ in range(args.iters):
                lat.dslash(out, pin, cola.COLA_OP_HOP, 0, prec, nrhs)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = lat.stats(prec)
            rec = {"mode": "hop", "lattice": list(dims), "prec": prec, "nrhs": nrhs,
                   "avg_ms": st["hop_seconds"] / st["hop_launches"] * 1e3,
                   "wall_ms": wall / args.iters * 1e3,
                   "GBs": st["hop_bytes"] / st["hop_seconds"] / 1e9,
                   "GFLOPs": st["hop_flops"] / st["hop_seconds"] / 1e9,
                   "bytes_per_site": st["hop_bytes"] / st["hop_launches"] / (np.prod(dims) / 2)}
            rec["frac_hbm"] = rec["GBs"] / HBM_PEAK_GBS
            if args.tune:
                rec["tune"] = cola.cola_tune_dump(lat.h)
            print(json.dumps(rec), flush=True)
            lat.close()
            del pin, out
            torch.cuda.empty_cache()


def copy_mode(args):
    """A plain device-to-device copy of known size (HBM counter calibration)."""
    import torch

    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.iters):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read": n, "bytes_written": n,
                      "copies": args.iters}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--mode", default="solve", choices=["solve", "hop", "copy"])
    ap.add_argument("--lattice", default="32,32,32,64", help="hop mode: Lx,Ly,Lz,Lt")
    ap.add_argument("--prec", default="0,2,3", help="hop mode: precisions (0 FP64 .. 3 FP16)")
    ap.add_argument("--nrhs", default="1,12", help="hop mode: right-hand-side counts")
    ap.add_argument("--iters", type=int, default=20, help="hop mode: timed launches")
    ap.add_argument("--tune", action="store_true", help="hop mode: autotune launch shapes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(domain decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "hop":
        hop_mode(args)
        return
    if args.mode == "copy":
        copy_mode(args)
        return

    import torch

    from paper_2302_00850_amd import cola
    from paper_2302_00850_amd.synth import Synth, bc_phases, point_sources

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    log(f"generating {DIMS} links (seed 0)")
    t0 = time.perf_counter()
    U = Synth(0, device=dev).gauge(DIMS)
    b = point_sources(DIMS, device=dev)
    log(f"fields ready in {time.perf_counter() - t0:.1f} s")
    bc = bc_phases((0, 0, 0, np.pi))
    lat = cola.Lattice(DIMS, KAPPA, bc, 0.0, cola.COLA_FLAG_TIMING)
    lat.set_gauge(U)
    assert lat.gauge_is_su3

    def solve():
        return lat.cg(b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP16_DEFECT, tol=TOL)

    for w in range(args.warmup):
        _, info = solve()
        log(f"warmup {w}: {info['iterations']} inner iterations, {info['outer_cycles']} cycles, "
            f"{info['seconds']:.3f} s, status {info['status']}")
    lat.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        x, info = solve()
        infos.append(info)
        log(f"step {k}: {info['iterations']} it, {info['outer_cycles']} cycles, "
            f"{info['seconds']:.3f} s, max residual {max(info['true_rel_residual']):.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st16 = lat.stats(cola.COLA_FP16)
    st64 = lat.stats(cola.COLA_FP64)
    ms_per_step = wall / args.steps * 1e3
    achieved = st16["hop_bytes"] / st16["hop_seconds"] / 1e9
    per_launch_ms = st16["hop_seconds"] / st16["hop_launches"] * 1e3
    ok = all(i["status"] == cola.COLA_OK for i in infos)

    fp64 = None
    if not args.no_fp64:
        lat64 = cola.Lattice(DIMS, KAPPA, bc, 0.0, cola.COLA_FLAG_TIMING)
        lat64.set_gauge(U)
        b1 = b[:1].clone()
        lat64.cg(b1, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)  # warm
        lat64.reset_stats()
        _, i64 = lat64.cg(b1, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        s64 = lat64.stats(cola.COLA_FP64)
        fp64 = {"seconds_per_source": i64["seconds"], "iterations": i64["iterations"],
                "hop_GBs": s64["hop_bytes"] / s64["hop_seconds"] / 1e9,
                "true_rel_residual": i64["true_rel_residual"][0]}
        log(f"FP64 single-source CG: {i64['iterations']} it, {i64['seconds']:.3f} s")
        lat64.close()

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(U.cpu().numpy(), b[0].cpu().numpy())

    per_source = ms_per_step / 1e3 / 12
    out = {
        "metric": METRIC,
        "value": round(achieved, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32 inner, f64 outer",
        "data": "synthetic",
        "config": {"workload": "wilson_eo_32x32x32x64_12rhs_fp16defect", "lattice": list(DIMS),
                   "kappa": KAPPA, "nrhs": 12, "sources": "point (12 spin-colour at origin)",
                   "solver": "lockstep 12-RHS CG, FP16 storage + FP64 defect correction",
                   "tol": TOL, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "hop_kernel FP16 12-real links, 12 rhs",
                     "bytes_per_launch": st16["hop_bytes"] / max(1, st16["hop_launches"]),
                     "avg_launch_ms": round(per_launch_ms, 4),
                     "launches": st16["hop_launches"]},
        "cg": {"seconds_per_source": per_source, "all_converged": ok,
               "inner_iterations": infos[-1]["iterations"], "outer_cycles": infos[-1]["outer_cycles"],
               "max_true_rel_residual": max(max(i["true_rel_residual"]) for i in infos),
               "fp64_outer_hop_GBs": (st64["hop_bytes"] / st64["hop_seconds"] / 1e9
                                      if st64["hop_seconds"] else None)},
        "fp64_single_rhs": fp64,
        "speedup_per_source_vs_fp64": (fp64["seconds_per_source"] / per_source) if fp64 else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    lat.close()


if __name__ == "__main__":
    main()
