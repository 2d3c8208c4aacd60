"""Benchmark of the Wilson-Dirac hot path on one MI355X.

Workload (the paper's CG benchmark names no lattice; this is the largest synthetic
configuration, at the paper's 32-bit inner / 64-bit outer arithmetic): 48^3 x 96
lattice (10.6M sites), clover-improved Wilson (c_sw = 1, kappa = 0.118), periodic
space / antiperiodic time, synthetic SU(3) links (seed 0), the 12 spin-colour point
sources at the origin.  One step = one solve of S^H S x_e = b_e (S the even-odd
clover Schur complement) for all 12 sources to a 1e-10 FP64 true relative residual,
FP32 CG (FP32 storage and arithmetic, 12-RHS batched hop) inside FP64 defect
correction.  Reported value: effective GB/s of the FP32 12-RHS clover hop
(t_o = A_oo^-1 D_oe p: 2688 B per site for links and spinors plus 288 B of clover
block, algorithmic bytes / HIP-event kernel time over the timed steps); also the
time per source against plain FP64 CG (one source, 18-real links), the blended
GB/s of every FP32 hop launch of the solve, the 32^3 x 64 FP16-storage workload,
and the FP64 CPU oracle's hop on the same lattice on the machine's host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s (% HBM peak); CG time-to-1e-10 residual, mixed/multi-RHS vs FP64"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFS = 78.6  # 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz
DIMS = (48, 48, 48, 96)       # the benchmark workload (clover, FP32 inner / FP64 outer)
KAPPA_C = 0.118
CSW = 1.0
DIMS3 = (32, 32, 32, 64)      # the FP16-storage workload, reported beside it
KAPPA = 0.12
TOL = 1e-10
WORKLOAD = "clover_eo_48x48x48x96_12rhs_fp32defect"


# rocprofv3 counter summary of the FP32 12-rhs clover hop launches of this workload (HBM
# bytes per launch); valid only for the hop sources it was taken with.
COUNTERS = os.path.join(ROOT, "profiles", "hop_fp32_12rhs_clover_48x48x48x96_solve_counters.txt")
HOP_SOURCES = ["hop_impl.h", "device.h", "common.h", "hop_f32_12.hip", "hop_dispatch.cpp",
               "ops.cpp"]


def hop_sources_sha256():
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(os.path.join(ROOT, "paper_2302_00850_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per FP32 clover hop launch (FETCH_SIZE and WRITE_SIZE, each scaled by the
    same counter's reading for a plain copy of known size) from the committed
    summary, or None when there is none or the hop sources changed since."""
    try:
        with open(COUNTERS) as fh:
            kv = dict(l.split(":", 1) for l in fh.read().splitlines()
                      if ":" in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("sources_sha256", "").strip() != hop_sources_sha256():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(U, psi, dims, budget_s=15.0):
    """The FP64 oracle's full-lattice hop D psi on the benchmark lattice, timed on host
    cores (a bounded sample of hops)."""
    import oracle

    from paper_2302_00850_amd.synth import bc_phases
    bc = bc_phases((0, 0, 0, np.pi))
    V = int(np.prod(dims))
    oracle.hop(U, psi, bc)  # warm (page in)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.hop(U, psi, bc)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 20:
            break
    per = el / n
    return {"value": V * 1536 / per / 1e9, "unit": "GB/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} FP64 full-lattice hops D psi on {dims[0]}^3x{dims[3]} (1 rhs), "
                      f"{per:.3f} s each; bytes counted as the GPU FP64 18-real hop "
                      f"(1536 B per output site)"}


def hop_mode(args):
    """Time the half-lattice hop alone: one JSON line per (precision, nrhs) case."""
    import torch

    from paper_2302_00850_amd import cola
    from paper_2302_00850_amd.synth import Synth, bc_phases

    dims = tuple(int(v) for v in args.lattice.split(","))
    # numpy draws on the host for small lattices; the device generator beyond 4M sites
    s = Synth(0, device="cuda", rng="torch" if np.prod(dims) > 4 * 2**20 else "numpy")
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
            for _ in range(max(3, args.iters)):  # warm caches and clocks as long as we time
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


def workloads_mode(args):
    """The other synthetic workloads, one JSON line each (time to a 1e-10 residual etc.)."""
    import torch

    from paper_2302_00850_amd import cola
    from paper_2302_00850_amd.synth import Synth, bc_phases, point_sources

    bc = bc_phases((0, 0, 0, np.pi))
    sel = args.workloads.split(",")

    def solve(lat, b, **kw):
        lat.cg(b, **kw)  # warm (allocations, first launches)
        lat.reset_stats()
        torch.cuda.synchronize()
        return lat.cg(b, **kw)

    def hop_gbs(lat, prec):
        st = lat.stats(prec)
        return st["hop_bytes"] / st["hop_seconds"] / 1e9 if st["hop_seconds"] else None

    if "mixed" in sel:
        dims = (16, 16, 16, 32)
        s = Synth(0, device="cuda")
        U = s.gauge(dims)
        b = s.gaussian_spinor(dims, 1)
        # the solves timed without per-launch events (which would keep the library from
        # replaying captured iteration blocks); a second handle with events gives the
        # hop GB/s
        lat = cola.Lattice(dims, KAPPA, bc, 0.0)
        lat.set_gauge(U)
        _, i64 = solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        _, i32 = solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP32_RELIABLE,
                       tol=TOL, reliable_interval=50)
        lat.close()
        lat = cola.Lattice(dims, KAPPA, bc, 0.0, cola.COLA_FLAG_TIMING)
        lat.set_gauge(U)
        solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        g64 = hop_gbs(lat, cola.COLA_FP64)
        solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP32_RELIABLE, tol=TOL,
              reliable_interval=50)
        g32 = hop_gbs(lat, cola.COLA_FP32)
        print(json.dumps({"workload": "wilson_eo_16x16x16x32_fp32_reliable", "lattice": list(dims),
                          "fp64": {"seconds": i64["seconds"], "iterations": i64["iterations"],
                                   "residual": i64["true_rel_residual"][0], "hop_GBs": g64},
                          "fp32_reliable": {"seconds": i32["seconds"],
                                            "iterations": i32["iterations"],
                                            "reliable_updates": i32["reliable_updates"],
                                            "residual": i32["true_rel_residual"][0],
                                            "hop_GBs": g32},
                          "speedup": i64["seconds"] / i32["seconds"],
                          "note": "working set below the 256 MB infinity cache"}), flush=True)
        lat.close()
    if "force" in sel:
        dims = (24, 24, 24, 48)
        s = Synth(0, device="cuda")
        U = s.gauge(dims)
        eta = s.gaussian_spinor(dims, 1)
        lat = cola.Lattice(dims, KAPPA, bc, 0.0, cola.COLA_FLAG_TIMING)
        lat.set_gauge(U)
        ep = lat.pack(eta, cola.COLA_FP64, -1)
        pp = lat.empty_packed(cola.COLA_FP64, 1, -1)
        lat.dslash(pp, ep, cola.COLA_OP_MDAG, -1, cola.COLA_FP64, 1)
        phi = lat.unpack(pp, cola.COLA_FP64, 1, -1)
        X, info = solve(lat, phi, system=cola.COLA_SYS_MDAGM, scheme=cola.COLA_CG_FP64,
                        tol=1e-12)
        Xp = lat.pack(X, cola.COLA_FP64, -1)
        Yp = lat.empty_packed(cola.COLA_FP64, 1, -1)
        lat.dslash(Yp, Xp, cola.COLA_OP_M, -1, cola.COLA_FP64, 1)
        Y = lat.unpack(Yp, cola.COLA_FP64, 1, -1)
        lat.force(X[0], Y[0])
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            lat.force(X[0], Y[0], cola.COLA_FORCE_LIE)
        ev1.record()
        torch.cuda.synchronize()
        fms = ev0.elapsed_time(ev1) / 5
        V = int(np.prod(dims))
        # X, Y at two sites per link read (cache-shared), links 144 B, force 144 B out
        fbytes = V * (2 * 192 + 4 * 144 + 4 * 144)
        print(json.dumps({"workload": "force_24x24x24x48", "lattice": list(dims),
                          "solve_seconds": info["seconds"], "iterations": info["iterations"],
                          "force_ms": fms, "force_GBs": fbytes / fms / 1e6}), flush=True)
        lat.close()
    if "hmc" in sel:
        # one HMC trajectory (leapfrog) with one pseudofermion on the force lattice, and
        # the gauge-force and link-update kernels timed alone
        dims = (24, 24, 24, 48)
        beta, eps, nsteps = 5.6, 0.02, 10
        s = Synth(0, device="cuda")
        U = s.gauge(dims)
        P = s.momenta(dims)
        eta = s.gaussian_spinor(dims, 1)
        lat = cola.Lattice(dims, KAPPA, bc, 0.0)
        lat.set_gauge(U)
        ep = lat.pack(eta, cola.COLA_FP64, -1)
        pp = lat.empty_packed(cola.COLA_FP64, 1, -1)
        lat.dslash(pp, ep, cola.COLA_OP_MDAG, -1, cola.COLA_FP64, 1)
        phi = lat.unpack(pp, cola.COLA_FP64, 1, -1)[0]
        U0, P0 = U.clone(), P.clone()
        lat.hmc_trajectory(U, P, beta, eps, 2, phi=phi, cg_tol=1e-10)  # warm
        U.copy_(U0)
        P.copy_(P0)
        torch.cuda.synchronize()
        info = lat.hmc_trajectory(U, P, beta, eps, nsteps, phi=phi, cg_tol=1e-10)
        # the same with the even-odd pseudofermion (phi_e = S^H eta_e)
        ee = lat.pack(eta, cola.COLA_FP64, 0)
        pe = lat.empty_packed(cola.COLA_FP64, 1, 0)
        lat.dslash(pe, ee, cola.COLA_OP_SCHUR_DAG, 0, cola.COLA_FP64, 1)
        phi_e = lat.unpack(pe, cola.COLA_FP64, 1, 0)[0]
        U.copy_(U0)
        P.copy_(P0)
        lat.hmc_trajectory(U, P, beta, eps, 2, phi=phi_e, cg_tol=1e-10, eo=True)  # warm
        U.copy_(U0)
        P.copy_(P0)
        torch.cuda.synchronize()
        ieo = lat.hmc_trajectory(U, P, beta, eps, nsteps, phi=phi_e, cg_tol=1e-10, eo=True)
        # Omelyan with half as many steps (about the same number of force evaluations)
        U.copy_(U0)
        P.copy_(P0)
        torch.cuda.synchronize()
        iom = lat.hmc_trajectory(U, P, beta, 2 * eps, nsteps // 2, phi=phi_e, cg_tol=1e-10,
                                 eo=True, integrator="omelyan")
        # the same with FP32 solves and FP64 reliable updates
        U.copy_(U0)
        P.copy_(P0)
        torch.cuda.synchronize()
        imx = lat.hmc_trajectory(U, P, beta, 2 * eps, nsteps // 2, phi=phi_e, cg_tol=1e-10,
                                 eo=True, integrator="omelyan",
                                 cg_scheme=cola.COLA_CG_FP32_RELIABLE)
        # two time scales: 5 fermion steps of 2 eps, 4 gauge sub-steps each
        U.copy_(U0)
        P.copy_(P0)
        torch.cuda.synchronize()
        its = lat.hmc_trajectory(U, P, beta, 2 * eps, nsteps // 2, phi=phi_e, cg_tol=1e-10,
                                 eo=True, integrator="leapfrog_mts", n_gauge=4,
                                 cg_scheme=cola.COLA_CG_FP32_RELIABLE)
        V = int(np.prod(dims))
        nl = 4 * V
        F = lat.gauge_force(U, beta)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        for _ in range(10):
            lat.gauge_force(U, beta)
        ev[1].record()
        for _ in range(10):
            lat.link_update(U, F, 1e-3)
        ev[2].record()
        torch.cuda.synchronize()
        gms = ev[0].elapsed_time(ev[1]) / 10
        lms = ev[1].elapsed_time(ev[2]) / 10
        # gauge force: every link read once (staples share them through the caches) and
        # the force written: 2 x 144 B per link; link update: P and U read, U written
        print(json.dumps({"workload": "hmc_24x24x24x48", "lattice": list(dims), "beta": beta,
                          "kappa": KAPPA, "eps": eps, "nsteps": nsteps,
                          "trajectory_seconds": info["seconds"], "dH": info["dH"],
                          "H0": info["H0"], "cg_iterations": info["cg_iterations"],
                          "status": info["status"],
                          "eo": {"trajectory_seconds": ieo["seconds"], "dH": ieo["dH"],
                                 "cg_iterations": ieo["cg_iterations"],
                                 "status": ieo["status"]},
                          "eo_omelyan_half_steps": {"trajectory_seconds": iom["seconds"],
                                                    "dH": iom["dH"],
                                                    "cg_iterations": iom["cg_iterations"],
                                                    "status": iom["status"]},
                          "eo_omelyan_fp32_reliable": {"trajectory_seconds": imx["seconds"],
                                                       "dH": imx["dH"],
                                                       "cg_iterations": imx["cg_iterations"],
                                                       "status": imx["status"]},
                          "eo_two_scales_fp32_reliable": {"trajectory_seconds": its["seconds"],
                                                          "dH": its["dH"],
                                                          "cg_iterations": its["cg_iterations"],
                                                          "n_gauge": 4, "status": its["status"]},
                          "gauge_force_ms": gms, "gauge_force_GBs": nl * 288 / gms / 1e6,
                          "link_update_ms": lms, "link_update_GBs": nl * 432 / lms / 1e6}),
              flush=True)
        lat.close()
    if "quenched" in sel:
        # pure-gauge HMC from a cold start: the first ntherm trajectories are always kept
        # (far from equilibrium they violate energy by a lot), then Metropolis; acceptance
        # and the mean plaquette afterwards (an end-to-end check of the sampler)
        from paper_2302_00850_amd.synth import unit_gauge
        dims = (8, 8, 8, 8)
        beta, eps, nsteps, ntraj, ntherm = 6.0, 0.05, 20, 400, 100
        s = Synth(7, device="cuda", rng="torch")
        rng = np.random.default_rng(7)  # the Metropolis draws
        lat = cola.Lattice(dims, KAPPA, bc, 0.0)
        U = unit_gauge(dims, device="cuda")
        V = int(np.prod(dims))
        acc, plaq, dHs = 0, [], []
        t0 = time.perf_counter()
        for k in range(ntraj):
            P = s.momenta(dims)
            U0 = U.clone()
            info = lat.hmc_trajectory(U, P, beta, eps, nsteps, integrator="omelyan")
            if k < ntherm or rng.random() < np.exp(min(0.0, -info["dH"])):
                acc += k >= ntherm
            else:
                U.copy_(U0)
            if k >= ntherm:
                dHs.append(info["dH"])
                plaq.append(1.0 - lat.gauge_action(U, beta) / (beta * 6 * V))
        sec = time.perf_counter() - t0
        n = ntraj - ntherm
        pl = np.array(plaq)
        # error of the mean from blocks of 20 trajectories (autocorrelation)
        blocks = pl[: n - n % 20].reshape(-1, 20).mean(1)
        print(json.dumps({"workload": "hmc_quenched_8x8x8x8", "lattice": list(dims),
                          "beta": beta, "eps": eps, "nsteps": nsteps, "integrator": "omelyan",
                          "trajectories": ntraj, "thermalisation": ntherm,
                          "acceptance": acc / n, "mean_exp_minus_dH": float(np.mean(np.exp(-np.array(dHs)))),
                          "plaquette": float(pl.mean()),
                          "plaquette_err": float(blocks.std(ddof=1) / np.sqrt(len(blocks))),
                          "seconds": sec}), flush=True)
        lat.close()
    if "multishift" in sel:
        # 12 shifts of the even-odd normal system (a rational-approximation-like spread)
        # against one unshifted FP64 CG on the benchmark lattice
        dims = (32, 32, 32, 64)
        shifts = [0.0] + list(np.geomspace(1e-3, 3.0, 11))
        s = Synth(0, device="cuda", rng="torch")
        U = s.gauge(dims)
        b = s.gaussian_spinor(dims, 1)[0]
        lat = cola.Lattice(dims, KAPPA, bc, 0.0, cola.COLA_FLAG_TIMING)
        lat.set_gauge(U)
        lat.cg_multishift(b, shifts, system=cola.COLA_SYS_SCHUR, tol=TOL)  # warm
        torch.cuda.synchronize()
        x, ims = lat.cg_multishift(b, shifts, system=cola.COLA_SYS_SCHUR, tol=TOL)
        _, i1 = solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        print(json.dumps({"workload": "multishift_eo_32x32x32x64_12shifts", "lattice": list(dims),
                          "shifts": shifts, "seconds": ims["seconds"],
                          "iterations": ims["iterations"], "status": ims["status"],
                          "max_true_rel_residual": max(ims["true_rel_residual"]),
                          "unshifted_cg_seconds": i1["seconds"],
                          "unshifted_cg_iterations": i1["iterations"],
                          "cost_vs_one_solve": ims["seconds"] / i1["seconds"]}), flush=True)
        lat.close()
    if "eigen" in sel:
        # the 24 lowest modes of S^H S on 16^3 x 32 near the critical kappa (accelerated CG,
        # a loose tolerance: the modes serve deflation), then FP64 CG on a Gaussian source
        # with and without them.  24 is the size of the lowest cluster of this smooth field's
        # spectrum (the next eigenvalue is 2.3x larger): a set that cuts through a cluster
        # converges slowly, the method resolving near-degenerate modes one by one
        dims = (16, 16, 16, 32)
        kappa_e = 0.124
        s = Synth(0, device="cuda", rng="torch")
        U = s.gauge(dims)
        b = s.gaussian_spinor(dims, 1)
        X0 = torch.cat([s.gaussian_spinor(dims, 12), s.gaussian_spinor(dims, 12)])
        lat = cola.Lattice(dims, kappa_e, bc, 0.0, cola.COLA_FLAG_TIMING)
        lat.set_gauge(U)
        lam, X, ie = lat.eigensolve(X0, system=cola.COLA_SYS_SCHUR, tol=1e-5, max_sweeps=60)
        _, i0 = solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        lat.cg_deflated(b, X, lam, system=cola.COLA_SYS_SCHUR, tol=TOL)  # warm
        torch.cuda.synchronize()
        _, idf = lat.cg_deflated(b, X, lam, system=cola.COLA_SYS_SCHUR, tol=TOL)
        print(json.dumps({"workload": "eigen_eo_16x16x16x32_24modes", "lattice": list(dims),
                          "kappa": kappa_e,
                          "eigensolve": {"seconds": ie["seconds"], "sweeps": ie["sweeps"],
                                         "applications": ie["applications"],
                                         "status": ie["status"], "eigenvalues": lam,
                                         "max_residual": max(ie["residuals"])},
                          "cg_fp64": {"seconds": i0["seconds"], "iterations": i0["iterations"]},
                          "cg_fp64_deflated": {"seconds": idf["seconds"],
                                               "iterations": idf["iterations"],
                                               "residual": idf["true_rel_residual"][0]}}),
              flush=True)
        lat.close()
        del X, X0
        torch.cuda.empty_cache()
    if "flic" in sel:
        # FLIC (APE alpha 0.7, 4 sweeps, c_sw 1) on 32^3 x 64: 12 point sources, FP32 inner /
        # FP64 outer propagator against one FP64 source
        dims = (32, 32, 32, 64)
        s = Synth(0, device="cuda", rng="torch")
        U = s.gauge(dims)
        b = point_sources(dims, device="cuda")
        lat = cola.Lattice(dims, 0.118, bc, 1.0, cola.COLA_FLAG_TIMING)
        lat.set_gauge(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = lat.ape_smear(U, 0.7, 4)
        torch.cuda.synchronize()
        t_ape = time.perf_counter() - t0
        lat.set_fat_gauge(F)
        _, i32 = solve(lat, b, system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP32_DEFECT,
                       tol=TOL)
        g32 = hop_gbs(lat, cola.COLA_FP32)
        b1 = b[:1].clone()
        _, i64 = solve(lat, b1, system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP64, tol=TOL)
        g64 = hop_gbs(lat, cola.COLA_FP64)
        print(json.dumps({"workload": "flic_eo_32x32x32x64_12rhs_fp32defect",
                          "lattice": list(dims), "ape": {"alpha": 0.7, "sweeps": 4,
                                                         "seconds": t_ape},
                          "mixed_12rhs": {"seconds": i32["seconds"],
                                          "per_source": i32["seconds"] / 12,
                                          "iterations": i32["iterations"],
                                          "max_residual": max(i32["true_rel_residual"]),
                                          "hop_GBs": g32},
                          "fp64_1rhs": {"seconds": i64["seconds"],
                                        "iterations": i64["iterations"],
                                        "residual": i64["true_rel_residual"][0], "hop_GBs": g64},
                          "speedup_per_source": i64["seconds"] / (i32["seconds"] / 12)}),
              flush=True)
        lat.close()
    if "clover" in sel:
        dims = (48, 48, 48, 96)
        s = Synth(0, device="cuda", rng="torch")
        U = s.gauge(dims)
        b = point_sources(dims, device="cuda")
        lat = cola.Lattice(dims, 0.118, bc, 1.0, cola.COLA_FLAG_TIMING)
        lat.set_gauge(U)
        _, i32 = solve(lat, b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP32_DEFECT, tol=TOL,
                    block=args.block)
        g32 = hop_gbs(lat, cola.COLA_FP32)
        b1 = b[:1].clone()
        _, i64 = solve(lat, b1, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        g64 = hop_gbs(lat, cola.COLA_FP64)
        print(json.dumps({"workload": "clover_eo_48x48x48x96_12rhs_fp32defect",
                          "lattice": list(dims), "block_cg": bool(args.block),
                          "mixed_12rhs": {"seconds": i32["seconds"],
                                          "per_source": i32["seconds"] / 12,
                                          "iterations": i32["iterations"],
                                          "outer_cycles": i32["outer_cycles"],
                                          "max_residual": max(i32["true_rel_residual"]),
                                          "hop_GBs": g32},
                          "fp64_1rhs": {"seconds": i64["seconds"],
                                        "iterations": i64["iterations"],
                                        "residual": i64["true_rel_residual"][0], "hop_GBs": g64},
                          "speedup_per_source": i64["seconds"] / (i32["seconds"] / 12)}),
              flush=True)
        lat.close()


def copy_mode(args):
    """A plain device-to-device copy of known size: HBM counter calibration and the
    achievable copy bandwidth (bytes read + written per second)."""
    import torch

    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.iters):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.iters
    print(json.dumps({"mode": "copy", "bytes_read": n, "bytes_written": n,
                      "copies": args.iters + 1, "avg_ms": ms,
                      "GBs": 2 * n / ms / 1e6}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--no-alt", action="store_true",
                    help="skip the other multi-rhs solver (block CG vs lockstep)")
    ap.add_argument("--no-c3", action="store_true", help="skip the 32^3x64 FP16 workload")
    ap.add_argument("--mode", default="solve", choices=["solve", "hop", "copy", "workloads"])
    ap.add_argument("--workloads",
                    default="mixed,force,clover,hmc,multishift,quenched,eigen,flic",
                    help="workloads mode: any of mixed, force, clover, hmc, multishift, "
                         "quenched, eigen, flic")
    ap.add_argument("--block", type=int, default=0, help="use block CG in the multi-RHS solves")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="inner relative residual reduction of the defect-correction solves "
                         "(0: the library's default)")
    ap.add_argument("--lattice", default="32,32,32,64", help="hop mode: Lx,Ly,Lz,Lt")
    ap.add_argument("--prec", default="0,2,3", help="hop mode: precisions (0 FP64 .. 3 FP16)")
    ap.add_argument("--nrhs", default="1,12", help="hop mode: right-hand-side counts")
    ap.add_argument("--iters", type=int, default=20, help="hop mode: timed launches")
    ap.add_argument("--tune", action="store_true",
                    help="hop mode: autotune launch shapes on first use")
    ap.add_argument("--no-tune", action="store_true",
                    help="solve mode: keep the library's default launch shapes (by default the "
                         "first warmup tunes every hop shape the solve uses)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(domain decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "hop":
        hop_mode(args)
        return
    if args.mode == "copy":
        copy_mode(args)
        return
    if args.mode == "workloads":
        workloads_mode(args)
        return

    import torch

    from paper_2302_00850_amd import cola
    from paper_2302_00850_amd.synth import Synth, bc_phases, point_sources

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    log(f"generating {DIMS} links (seed 0, device generator)")
    t0 = time.perf_counter()
    U = Synth(0, device=dev, rng="torch").gauge(DIMS)
    b = point_sources(DIMS, device=dev)
    bc = bc_phases((0, 0, 0, np.pi))
    lat = cola.Lattice(DIMS, KAPPA_C, bc, CSW, cola.COLA_FLAG_TIMING)
    lat.set_gauge(U)
    assert lat.gauge_is_su3
    log(f"fields and clover blocks ready in {time.perf_counter() - t0:.1f} s")
    tune = not args.no_tune and args.warmup > 0  # tuning stays out of the timed steps
    if tune:
        cola.cola_set_tuning(lat.h, 1)  # launch shapes measured on first use (warmup)
    block = args.block

    def solve(blk):
        return lat.cg(b, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP32_DEFECT, tol=TOL,
                      block=blk, inner_tol=args.inner_tol)

    for w in range(args.warmup):
        _, info = solve(block)
        log(f"warmup {w}: {info['iterations']} inner iterations, {info['outer_cycles']} cycles, "
            f"{info['seconds']:.3f} s, status {info['status']}")
    lat.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        x, info = solve(block)
        infos.append(info)
        log(f"step {k}: {info['iterations']} it, {info['outer_cycles']} cycles, "
            f"{info['seconds']:.3f} s, max residual {max(info['true_rel_residual']):.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st32 = lat.stats(cola.COLA_FP32)
    st64 = lat.stats(cola.COLA_FP64)
    ms_per_step = wall / args.steps * 1e3
    ok = all(i["status"] == cola.COLA_OK for i in infos)
    del x
    # the dominant kernel: the FP32 12-rhs hop with the clover epilogue (t_o = A^-1 D p),
    # 2688 B per site of links and spinors plus the 288 B clover block it reads
    kc = st32["kinds"].get(cola.COLA_HOP_CLOV, {"launches": 0, "seconds": 0.0, "bytes": 0.0})
    achieved = kc["bytes"] / kc["seconds"] / 1e9 if kc["seconds"] else 0.0
    per_launch_ms = kc["seconds"] / max(1, kc["launches"]) * 1e3
    blended = st32["hop_bytes"] / st32["hop_seconds"] / 1e9 if st32["hop_seconds"] else None
    kinds = {str(k): {"launches": v["launches"],
                      "avg_ms": round(v["seconds"] / v["launches"] * 1e3, 4),
                      "GBs": round(v["bytes"] / v["seconds"] / 1e9, 1)}
             for k, v in st32["kinds"].items()}

    alt = None
    if not args.no_alt:
        # the other multi-rhs solver on the same workload (one warm-up, one timed solve)
        solve(1 - block)
        torch.cuda.synchronize()
        _, ia = solve(1 - block)
        alt = {"solver": "block CG" if block == 0 else "lockstep", "seconds_per_source":
               ia["seconds"] / 12, "iterations": ia["iterations"],
               "outer_cycles": ia["outer_cycles"], "status": ia["status"],
               "max_true_rel_residual": max(ia["true_rel_residual"])}
        log(f"{alt['solver']}: {ia['iterations']} it, {ia['seconds']:.3f} s")

    fp64 = None
    if not args.no_fp64:
        b1 = b[:1].clone()
        lat.cg(b1, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)  # warm
        lat.reset_stats()
        _, i64 = lat.cg(b1, system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=TOL)
        s64 = lat.stats(cola.COLA_FP64)
        fp64 = {"seconds_per_source": i64["seconds"], "iterations": i64["iterations"],
                "hop_GBs": s64["hop_bytes"] / s64["hop_seconds"] / 1e9,
                "true_rel_residual": i64["true_rel_residual"][0]}
        log(f"FP64 single-source CG: {i64['iterations']} it, {i64['seconds']:.3f} s")
        del b1
    lat.close()
    del b
    torch.cuda.empty_cache()

    c3 = None
    if not args.no_c3:
        c3 = fp16_workload(args)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        Uc = U.cpu().numpy()
        del U
        # a point source: the values do not change the oracle's cost
        psi = np.zeros(tuple(reversed(DIMS)) + (4, 3), dtype=np.complex128)
        psi[0, 0, 0, 0, 0, 0] = 1.0
        cpu = cpu_baseline(Uc, psi, DIMS)
        del Uc, psi

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
        "dtype": "f32 inner (storage and arithmetic), f64 outer",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "lattice": list(DIMS), "kappa": KAPPA_C, "csw": CSW,
                   "nrhs": 12, "sources": "point (12 spin-colour at origin)",
                   "solver": ("block CG" if block else "lockstep 12-RHS CG")
                             + ", FP32 inner + FP64 defect correction, even-odd clover Schur",
                   "tol": TOL, "inner_tol": args.inner_tol if args.inner_tol > 0 else 1e-5,
                   "parallelism": "none (1 GPU)",
                   "launch_shapes": "autotuned in warmup" if tune else "library defaults"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(), "hop_sources_sha256": hop_sources_sha256(),
                     "kernel": "hop_kernel FP32 12-real links, 12 rhs, clover epilogue "
                               "(A^-1 D p)",
                     "bytes_per_launch": kc["bytes"] / max(1, kc["launches"]),
                     "avg_launch_ms": round(per_launch_ms, 4),
                     "launches": kc["launches"]},
        "hop_fp32_all_launches": {"GBs": round(blended, 1) if blended else None,
                                  "launches": st32["hop_launches"],
                                  "TFs": round(st32["hop_flops"] / st32["hop_seconds"] / 1e12, 2)
                                  if st32["hop_seconds"] else None,
                                  "by_kind": kinds},
        "cg": {"seconds_per_source": per_source, "all_converged": ok,
               "inner_iterations": infos[-1]["iterations"], "outer_cycles": infos[-1]["outer_cycles"],
               "max_true_rel_residual": max(max(i["true_rel_residual"]) for i in infos),
               "fp64_outer_hop_GBs": (st64["hop_bytes"] / st64["hop_seconds"] / 1e9
                                      if st64["hop_seconds"] else None)},
        "other_solver": alt,
        "fp64_single_rhs": fp64,
        "speedup_per_source_vs_fp64": (fp64["seconds_per_source"] / per_source) if fp64 else None,
        "fp16_32x32x32x64": c3,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def fp16_workload(args):
    """The 32^3 x 64 plain-Wilson workload with FP16 storage (the spin projection in packed
    FP16 arithmetic, SU(3) products of FP16 pairs summed in FP32, FP32 elsewhere) inside FP64
    defect correction, 12 point sources, against one FP64 source."""
    import torch

    from paper_2302_00850_amd import cola
    from paper_2302_00850_amd.synth import Synth, bc_phases, point_sources

    dev = torch.device("cuda:0")
    U = Synth(0, device=dev).gauge(DIMS3)
    b = point_sources(DIMS3, device=dev)
    lat = cola.Lattice(DIMS3, KAPPA, bc_phases((0, 0, 0, np.pi)), 0.0, cola.COLA_FLAG_TIMING)
    lat.set_gauge(U)

    def solve(scheme, rhs):
        return lat.cg(rhs, system=cola.COLA_SYS_SCHUR, scheme=scheme, tol=TOL)

    solve(cola.COLA_CG_FP16_DEFECT, b)
    lat.reset_stats()
    torch.cuda.synchronize()
    n = 3
    t0 = time.perf_counter()
    for _ in range(n):
        _, info = solve(cola.COLA_CG_FP16_DEFECT, b)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / n / 12
    st = lat.stats(cola.COLA_FP16)
    kp = st["kinds"].get(cola.COLA_HOP_PLAIN)
    b1 = b[:1].clone()
    solve(cola.COLA_CG_FP64, b1)
    _, i64 = solve(cola.COLA_CG_FP64, b1)
    lat.close()
    log(f"32^3x64 FP16: {per * 12:.3f} s per 12 sources, FP64 {i64['seconds']:.3f} s per source")
    return {"workload": "wilson_eo_32x32x32x64_12rhs_fp16defect",
            "dtype": "f16 storage; spin projection in packed f16 arithmetic, SU(3) products "
                     "of f16 pairs summed in f32, f32 elsewhere; f64 outer",
            "seconds_per_source": per, "inner_iterations": info["iterations"],
            "outer_cycles": info["outer_cycles"],
            "max_true_rel_residual": max(info["true_rel_residual"]),
            "plain_hop_GBs": kp["bytes"] / kp["seconds"] / 1e9 if kp else None,
            "plain_hop_avg_ms": kp["seconds"] / kp["launches"] * 1e3 if kp else None,
            "all_hops_GBs": st["hop_bytes"] / st["hop_seconds"] / 1e9,
            "fp64_seconds_per_source": i64["seconds"],
            "speedup_per_source_vs_fp64": i64["seconds"] / per}


if __name__ == "__main__":
    main()
