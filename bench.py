#!/usr/bin/env python3
"""Benchmark of the octree multigrid solver on one MI355X.

Workload (default): the 3D manufactured problem on the unit cube, 256^3
cells in 16^3-cell blocks (4681 blocks on 6 levels incl. the 8^3 coarse
grid), sphere r = 0.3 at the centre, phi = exp(x) sin(pi y) cos(pi z) for the
rhs and all Dirichlet data, FP64.

One step = one full solve from phi = 0 to a relative max-norm residual of
1e-10 with FAS V(2,2) cycles: every step of the method's hot path
(red-black smoothing, residuals, FAS restriction, prolongation, coarse
solve, convergence control) over one right-hand side already resident in
HBM.  Printed as one JSON line:

  value      whole-job smoother throughput, Mcell-updates/s: smoother cell
             updates on all levels during the timed solves / timed wall time
  roofline   the dominant kernel (finest-level red-black half sweep):
             algorithmic bytes per launch / its mean duration from HIP
             events recorded on the solve's stream, against 8 TB/s
  cpu_baseline  the FP64 CPU oracle timed on the host cores over a bounded
             sample (a few V-cycles of the same problem)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
PMC_RECORD = os.path.join(ROOT, "profiles", "gs_half3_mms3d_256_pmc.json")


def achievable_copy_gbs(torch, stream, mib=256, reps=5):
    """Best rate of a plain 256 MiB device-to-device copy on this GPU (bytes
    read + written per second, GB/s): the bandwidth an HBM-bound kernel can
    reach in practice, beside the 8 TB/s peak."""
    x = torch.ones(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    best = float("inf")
    with torch.cuda.stream(stream):
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            y.copy_(x)
            b.record(stream)
            b.synchronize()
            best = min(best, a.elapsed_time(b))
    return 2 * x.numel() * 8 / (best * 1e-3) / 1e9


def measured_traffic():
    """HBM bytes per launch of the finest-level sweep from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, if they were taken on the current
    kernel source (sha256 recorded with them); otherwise None."""
    import hashlib
    try:
        rec = json.load(open(PMC_RECORD))
        src = open(os.path.join(ROOT, "paper_2205_09411_amd", "csrc", "kernels.hip"), "rb").read()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec["hbm_bytes_per_launch"]


def workload(name):
    from paper_2205_09411_amd import workloads as W
    if name == "mms3d_256":
        return W.mms3d(max_level=5, block_n=16)
    if name == "mms3d_128":
        return W.mms3d(max_level=4, block_n=16)
    if name == "mms3d_512":
        return W.mms3d(max_level=6, block_n=16)
    raise SystemExit(f"unknown workload {name}")


def smoother_updates_per_vcycle(levels, n_smooth=4):
    # every level above the coarsest is smoothed n_down + n_up times per cycle
    return sum(l["nblocks"] * l["Nb"] ** 3 for l in levels[1:]) * n_smooth


def timed_solves(S, n, stream, **kw):
    import torch
    S.solve(stream=stream, zero_start=True, **kw)  # warm (graphs captured here)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = [S.solve(stream=stream, zero_start=True, **kw) for _ in range(n)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / n, reps[-1]


# set by main(): compare results with the FP64 oracle (host CPU) after the GPU work
ORACLE_CHECKS = True


def vs_oracle(o, phi, r0, cycles=3):
    """A GPU result against the FP64 oracle on the same problem: the oracle's
    leaf residual of the result (relative to the residual of phi = 0), then
    `cycles` of the oracle's own V-cycles started from the result, and the
    max difference between the result and that oracle iterate.  The oracle's
    residual after its cycles is reported too: when it is far below the
    result's, the difference is the result's error against the converged
    FP64 oracle solution."""
    t = time.perf_counter()
    r = float(np.abs(o.leaf_residual(phi)).max())  # also sets the oracle's phi to the result
    for _ in range(cycles):
        o.vcycle()
    ref = o.get_solution()
    err = float(np.abs(phi - ref).max())
    return {"oracle_rel_residual_of_result": r / r0, "oracle_rel_residual_after": o.residual_max() / r0,
            "oracle_cycles_from_result": cycles, "max_abs_diff_vs_oracle": err,
            "rel_diff_vs_oracle": err / max(float(np.abs(ref).max()), 1e-300),
            "oracle_s": round(time.perf_counter() - t, 1)}


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def leg_mixed(G, w, phi64, t64, stream, steps, rtol, tune=True):
    """Same problem, FP32 inner cycles inside FP64 defect correction, in the
    launch configuration the autotuner picks for it."""
    from paper_2205_09411_amd import octmg
    S = octmg.State(G, 1, octmg.MIXED)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    S.set_rhs(w.rhs(xyz))
    tuned, cand_ms = S.autotune(rtol=rtol, reps=2, stream=stream) if tune else (S.get_launch(), [])
    # FP32 finest-level half sweeps timed with HIP events (eager launches)
    S.profile(True)
    S.profile_read()
    for _ in range(steps):
        S.solve(rtol=rtol, max_cycles=40, zero_start=True, stream=stream)
    prof = S.profile_read()
    S.profile(False)
    dt, rep = timed_solves(S, steps, stream, rtol=rtol, max_cycles=40, graph_mode=tuned["graph_mode"])
    phi = S.get_solution()
    MIXED_PHI["phi"] = phi
    top = G.level_info(G.n_levels - 1)
    ncell = top["nblocks"] * top["Nb"] ** 3
    # algorithmic bytes of one FP32 half sweep: 6 B per cell of the level
    # (other colour's phi, g and the written phi of half the cells, 4 B
    # each) plus the FP32 stencil record (32 B) and boundary term (4 B) of
    # the custom cells of that colour
    b32 = 6.0 * ncell + 18.0 * top["nrec"]
    ms32 = prof["finest_half_sweep_ms"] / max(1, prof["finest_half_sweeps"])
    a32 = b32 / (ms32 * 1e-3) / 1e9
    return {"solves_per_s": round(1 / dt, 3), "ms_per_solve": round(dt * 1e3, 3), "speedup_vs_fp64": round(t64 / dt, 3),
            "launch": {"chosen": tuned, "autotune_ms_per_solve": [round(v, 3) for v in cand_ms]},
            "sweep_roofline_fp32": {"bound": "hbm", "achieved": round(a32, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(a32 / HBM_PEAK_GBS, 4), "kernel": "k_gs_half3<float,16> (finest level)",
                                    "bytes_per_launch": b32, "mean_launch_ms": round(ms32, 5),
                                    "launches_timed": prof["finest_half_sweeps"]},
            "outer_iterations": rep.cycles, "final_rel_residual": rep.r_final / rep.r0,
            "rel_diff_vs_fp64_solution": rel(phi, phi64), "max_err_vs_exact": float(np.abs(phi - w.exact(xyz)).max())}


MIXED_PHI = {}  # the mixed leg's solution, compared with the oracle at the end


def leg_batched(stream, rtol, reps=3, n_single=4):
    """Cylinder r=0.2, 128^3 in 16^3 blocks, 64 Gaussian-source rhs solved
    together (FP32 inner / FP64 outer, captured cycle graph) against FP64
    and one-rhs-at-a-time solves on the same GPU."""
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    w = W.cylinder(max_level=4, n_rhs=64)
    G = octmg.Geometry(w.geom)
    xyz, _ = G.leaf_coords()
    g = np.stack([w.rhs(xyz, i) for i in range(64)])
    out = {"workload": f"{w.geom.name}: 128^3 in 16^3 blocks ({G.n_blocks} blocks), 64 rhs, phi=0 on cylinder and cube",
           "cells_all_levels_per_rhs": int(sum(G.level_info(i)["nblocks"] * G.level_info(i)["Nb"] ** 3
                                              for i in range(G.n_levels)))}
    sols, r0s = {}, {}
    for name, prec in (("mixed", octmg.MIXED), ("fp64", octmg.FP64)):
        S = octmg.State(G, 64, prec)
        S.set_boundary(None, np.zeros(G.n_domain))
        S.set_rhs(g)
        # the cycle count of this batch, so that the whole-solve graph
        # candidates capture one cycle more than it needs
        first = S.solve(rtol=rtol, max_cycles=40, zero_start=True, stream=stream)
        mc = first.cycles + 1
        tuned, cand_ms = S.autotune(rtol=rtol, max_cycles=mc, reps=1, stream=stream)
        dt, rep = timed_solves(S, reps, stream, rtol=rtol, max_cycles=mc, graph_mode=tuned["graph_mode"])
        sols[name] = S.get_solution()
        r0s[name] = rep.per_rhs["r0"].copy()
        # candidates 0..13 launch cycle by cycle, the last two run the solve
        # as captured chunks of cycles (512- and 256-thread kernels): one
        # graph launch once the first chunk is sized by the previous solve
        one = min(cand_ms[-2:])
        other = min(cand_ms[:-2])
        out[name] = {"batch_ms": round(dt * 1e3, 3), "rhs_solves_per_s": round(64 / dt, 2), "cycles": rep.cycles,
                     "final_rel_residual": rep.r_final / rep.r0,
                     "launch": {"chosen": tuned, "autotune_ms_per_batch": [round(v, 3) for v in cand_ms],
                                "whole_solve_graph_ms": round(one, 3), "best_per_cycle_launch_ms": round(other, 3),
                                "winner": "whole-solve graph" if one < other else "per-cycle launches",
                                "whole_solve_graph_vs_best_other": round(other / one, 3)}}
        del S
    S1 = octmg.State(G, 1, octmg.FP64)
    S1.set_boundary(None, np.zeros(G.n_domain))
    t1 = 0.0
    d1 = 0.0
    for i in range(n_single):
        S1.set_rhs(g[i])
        dt, _ = timed_solves(S1, 1, stream, rtol=rtol, max_cycles=40, graph_mode=1)
        t1 += dt
        d1 = max(d1, rel(sols["fp64"][i], S1.get_solution()))
    out["single_rhs_fp64"] = {"ms_per_rhs": round(t1 / n_single * 1e3, 3), "rhs_solves_per_s": round(n_single / t1, 2),
                              "sample": f"first {n_single} rhs, one at a time"}
    out["batched_fp64_vs_single_max_rel_diff"] = d1
    out["mixed_vs_fp64_max_rel_diff"] = rel(sols["mixed"], sols["fp64"])
    if ORACLE_CHECKS:
        import oracle
        o = oracle.Oracle(w.geom)
        o.set_boundary(np.zeros(len(o.iface_points())), np.zeros(len(o.domain_points())))
        chk = {}
        for lane in (0, 63):
            o.set_rhs(g[lane])
            for name in ("mixed", "fp64"):
                chk[f"{name}_lane{lane}"] = vs_oracle(o, sols[name][lane], float(r0s[name][lane]))
        out["vs_oracle"] = chk
    out["speedup_mixed_batch_vs_single_fp64"] = round(out["mixed"]["rhs_solves_per_s"] /
                                                      out["single_rhs_fp64"]["rhs_solves_per_s"], 2)
    return out


def leg_adaptive(stream, rtol, reps=3):
    """20 seeded spheres, adaptive 16^3-block octree to level 6 (dx = 1/512),
    phi=1 on the spheres, 0 on the cube, g ~ N(0,1): FP64 against mixed."""
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    w = W.spheres()
    t = time.perf_counter()
    G = octmg.Geometry(w.geom)
    setup = time.perf_counter() - t
    xyz, _ = G.leaf_coords()
    g = w.rhs(xyz)
    out = {"workload": f"{w.geom.name}: adaptive octree, {G.n_levels} levels, {G.n_blocks} blocks",
           "leaf_cells": int(G.n_leaf), "interface_records": int(G.n_records), "setup_s": round(setup, 3)}
    sols = {}
    for name, prec in (("fp64", octmg.FP64), ("mixed", octmg.MIXED)):
        S = octmg.State(G, 1, prec)
        S.set_boundary_fn(w.iface_value, w.domain_value)
        S.set_rhs(g)
        dt, rep = timed_solves(S, reps, stream, rtol=rtol, max_cycles=40, graph_mode=1)
        sols[name] = S.get_solution()
        r0 = rep.r0
        out[name] = {"ms_per_solve": round(dt * 1e3, 3), "solves_per_s": round(1 / dt, 3), "cycles": rep.cycles,
                     "final_rel_residual": rep.r_final / rep.r0,
                     "leaf_cell_solves_per_s_G": round(G.n_leaf / dt / 1e9, 3)}
        del S
    out["mixed_vs_fp64_max_rel_diff"] = rel(sols["mixed"], sols["fp64"])
    if ORACLE_CHECKS:
        import oracle
        del G
        o = oracle.setup_workload(w)
        out["vs_oracle"] = {name: vs_oracle(o, sols[name], r0, cycles=2) for name in ("fp64", "mixed")}
    return out


def leg_serving(stream, n_requests=1000, rtol=1e-8, budget_gb=64, max_lanes=16):
    """Poisson arrivals over 4 sphere-union geometries x {64^3, 128^3, 256^3}
    (16^3 blocks), each request its own Gaussian-source rhs (seed 10000 + i,
    resident in HBM), rtol 1e-8: the batching server (mixed precision) against
    a plain FP64 one-at-a-time loop on the same GPU, at 0.8x the plain loop's
    throughput and above."""
    import torch
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    params = W.serving_geometries()
    pairs = {}
    t = time.perf_counter()
    for lv in (3, 4, 5):
        for gid, p in enumerate(params):
            geom = W.Geometry(dim=3, block_n=16, max_level=lv, lsf_kind=W.LSF_SPHERES, lsf_params=p,
                              w_min=8e-3, name=f"serve_g{gid}_{16 << (lv - 1)}")
            G = octmg.Geometry(geom)
            xyz, _ = G.leaf_coords()
            pairs[(lv, gid)] = {"G": G, "x": torch.tensor(xyz, device="cuda"), "iface": np.ones(G.n_iface),
                                "dom": np.zeros(G.n_domain), "free": []}
    torch.cuda.synchronize()
    geometry_s = time.perf_counter() - t

    def sources(x, seed):  # workloads.gaussian_sources on the device
        amp, wid, cen = W.gaussian_params(seed)
        g = torch.zeros(x.shape[0], dtype=torch.float64, device="cuda")
        for a, w_, c in zip(amp, wid, cen):
            d2 = ((x - torch.tensor(c, device="cuda")) ** 2).sum(dim=1)
            g += a * torch.exp(-d2 / (2.0 * w_ * w_))
        return g

    # every stream below draws the same (size, geometry, seed) per request
    stream0 = W.serving_stream(n_requests, 1.0)
    req_rhs = {seed: sources(pairs[(lv, gid)]["x"], seed) for (_, lv, gid, seed) in stream0}
    for pr in pairs.values():
        pr["warm"] = sources(pr["x"], 9999)  # warm-up and service-time probes
        del pr["x"]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t

    def out_buf(pr):
        return pr["free"].pop() if pr["free"] else torch.empty(pr["G"].n_leaf, dtype=torch.float64, device="cuda")

    # plain loop: one FP64 state per pair, one request at a time
    plain = {}
    for key, pr in pairs.items():
        S = octmg.State(pr["G"], 1, octmg.FP64)
        S.set_boundary(pr["iface"], pr["dom"])
        pr["plain"] = S
        S.set_rhs(pr["warm"], stream=stream)
        S.solve(rtol=rtol, zero_start=True, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for j in range(2):
            S.solve(rtol=rtol, zero_start=True, stream=stream)
        torch.cuda.synchronize()
        plain[key] = (time.perf_counter() - t) / 2
    mu_plain = 1.0 / float(np.mean(list(plain.values())))

    def run_plain(reqs):
        lat = []
        t0 = time.perf_counter()
        for (ta, lv, gid, seed) in reqs:
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            pr = pairs[(lv, gid)]
            S = pr["plain"]
            S.set_rhs(req_rhs[seed], stream=stream)
            S.solve(rtol=rtol, zero_start=True, stream=stream)
            lat.append(time.perf_counter() - t0 - ta)
        return np.array(lat), time.perf_counter() - t0

    def run_server(reqs):
        srv = octmg.Server(hbm_budget_bytes=budget_gb << 30, max_lanes=max_lanes, precision=octmg.MIXED)
        slot = {key: srv.add_geometry(pr["G"], pr["iface"], pr["dom"]) for key, pr in pairs.items()}
        # warm-up: one request per geometry creates its resident state and
        # captures its cycle graph before the timed stream starts
        warm = [srv.submit(slot[key], pr["warm"], out_buf(pr), rtol) for key, pr in pairs.items()]
        while warm:
            for r in srv.poll():
                warm.remove(r["id"])
            time.sleep(0.001)
        meta = {}
        done = {}
        t0 = time.perf_counter()
        i = 0
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i][0] <= now:
                ta, lv, gid, seed = reqs[i]
                pr = pairs[(lv, gid)]
                o = out_buf(pr)
                rid = srv.submit(slot[(lv, gid)], req_rhs[seed], o, rtol)
                meta[rid] = (ta, pr, o)
                i += 1
            for r in srv.poll():
                ta, pr, o = meta.pop(r["id"])
                pr["free"].append(o)
                done[r["id"]] = r
            time.sleep(0.0002)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        bad = sum(1 for r in done.values() if r["status"] != 0)
        lat = np.array([r["t_done"] - r["t_submit"] for r in done.values()])
        return lat, wall, st, bad

    def summary(lat, wall, n):
        return {"solves_per_s": round(n / wall, 1), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "wall_s": round(wall, 2)}

    out = {"workload": "4 geometries (unions of 1/5/10/20 spheres, phi=1 on spheres, 0 on cube) x {64^3,128^3,256^3} "
                       "in 16^3 blocks, one Gaussian-source rhs per request (seed 10000+i) resident in HBM, "
                       "Poisson arrivals, rtol 1e-8",
           "rhs_resident_gb": round(sum(v.numel() for v in req_rhs.values()) * 8 / 2 ** 30, 1),
           "requests": n_requests, "setup_s": round(setup_s, 2), "geometry_setup_s": round(geometry_s, 2),
           "rhs_generation_s": round(setup_s - geometry_s, 2),
           "plain_fp64_service_ms": {f"{16 << (k[0] - 1)}^3/g{k[1]}": round(v * 1e3, 3) for k, v in plain.items()},
           "plain_fp64_capacity_solves_per_s": round(mu_plain, 1)}
    lam = 0.8 * mu_plain
    reqs = W.serving_stream(n_requests, lam)
    lat, wall = run_plain(reqs)
    out["plain_fp64_at_0.8x"] = dict(summary(lat, wall, n_requests), rate_hz=round(lam, 1))
    for f in (0.8, 2.0, 4.0):
        reqs = W.serving_stream(n_requests, f * mu_plain)
        lat, wall, st, bad = run_server(reqs)
        out[f"server_mixed_at_{f}x"] = dict(summary(lat, wall, n_requests), rate_hz=round(f * mu_plain, 1),
                                            failed=bad, states_created=st["states_created"],
                                            lanes_per_cycle=round(st["lane_cycles"] / max(1, st["cycles_launched"]), 2),
                                            peak_gb=round(st["peak_bytes"] / 2 ** 30, 2))
        print(f"serving at {f}x done", file=sys.stderr, flush=True)
    for pr in pairs.values():
        del pr["plain"]
    req_rhs.clear()
    return out


def leg_table1(stream, n_fmg=40):
    """The Sec. 4.1 sphere (R = 1/4, domain [-1/2,1/2]^3, exact solution on
    the domain boundary) on a uniform 512^3 grid, FP64: time per FMG cycle
    over n_fmg consecutive FMG cycles, for 8^3 and 16^3 blocks, beside the
    paper's Table 1 (Epyc 7H12, 32 cores: 1.46 s and 0.95 s)."""
    import torch
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    paper_32 = {8: 1.46, 16: 0.95}
    out = {"workload": "sphere R=1/4 centred in [-1/2,1/2]^3, uniform 512^3, FP64, FMG cycles from the previous "
                       "iterate (the first from phi=0)"}
    for bn, lmax in ((8, 7), (16, 6)):
        w = W.sphere_f1(dim=3, max_level=lmax, block_n=bn)
        t = time.perf_counter()
        G = octmg.Geometry(w.geom)
        setup = time.perf_counter() - t
        S = octmg.State(G)
        S.set_boundary_fn(w.iface_value, w.domain_value)
        xyz, _ = G.leaf_coords()
        S.set_rhs(np.zeros(G.n_leaf))
        outside = np.sqrt((xyz ** 2).sum(axis=1)) > 0.25
        ex = w.exact(xyz)[outside]
        errs = []
        S.fmg(have_guess=False, stream=stream)
        for k in range(2):
            errs.append(float(np.abs(S.get_solution()[outside] - ex).max()))
            S.fmg(have_guess=True, stream=stream)
        errs.append(float(np.abs(S.get_solution()[outside] - ex).max()))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n_fmg):
            S.fmg(have_guess=True, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / n_fmg
        out[f"blocks_{bn}^3"] = {"ms_per_fmg": round(dt * 1e3, 3), "setup_s": round(setup, 2),
                                 "blocks": G.n_blocks, "cells_per_fmg_second_G": round(512 ** 3 / dt / 1e9, 2),
                                 "paper_epyc_7h12_32_cores_s": paper_32[bn],
                                 "speedup_vs_paper_32_cores": round(paper_32[bn] / dt, 1),
                                 "max_err_outside_sphere_fmg_1_2_3": errs}
        del S, G
        torch.cuda.empty_cache()
    out["blocks_32^3"] = "not supported: the colour tile of a 32^3 block (166 KB in FP64) exceeds the 160 KB LDS"
    return out


def leg_sharp(stream, n_fmg=4, reps=5):
    """Sec. 4.2: the spheroid, rhombus, heart and astroid boundaries
    (phi = 1 on them, 0 on the domain boundary, Laplace equation) on uniform
    1024^2 and 2048^2 grids (8^2 blocks, 8^2 coarse grid) and 256^3 (16^3
    blocks over an 8^3 grid), FP64: residual reduction per FMG iteration and
    time per FMG."""
    import torch
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    out = {"workload": "sharp shapes of Sec. 4.2, p = 4(x-0.5), q = 4(y-0.5) (3D, axisymmetric: "
                       "p = 4(sqrt(x^2+y^2)-0.5), q = 4(z-0.5)), phi=1 on the shape, 0 on the domain boundary, "
                       "FMG from phi=0"}
    for dim, lmax, bn, label in ((2, 8, 8, "1024^2"), (2, 9, 8, "2048^2"), (3, 5, 16, "256^3")):
        for shape in W.SHAPES:
            w = W.sharp_shape(shape, dim=dim, max_level=lmax, block_n=bn)
            G = octmg.Geometry(w.geom)
            S = octmg.State(G)
            S.set_boundary_fn(w.iface_value, w.domain_value)
            S.set_rhs(np.zeros(G.n_leaf))
            r = [float(S.residual_norm(phi_zero=True)[0])]
            for k in range(n_fmg):
                S.fmg(have_guess=k > 0, stream=stream)
                r.append(float(S.residual_norm(stream=stream)[0]))
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                S.fmg(have_guess=True, stream=stream)
            torch.cuda.synchronize()
            out[f"{shape}_{label}"] = {
                "reduction_per_fmg": [round(r[i] / r[i + 1], 1) if r[i + 1] > 0 else None for i in range(n_fmg)],
                "ms_per_fmg": round((time.perf_counter() - t) / reps * 1e3, 3),
                "interface_records": int(G.n_records)}
            del S, G
    return out


def leg_electrodes(stream, n_fmg=4, reps=3):
    """Sec. 4.3: rod (phi = 1) and half sphere (phi = 0) electrodes, phi = 1
    on top, 0 at the bottom, zero flux on the sides; dx = 1/128 everywhere
    and 1/512 near the electrodes (8^3 blocks): residual reduction per FMG
    iteration (the paper: about 30-40), time per FMG and per solve to 1e-10
    (FP64 and mixed), and the field |grad phi| by face differences."""
    import torch
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    w = W.two_electrodes()
    t = time.perf_counter()
    G = octmg.Geometry(w.geom)
    out = {"workload": "two electrodes, uniform 128^3 + refinement to 1/512 near the electrodes, 8^3 blocks, "
                       "zero-flux sides", "setup_s": round(time.perf_counter() - t, 3), "leaf_cells": int(G.n_leaf),
           "blocks": int(G.n_blocks), "levels": int(G.n_levels), "interface_records": int(G.n_records)}
    S = octmg.State(G)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    S.set_rhs(np.zeros(G.n_leaf))
    r = [float(S.residual_norm(phi_zero=True)[0])]
    for k in range(n_fmg):
        S.fmg(have_guess=k > 0, stream=stream)
        r.append(float(S.residual_norm(stream=stream)[0]))
    out["reduction_per_fmg"] = [round(r[i] / r[i + 1], 1) for i in range(n_fmg)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        S.fmg(have_guess=True, stream=stream)
    torch.cuda.synchronize()
    out["ms_per_fmg"] = round((time.perf_counter() - t) / reps * 1e3, 3)
    t = time.perf_counter()
    E = S.gradient(inside_zero=True, stream=stream)
    out["gradient_s_incl_copy"] = round(time.perf_counter() - t, 3)
    mag = np.linalg.norm(E, axis=1)
    out["max_abs_grad_phi"] = round(float(mag.max()), 3)
    for name, prec in (("fp64", octmg.FP64), ("mixed", octmg.MIXED)):
        Sp = octmg.State(G, 1, prec)
        Sp.set_boundary_fn(w.iface_value, w.domain_value)
        Sp.set_rhs(np.zeros(G.n_leaf))
        dt, rep = timed_solves(Sp, reps, stream, rtol=1e-10, max_cycles=40, graph_mode=1)
        out[name] = {"ms_per_solve": round(dt * 1e3, 3), "cycles": rep.cycles, "final_rel_residual": rep.r_final / rep.r0}
        del Sp
    return out


def leg_adapt(stream):
    """Mesh adaptation on the 20-sphere adaptive problem (16^3 blocks, to
    level 6): the leaves that a wider refinement band refines are flagged;
    time of the adapted geometry (unchanged blocks keep their records)
    against a setup from scratch of the same tree, and of carrying phi over."""
    import torch
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    narrow = W.spheres(refine_width=1.5)
    wide = W.spheres()
    G0 = octmg.Geometry(narrow.geom)
    target = {}
    for il in range(len(octmg.plan_levels(wide.geom))):
        pos, leaf = octmg.plan_blocks(wide.geom, il)
        for p_, lf in zip(pos, leaf):
            target[(il, *map(int, p_))] = int(lf)
    flags = np.array([1 if target.get(tuple(int(v) for v in lb), 1) == 0 else 0 for lb in G0.leaf_blocks()],
                     dtype=np.int8)
    S0 = octmg.State(G0)
    S0.set_boundary_fn(narrow.iface_value, narrow.domain_value)
    x0, _ = G0.leaf_coords()
    S0.set_rhs(narrow.rhs(x0))
    S0.solve(rtol=1e-10)
    torch.cuda.synchronize()
    t = time.perf_counter()
    G1, stats = G0.adapt(flags, reuse=True)
    t_adapt = time.perf_counter() - t
    t = time.perf_counter()
    G2, _ = G0.adapt(flags, reuse=False)
    t_scratch = time.perf_counter() - t
    S1 = octmg.State(G1)
    t = time.perf_counter()
    S1.remap_from(S0)
    t_remap = time.perf_counter() - t
    return {"workload": "20 spheres, 16^3 blocks to level 6: refinement band 1.5 -> 2.87 block widths in one step",
            "leaf_cells_before": int(G0.n_leaf), "leaf_cells_after": int(G1.n_leaf),
            "flagged_blocks": int(flags.sum()), "blocks_kept": int(stats[0]), "blocks_set_up": int(stats[1]),
            "records_kept": int(stats[2]), "records_computed": int(stats[3]),
            "adapt_s_reusing_records": round(t_adapt, 3), "adapt_s_from_scratch": round(t_scratch, 3),
            "remap_phi_s": round(t_remap, 4)}


def leg_2d(stream, steps=20):
    """2D 64^2 in 8^2 blocks, circle r=0.25, manufactured solution, FP64,
    V(2,2) to 1e-10 (launch-bound at this size)."""
    import torch
    from paper_2205_09411_amd import octmg
    from paper_2205_09411_amd import workloads as W
    w = W.mms2d(max_level=4)
    G = octmg.Geometry(w.geom)
    S = octmg.State(G)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    S.set_rhs(w.rhs(xyz))
    dt, rep = timed_solves(S, steps, stream, rtol=1e-10, max_cycles=40, graph_mode=1)
    hist = [rep.r0] + list(rep.history[:rep.cycles])
    factors = [hist[i + 1] / hist[i] for i in range(len(hist) - 1)]
    phi = S.get_solution()
    out = {"workload": "2D unit square 64^2 in 8^2 blocks, circle r=0.25, phi=sin(2 pi x)cos(3 pi y)+x^2",
           "ms_per_solve": round(dt * 1e3, 3), "cycles": rep.cycles,
           "residual_factor_per_cycle": [round(f, 4) for f in factors],
           "max_err_vs_exact": float(np.abs(phi - w.exact(xyz)).max())}
    if ORACLE_CHECKS:
        import oracle
        out["vs_oracle"] = vs_oracle(oracle.setup_workload(w), phi, rep.r0, cycles=10)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(o, w, n_cycles):
    """The oracle as it stands, timed on the host: n_cycles V-cycles with
    the OpenMP threads it runs with, then one V-cycle on one thread."""
    import oracle as orc
    threads = orc.get_threads()
    o.zero_solution()
    o.vcycle()  # warm
    levels = [o.level_info(i) for i in range(o.n_levels)]
    t0 = time.perf_counter()
    for _ in range(n_cycles):
        o.vcycle()
    dt = time.perf_counter() - t0
    upd = smoother_updates_per_vcycle(levels)
    orc.set_threads(1)
    t1 = time.perf_counter()
    o.vcycle()
    dt1 = time.perf_counter() - t1
    orc.set_threads(threads)
    return {"value": upd * n_cycles / dt / 1e6, "unit": "Mcell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_cycles} FAS V(2,2) cycles of the same {w.geom.name} problem (setup excluded), "
                      f"{dt:.1f} s, smoother updates on all levels / wall time; then 1 cycle on 1 thread, "
                      f"{dt1:.1f} s",
            "one_thread_value": upd / dt1 / 1e6, "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
            "oracle_build": "gcc -O3 -ffp-contract=off -fopenmp"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mms3d_256")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--cpu-cycles", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the comparisons of the results with the FP64 oracle (host CPU)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--block-order", type=int, default=None,
                    help="with --no-tune: block order of the 3D kernels (0 XCD ranges, 1 hardware, 2 octant walk)")
    ap.add_argument("--pair-max-blocks", type=int, default=None,
                    help="with --no-tune: largest launch (workgroups) of the 3D transfer and residual kernels "
                         "that takes the 512-thread colour-pair variants")
    ap.add_argument("--legs", default="mixed,batched,adaptive,serving,table1,2d,sharp,electrodes,adapt",
                    help="extra measurements after the headline: mixed,batched,adaptive,serving,table1,2d,sharp,"
                         "electrodes,adapt or none")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    global ORACLE_CHECKS
    ORACLE_CHECKS = not args.no_oracle
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2205_09411_amd import octmg

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_probe_mb:
        x = torch.ones(args.copy_probe_mb * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 8, "copies": 3}))
        return
    w = workload(args.workload)

    t = time.perf_counter()
    G = octmg.Geometry(w.geom)
    setup_s = time.perf_counter() - t
    levels = [G.level_info(i) for i in range(G.n_levels)]
    top = levels[-1]
    S = octmg.State(G)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    exact = w.exact(xyz)
    S.set_rhs(w.rhs(xyz))

    # launch configuration: the autotuner times every candidate (all give
    # identical iterates) and keeps the fastest
    if args.no_tune:
        if args.block_order is not None or args.pair_max_blocks is not None:
            S.set_launch(block_order=args.block_order or 0,
                         pair_max_blocks=(1 << 30) if args.pair_max_blocks is None else args.pair_max_blocks)
        tuned, cand_ms = S.get_launch(), []
    else:
        tuned, cand_ms = S.autotune(rtol=args.rtol, reps=2, stream=stream)
    gm = tuned["graph_mode"]
    for _ in range(args.warmup):
        S.solve(rtol=args.rtol, max_cycles=40, zero_start=True, stream=stream, graph_mode=gm)
    # kernel timing pass: eager launches, HIP events around the finest-level
    # sweeps on the solve's stream
    S.profile(True)
    S.profile_read()
    for _ in range(args.steps):
        S.solve(rtol=args.rtol, max_cycles=40, zero_start=True, stream=stream)
    prof = S.profile_read()
    S.profile(False)
    # timed region: whole solves in the tuned configuration
    torch.cuda.synchronize()
    # per-solve HIP events on the solve's stream (they add no synchronisation)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    reps = []
    ev[0].record(stream)
    for k in range(args.steps):
        reps.append(S.solve(rtol=args.rtol, max_cycles=40, zero_start=True, stream=stream, graph_mode=gm))
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    solve_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    copy_gbs = achievable_copy_gbs(torch, stream)
    phi = S.get_solution()
    err = float(np.abs(phi - exact).max())
    cycles = reps[-1].cycles
    updates = smoother_updates_per_vcycle(levels) * sum(r.cycles for r in reps)

    ncell = top["nblocks"] * top["Nb"] ** 3
    # algorithmic bytes of one FP64 half sweep: read the other colour's phi,
    # read g, write phi for half the cells (24 B per cell per red+black
    # step), plus the stencil record (64 B) and boundary term (8 B) of the
    # custom cells of that colour
    bytes_per_launch = 12.0 * ncell + 36.0 * top["nrec"]
    mean_ms = prof["finest_half_sweep_ms"] / max(1, prof["finest_half_sweeps"])
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    value = updates / dt / 1e6
    out = {
        "metric": "Mcell-updates/s per smoother sweep (% HBM peak); solves/s to 1e-10 rel; p99 lat",
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.geom.name}: 3D unit cube, {top['n']}^3 cells in 16^3 blocks, sphere r=0.3, "
                               "manufactured phi=exp(x)sin(pi y)cos(pi z), FP64, FAS V(2,2) to 1e-10 rel residual",
                   "cells_finest": ncell, "blocks": G.n_blocks, "levels": G.n_levels,
                   "interface_records": G.n_records, "rtol": args.rtol},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "k_gs_half3<double,16> (finest level)",
                     "bytes_per_launch": bytes_per_launch, "mean_launch_ms": round(mean_ms, 5),
                     "achievable_copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "solves_per_s": round(args.steps / dt, 3),
        "solve_ms_p10_p50_p90": [round(float(np.percentile(solve_ms, q)), 3) for q in (10, 50, 90)],
        "launch": {"chosen": tuned, "autotune_ms_per_solve": [round(v, 3) for v in cand_ms]},
        "cycles_per_solve": int(np.mean([r.cycles for r in reps])),
        # a V-cycle with its residual norm: the solve's time over its cycles
        # (the residual of phi = 0 that the test starts from is cached)
        "ms_per_vcycle": round(dt / sum(r.cycles for r in reps) * 1e3, 4),
        "final_rel_residual": max(r.r_final / r.r0 for r in reps),
        "max_err_vs_exact": err,
        "sweep_kernel_mcups": round(ncell / 2 / (mean_ms * 1e-3) / 1e6, 1),
        "setup_s": round(setup_s, 3),
    }
    legs = {}
    for leg in [x for x in args.legs.split(",") if x and x != "none"]:
        t = time.perf_counter()
        try:
            if leg == "mixed":
                legs[leg] = leg_mixed(G, w, phi, dt / args.steps, stream, args.steps, args.rtol, not args.no_tune)
            elif leg == "batched":
                legs[leg] = leg_batched(stream, args.rtol)
            elif leg == "adaptive":
                legs[leg] = leg_adaptive(stream, args.rtol)
            elif leg == "serving":
                legs[leg] = leg_serving(stream)
            elif leg == "table1":
                legs[leg] = leg_table1(stream)
            elif leg == "2d":
                legs[leg] = leg_2d(stream)
            elif leg == "sharp":
                legs[leg] = leg_sharp(stream)
            elif leg == "electrodes":
                legs[leg] = leg_electrodes(stream)
            elif leg == "adapt":
                legs[leg] = leg_adapt(stream)
            else:
                raise ValueError(f"unknown leg {leg}")
        except Exception as e:  # a failed leg is reported, the headline stands
            legs[leg] = {"error": f"{type(e).__name__}: {e}"}
        legs[leg]["leg_wall_s"] = round(time.perf_counter() - t, 1)
        print(f"leg {leg} done in {legs[leg]['leg_wall_s']} s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if legs:
        out["legs"] = legs
    if ORACLE_CHECKS or not args.no_cpu_baseline:
        import oracle
        o = oracle.setup_workload(w)
        if ORACLE_CHECKS:
            r0 = reps[-1].r0
            out["vs_oracle"] = {"fp64": vs_oracle(o, phi, r0)}
            if "phi" in MIXED_PHI:
                legs["mixed"]["vs_oracle"] = vs_oracle(o, MIXED_PHI["phi"], r0)
            print("oracle comparisons done", file=sys.stderr, flush=True)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(o, w, args.cpu_cycles)
        del o
    print(json.dumps(out), flush=True)
    octmg.close_all()  # release every device object before the interpreter exits


if __name__ == "__main__":
    main()
