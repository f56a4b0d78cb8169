"""Serving engine: every request's result equals a one-rhs solve of the same
problem alone (same cycles, identical solution), whatever else is batched or
in flight; budget admission, lane reuse, state release and error results."""
import time

import numpy as np
import pytest
import torch

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu


def geometry(n_spheres, seed, max_level):
    w = W.spheres(n_spheres=n_spheres, max_level=max_level, block_n=16, seed=seed, adaptive=False)
    G = octmg.Geometry(w.geom)
    return w, G


def wait_all(server, ids, timeout=120.0):
    got = {}
    t = time.perf_counter()
    while len(got) < len(ids):
        for r in server.poll():
            got[r["id"]] = r
        assert time.perf_counter() - t < timeout, f"{len(got)} of {len(ids)} results after {timeout} s"
        time.sleep(0.001)
    return got


def alone(G, w, g, precision, rtol, max_cycles=40):
    S = octmg.State(G, 1, precision)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    S.set_rhs(g)
    rep = S.solve(rtol=rtol, max_cycles=max_cycles, zero_start=True, raise_on_fail=False)
    return rep, S.get_solution()


@pytest.mark.parametrize("precision", [octmg.FP64, octmg.MIXED])
def test_results_equal_solves_alone(precision):
    print("server parity precision", precision, flush=True)
    geoms = [geometry(1, 500, 2), geometry(5, 501, 3), geometry(10, 502, 3)]
    lane = max(octmg_lane_bytes(G, precision) for _, G in geoms)
    # room for about one 4-lane state of the larger grids: forces waiting and state release
    server = octmg.Server(hbm_budget_bytes=5 * lane, max_lanes=4, precision=precision)
    slots = [server.add_geometry(G, w.iface_value(G.iface_points()), w.domain_value(G.domain_points()))
             for w, G in geoms]
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(14):
        k = int(rng.integers(0, 3))
        w, G = geoms[k]
        xyz, _ = G.leaf_coords()
        g = W.gaussian_sources(xyz, 10000 + i)
        out = np.full(G.n_leaf, np.nan)
        rtol = 1e-8 if i % 3 else 1e-10
        rid = server.submit(slots[k], g, out, rtol)
        reqs.append((rid, k, g, out, rtol))
        if i % 5 == 4:
            time.sleep(0.002)  # let some requests start before the next arrive
    got = wait_all(server, [r[0] for r in reqs])
    st = server.stats()
    server.close()
    print("stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["states_released"] >= 1
    assert st["peak_bytes"] <= 5 * lane
    for rid, k, g, out, rtol in reqs:
        w, G = geoms[k]
        rep, ref = alone(G, w, g, precision, rtol)
        r = got[rid]
        assert r["status"] == 0 and rep.status == 0
        assert r["cycles"] == rep.cycles, (rid, r["cycles"], rep.cycles)
        assert r["r0"] == rep.r0 and r["r_final"] == rep.r_final
        assert np.array_equal(out, ref), (rid, np.abs(out - ref).max())
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def octmg_lane_bytes(G, precision):
    cells = sum(G.level_info(i)["nblocks"] * G.level_info(i)["Nb"] ** 3 for i in range(G.n_levels))
    return cells * (24 + (12 if precision == octmg.MIXED else 0))


def test_device_buffers_budget_and_errors():
    print("server device buffers, budget, errors", flush=True)
    small_w, small = geometry(1, 500, 2)
    big_w, big = geometry(5, 501, 3)
    budget = 2 * octmg_lane_bytes(small, octmg.MIXED)
    assert octmg_lane_bytes(big, octmg.MIXED) > budget
    server = octmg.Server(hbm_budget_bytes=budget, max_lanes=8, precision=octmg.MIXED)
    s_small = server.add_geometry(small, small_w.iface_value(small.iface_points()),
                                  small_w.domain_value(small.domain_points()))
    s_big = server.add_geometry(big, big_w.iface_value(big.iface_points()), big_w.domain_value(big.domain_points()))
    xyz, _ = small.leaf_coords()
    g = torch.tensor(W.gaussian_sources(xyz, 7), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(g)
    bad = g.clone()
    bad[11] = float("nan")
    out_bad = torch.zeros_like(g)
    xb, _ = big.leaf_coords()
    gb = W.gaussian_sources(xb, 8)
    ob = np.zeros(big.n_leaf)
    torch.cuda.synchronize()
    ids = [server.submit(s_small, g, out, 1e-8), server.submit(s_small, bad, out_bad, 1e-8),
           server.submit(s_big, gb, ob, 1e-8)]
    got = wait_all(server, ids)
    server.close()
    assert got[ids[0]]["status"] == 0
    assert got[ids[1]]["status"] == octmg.ERR_NONFINITE
    assert got[ids[2]]["status"] == octmg.ERR_BUDGET
    rep, ref = alone(small, small_w, g.cpu().numpy(), octmg.MIXED, 1e-8)
    assert np.array_equal(out.cpu().numpy(), ref) and got[ids[0]]["cycles"] == rep.cycles


def test_invalid_server_arguments():
    with pytest.raises(octmg.OctmgError):
        octmg.Server(max_lanes=0)
    with pytest.raises(octmg.OctmgError):
        octmg.Server(hbm_budget_bytes=0)
    server = octmg.Server()
    with pytest.raises(octmg.OctmgError):
        server.submit(3, np.zeros(8), np.zeros(8), 1e-8)
    server.close()


def inverse_norm(orc, w):
    """|A^-1 1|_inf from the oracle (A u = 1, zero boundary data): |A^-1|_inf
    of the M-matrix operator of a uniform tree."""
    o = orc.Oracle(w.geom)
    o.set_boundary(np.zeros(len(o.iface_points())), np.zeros(len(o.domain_points())))
    o.set_rhs(np.ones(o.n_leaf))
    o.solve(rtol=1e-12, max_cycles=60)
    return float(np.abs(o.get_solution()).max())


@pytest.mark.parametrize("precision", [octmg.FP64, octmg.MIXED])
def test_served_results_against_oracle(orc, precision):
    """Each served result against the oracle's converged solution of the same
    rhs: its residual, recomputed by the oracle, meets the request's rtol, and
    |phi - phi*|_inf <= 2 |A^-1|_inf (|r_served| + |r_oracle|) (both solve the
    same discrete system up to their residuals; factor 2 as margin)."""
    print("served results vs oracle, precision", precision, flush=True)
    geoms = [geometry(1, 500, 2), geometry(5, 501, 3)]
    server = octmg.Server(max_lanes=4, precision=precision)
    slots = [server.add_geometry(G, w.iface_value(G.iface_points()), w.domain_value(G.domain_points()))
             for w, G in geoms]
    reqs = []
    for i in range(6):
        k = i % 2
        w, G = geoms[k]
        xyz, _ = G.leaf_coords()
        g = W.gaussian_sources(xyz, 10000 + i)
        out = np.full(G.n_leaf, np.nan)
        reqs.append((server.submit(slots[k], g, out, 1e-8), k, g, out))
    got = wait_all(server, [r[0] for r in reqs])
    server.close()
    ora = []
    for w, G in geoms:
        o = orc.Oracle(w.geom)
        o.set_boundary(w.iface_value(o.iface_points()), w.domain_value(o.domain_points()))
        ora.append((o, inverse_norm(orc, w)))
    for rid, k, g, out in reqs:
        o, ainv = ora[k]
        assert got[rid]["status"] == 0
        o.set_rhs(g)
        o.zero_solution()
        r0, _ = o.solve(rtol=1e-13, max_cycles=60)
        ref, r_o = o.get_solution(), o.residual_max()
        r_s = float(np.abs(o.leaf_residual(out)).max())
        assert r_s <= 1.01e-8 * r0, (rid, r_s, r0)
        err = float(np.abs(out - ref).max())
        bound = 2.0 * ainv * (r_s + r_o)
        print(f"  request {rid}: cycles {got[rid]['cycles']}, |err| {err:.2e}, bound {bound:.2e}")
        assert err <= bound, (rid, err, bound)


def test_exit_with_open_handles():
    """A program that ends with a server (worker thread running), states with
    captured graphs and geometries still open exits cleanly: the binding
    closes them before the interpreter and the HIP runtime shut down."""
    import os
    import subprocess
    import sys
    code = (
        "import numpy as np\n"
        "from paper_2205_09411_amd import octmg, workloads as W\n"
        "w = W.spheres(n_spheres=1, max_level=2, block_n=16, seed=500, adaptive=False)\n"
        "G = octmg.Geometry(w.geom)\n"
        "S = octmg.State(G, 2, octmg.MIXED)\n"
        "S.set_boundary_fn(w.iface_value, w.domain_value)\n"
        "xyz, _ = G.leaf_coords()\n"
        "S.set_rhs(np.stack([W.gaussian_sources(xyz, 1), W.gaussian_sources(xyz, 2)]))\n"
        "S.solve(rtol=1e-8, zero_start=True, graph_mode=1)\n"
        "srv = octmg.Server(max_lanes=2)\n"
        "slot = srv.add_geometry(G, w.iface_value(G.iface_points()), w.domain_value(G.domain_points()))\n"
        "out = np.zeros(G.n_leaf)\n"
        "srv.submit(slot, W.gaussian_sources(xyz, 3), out, 1e-8)\n"
        "print('exiting with open handles', flush=True)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=100)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "exiting with open handles" in r.stdout
