"""Captured solves (graph_mode 1: one HIP graph per cycle, replayed; 2: the
whole solve as one graph with the convergence test on the device) give the
same iterates, bit for bit, and the same cycle counts as eager launches.

Each graph is replayed several times with the program's own eager work and
synchronisations between the replays, and every replay is checked against
the eager result."""
import numpy as np
import pytest
import torch

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu


def state(w, n_rhs=1, precision=octmg.FP64, n_rhs_distinct=True):
    G = octmg.Geometry(w.geom)
    S = octmg.State(G, n_rhs, precision)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    if n_rhs == 1:
        S.set_rhs(w.rhs(xyz))
    else:
        S.set_rhs(np.stack([w.rhs(xyz, i) for i in range(n_rhs)]))
    return G, S


def eager_then_graph(S, mode, kind=octmg.CYCLE_V, stream=None, replays=3, max_cycles=40):
    rep = S.solve(rtol=1e-10, max_cycles=max_cycles, kind=kind, zero_start=True, stream=stream)
    ref = S.get_solution()
    ref_hist = list(rep.history[:rep.cycles])
    for k in range(replays):
        # eager work between the replays
        S.zero_solution()
        S.cycle(octmg.CYCLE_V)
        _ = S.residual_norm()
        torch.cuda.synchronize()
        r = S.solve(rtol=1e-10, max_cycles=max_cycles if mode == 1 else rep.cycles + 2, kind=kind,
                    zero_start=True, stream=stream, graph_mode=mode)
        assert r.cycles == rep.cycles, (k, r.cycles, rep.cycles)
        assert list(r.history[:r.cycles]) == ref_hist, k
        got = S.get_solution()
        assert np.array_equal(got, ref), (k, np.abs(got - ref).max())
    return rep


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_fp64_matches_eager(mode):
    print("graph fp64 mode", mode, flush=True)
    _, S = state(W.mms3d(max_level=3, block_n=16))
    rep = eager_then_graph(S, mode, stream=torch.cuda.Stream())
    assert rep.status == 0


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_null_stream_and_fmg(mode):
    print("graph null stream fmg mode", mode, flush=True)
    _, S = state(W.mms2d(max_level=4))
    eager_then_graph(S, mode, kind=octmg.CYCLE_FMG, stream=None)


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_mixed_precision(mode):
    print("graph mixed mode", mode, flush=True)
    _, S = state(W.mms3d(max_level=3, block_n=16), precision=octmg.MIXED)
    eager_then_graph(S, mode)


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_batched_adaptive(mode):
    """Several right-hand sides converging after different cycle counts on an
    adaptive grid: frozen rhs stay frozen inside the captured solve."""
    print("graph batched adaptive mode", mode, flush=True)
    w = W.spheres(n_spheres=5, max_level=5, block_n=8, seed=9)
    G = octmg.Geometry(w.geom)
    S = octmg.State(G, 3)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    g = np.stack([w.rhs(xyz), 1e-3 * w.rhs(xyz) + np.sin(7 * xyz[:, 0]), np.cos(3 * xyz[:, 1])])
    S.set_rhs(g)
    eager_then_graph(S, mode, replays=2)


def test_graph_rebuilt_after_smoothing_change():
    print("graph rebuilt after smoothing change", flush=True)
    _, S = state(W.mms3d(max_level=3, block_n=8))
    eager_then_graph(S, 1, replays=1)
    S.set_smoothing(3, 3)
    eager_then_graph(S, 1, replays=2)
    S.set_smoothing(2, 2)
    eager_then_graph(S, 2, replays=1)


def test_graph_rejects_fused_levels():
    _, S = state(W.mms3d(max_level=3, block_n=8))
    S.set_fused_levels(64)
    with pytest.raises(octmg.OctmgError):
        S.solve(rtol=1e-10, graph_mode=1)
    S.set_fused_levels(0)
    S.solve(rtol=1e-10, graph_mode=1, zero_start=True)


def test_launch_configurations_and_autotune_identical():
    """Every launch configuration the autotuner picks from gives the same
    iterates bit for bit; the autotuner keeps one of them."""
    print("launch configurations and autotune", flush=True)
    w = W.cylinder(max_level=3)
    G = octmg.Geometry(w.geom)
    S = octmg.State(G, 3, octmg.MIXED)
    S.set_boundary(None, np.zeros(G.n_domain))
    xyz, _ = G.leaf_coords()
    S.set_rhs(np.stack([w.rhs(xyz, i) for i in range(3)]))
    ref_rep = S.solve(rtol=1e-10, zero_start=True)
    ref = S.get_solution()
    configs = [dict(block_order=o, bottom_kind=b, bottom_max_blocks=m, graph_mode=g, pair_max_blocks=1 << 30,
                    prolong_fused=1, red_preset=1, update_fused=1)
               for o in (0, 1, 2) for (b, m, g) in ((0, 0, 0), (0, 0, 1), (0, 0, 2), (1, 8, 0), (1, 64, 0))]
    # the 512-thread kernels on no level, on the levels of at most 64 blocks;
    # prolongation and red half sweep as separate launches; the mixed
    # defect without the first red half sweep; the FP64 update apart from
    # the last black half sweep
    configs += [dict(block_order=0, bottom_kind=0, bottom_max_blocks=0, graph_mode=g, pair_max_blocks=p,
                     prolong_fused=f, red_preset=r, update_fused=u)
                for p in (0, 64) for g in (0, 2) for f in (0, 1) for (r, u) in ((0, 0), (1, 1), (1, 0))]
    for c in configs:
        S.set_launch(**c)
        assert S.get_launch() == c
        r = S.solve(rtol=1e-10, zero_start=True, graph_mode=c["graph_mode"], max_cycles=ref_rep.cycles + 1)
        assert r.cycles == ref_rep.cycles, c
        assert np.array_equal(S.get_solution(), ref), c
    best, ms = S.autotune(rtol=1e-10, reps=1)
    print("autotune", best, ms, flush=True)
    assert len(ms) == 16 and all(m > 0 for m in ms)
    assert S.get_launch() == best
    assert np.array_equal(S.get_solution(), ref)
    with pytest.raises(octmg.OctmgError):
        S.set_launch(bottom_kind=1, bottom_max_blocks=8, graph_mode=1)


@pytest.mark.parametrize("precision", [octmg.FP64, octmg.MIXED])
def test_thread_variants_identical_adaptive(precision):
    """The 512-lane kernels (every launch), the 256-lane kernels (none) and a
    mix (levels of at most 64 blocks) give the same iterates, bit for bit, on
    an adaptive octree with refinement-boundary ghosts, 16^3 and 8^3 blocks."""
    print("thread variants, adaptive", precision, flush=True)
    for bn in (16, 8):
        w = W.spheres(n_spheres=6, max_level=5, block_n=bn, refine_width=1.0)
        G, S = state(w, 2 if precision == octmg.MIXED else 1, precision)
        assert any(G.level_info(i)["nleaf"] not in (0, G.level_info(i)["nblocks"]) for i in range(G.n_levels))
        ref = None
        for p in (1 << 30, 0, 64):
            S.set_launch(pair_max_blocks=p)
            r = S.solve(rtol=1e-10, zero_start=True)
            sol = S.get_solution()
            if ref is None:
                ref, ref_cycles = sol, r.cycles
            assert r.cycles == ref_cycles, p
            assert np.array_equal(sol, ref), p


@pytest.mark.parametrize("max_cycles", [17, 40])
def test_whole_solve_graph_in_chunks(max_cycles):
    """Graph mode 2 replays a captured chunk of 8 cycles when max_cycles is
    above 16: the same cycles, norms and solution bits as eager launches,
    also when the solve stops at max_cycles inside a chunk (rtol out of
    reach)."""
    print("graph mode 2 in chunks, max_cycles", max_cycles, flush=True)
    _, S = state(W.cylinder(max_level=3), n_rhs=3)
    for rtol in (1e-10, 1e-14):
        ra = S.solve(rtol=rtol, max_cycles=max_cycles, zero_start=True, graph_mode=0, raise_on_fail=False)
        a = S.get_solution()
        rb = S.solve(rtol=rtol, max_cycles=max_cycles, zero_start=True, graph_mode=2, raise_on_fail=False)
        b = S.get_solution()
        if ra.status == octmg.ERR_NOT_CONVERGED and ra.cycles < max_cycles:
            continue  # the eager loop's stall test stopped it (graph mode 2 has none)
        assert ra.status == rb.status and ra.cycles == rb.cycles, (rtol, ra.cycles, rb.cycles)
        assert ra.r_final == rb.r_final
        assert np.array_equal(a, b), rtol


def test_graph_chunk_from_previous_solve():
    """Graph mode 2's first chunk has as many cycles as the state's previous
    solve: too few (a looser rtol before a tighter one: one-cycle chunks
    follow) and too many (a tighter rtol before a looser one: the extra
    cycles exit at once) give the cycles, norms and bits of eager launches
    on another state, for three distinct rhs; a solve cut off at max_cycles
    sets no hint."""
    print("graph mode 2 chunk from the previous solve", flush=True)
    w = W.cylinder(max_level=3)
    _, A = state(w, n_rhs=3)
    _, B = state(w, n_rhs=3)
    for rtol in (1e-5, 1e-11, 1e-5, 1e-8):
        ra = A.solve(rtol=rtol, max_cycles=30, zero_start=True, graph_mode=0)
        rb = B.solve(rtol=rtol, max_cycles=30, zero_start=True, graph_mode=2)
        assert ra.cycles == rb.cycles and ra.r_final == rb.r_final, (rtol, ra.cycles, rb.cycles)
        assert np.array_equal(ra.per_rhs["cycles"], rb.per_rhs["cycles"]), rtol
        assert np.array_equal(ra.per_rhs["r_final"], rb.per_rhs["r_final"]), rtol
        assert np.array_equal(A.get_solution(), B.get_solution()), rtol
    # a solve cut off at max_cycles leaves no hint: the next one starts with
    # the default chunk
    ra = A.solve(rtol=1e-11, max_cycles=3, zero_start=True, graph_mode=0, raise_on_fail=False)
    rb = B.solve(rtol=1e-11, max_cycles=3, zero_start=True, graph_mode=2, raise_on_fail=False)
    assert ra.status == rb.status == octmg.ERR_NOT_CONVERGED and ra.cycles == rb.cycles == 3
    assert ra.r_final == rb.r_final and np.array_equal(A.get_solution(), B.get_solution())
    ra = A.solve(rtol=1e-8, max_cycles=30, zero_start=True, graph_mode=0)
    rb = B.solve(rtol=1e-8, max_cycles=30, zero_start=True, graph_mode=2)
    assert ra.cycles == rb.cycles and ra.r_final == rb.r_final
    assert np.array_equal(A.get_solution(), B.get_solution())
