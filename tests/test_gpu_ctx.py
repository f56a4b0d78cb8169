"""Contexts (octmg_ctx): every device buffer of a geometry, its states and
their calls' temporaries comes from the context's allocator (here PyTorch's
caching allocator through a callback) with the same results as hipMalloc;
the tune cache records the autotuner's choice and serves it to the next
state of the same problem without timing."""
import os

import numpy as np
import pytest
import torch

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu


def solve(G, w, n_rhs=2, precision=octmg.MIXED):
    S = octmg.State(G, n_rhs, precision)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    S.set_rhs(np.stack([w.rhs(xyz, i) for i in range(n_rhs)]))  # host buffer: staged through a temporary
    rep = S.solve(rtol=1e-10, zero_start=True, graph_mode=1)
    return S, rep, S.get_solution()


def test_allocator_serves_every_buffer():
    w = W.cylinder(max_level=3)
    ref_S, ref_rep, ref = solve(octmg.Geometry(w.geom), w)
    alloc = octmg.TorchAllocator()
    ctx = octmg.Context(0, allocator=alloc)
    before = torch.cuda.memory_allocated()
    G = octmg.Geometry(w.geom, ctx=ctx)
    g_bytes = alloc.bytes_held()
    assert g_bytes >= G.device_bytes > 0
    S, rep, got = solve(G, w)
    assert alloc.bytes_held() > g_bytes  # the state's fields
    assert torch.cuda.memory_allocated() - before >= alloc.bytes_held()
    assert rep.cycles == ref_rep.cycles and np.array_equal(got, ref)
    # an adapted geometry allocates from the same context
    flags = np.zeros(G.n_leaf_blocks, dtype=np.int8)
    flags[:8] = 1
    Ga, _ = G.adapt(flags)
    held = alloc.bytes_held()
    S.close()
    G.close()
    ctx.close()  # the adapted geometry keeps the context alive
    assert 0 < alloc.bytes_held() < held
    Sa = octmg.State(Ga)
    Sa.set_boundary_fn(w.iface_value, w.domain_value)
    xa, _ = Ga.leaf_coords()
    Sa.set_rhs(w.rhs(xa, 0))
    assert Sa.solve(rtol=1e-10, zero_start=True).status == 0
    Sa.close()
    Ga.close()
    assert alloc.bytes_held() == 0


def test_tune_cache_serves_the_next_state(tmp_path):
    path = str(tmp_path / "tune.txt")
    w = W.cylinder(max_level=3)
    ctx = octmg.Context(0, tune_cache=path)
    G = octmg.Geometry(w.geom, ctx=ctx)
    S, _, ref = solve(G, w, n_rhs=2)
    best, ms = S.autotune(rtol=1e-10, reps=1)
    assert len(ms) == 16 and os.path.exists(path)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and "\t" in lines[0]
    S2, _, _ = solve(G, w, n_rhs=2)
    best2, ms2 = S2.autotune(rtol=1e-10, reps=1)
    assert ms2 == [] and best2 == best and S2.get_launch() == best
    assert len(open(path).read().splitlines()) == 1
    # another problem (one rhs) is timed and recorded as a second line
    S3, _, _ = solve(G, w, n_rhs=1)
    _, ms3 = S3.autotune(rtol=1e-10, reps=1)
    assert len(ms3) == 16 and len(open(path).read().splitlines()) == 2
