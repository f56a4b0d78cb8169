"""A C99 program drives the library through include/octmg.h alone
(tests/abi_client.c): the header compiles as strict C with every warning an
error, the program links against liboctmg.so, its host-only tree planning
equals the oracle's tree, and (GPU) it solves the 64^3 manufactured sphere
problem, with the built-in level set and with the same level set given as a
C function, in the cycles the Python binding's solve takes, bit for bit
equal between the two."""
import os
import subprocess

import numpy as np
import pytest

from paper_2205_09411_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2205_09411_amd")
LIB = os.path.join(PKG, "liboctmg.so")


def build_client(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("liboctmg.so is not built")
    exe = str(tmp_path / "abi_client")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-pedantic", "-ffp-contract=off",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_client.c"), "-o", exe,
           "-L", PKG, "-loctmg", "-lm", "-Wl,-rpath," + PKG]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_client_plans_the_oracle_tree(tmp_path, orc):
    exe = build_client(tmp_path)
    r = subprocess.run([exe, "plan"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    n_levels = int(lines[0].split()[1])
    o = orc.Oracle(W.mms3d(max_level=5, block_n=16).geom)
    assert n_levels == o.n_levels
    for il in range(n_levels):
        f = lines[1 + il].split()
        info = o.level_info(il)
        assert int(f[3]) == info["n"] and int(f[5]) == info["Nb"] and int(f[7]) == info["nblocks"], (il, f, info)


@pytest.mark.gpu
def test_c_client_solves(tmp_path):
    from paper_2205_09411_amd import octmg
    exe = build_client(tmp_path)
    print("C client solve", flush=True)
    r = subprocess.run([exe, "solve"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr)
    f = r.stdout.split()
    out = dict(zip(f[0::2], f[1::2]))
    print(r.stdout, flush=True)
    w = W.mms3d(max_level=3, block_n=16)
    G = octmg.Geometry(w.geom)
    S = octmg.State(G)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    S.set_rhs(w.rhs(xyz))
    rep = S.solve(rtol=1e-10, zero_start=True)
    err = float(np.abs(S.get_solution() - w.exact(xyz)).max())
    assert int(out["leaf"]) == G.n_leaf
    assert int(out["cycles"]) == rep.cycles and int(out["callback_cycles"]) == rep.cycles
    assert int(out["callback_bitwise_equal"]) == 1
    assert abs(float(out["err"]) - err) <= 1e-12 + 1e-6 * err
