"""The GPU parity cases reach every row-loop and gather path of the kernels.

Checked on the CPU by emulating the tile geometry (tests/tile_geometry.py)
on the cases' own inputs, for the uniform-batch kernels (compiled maximum
degree in v = q) and the persistent plan kernels (5 or 7)."""
import numpy as np

from tests import tile_geometry as G
from tests.cases import EDGE, one_surface


def case_tiles(i):
    p, q, nu_c, nv_c, nu_s, nv_s, rep, on_knots, clustered = EDGE[i]
    out = []
    for j in range(2):
        d = one_surface(1000 * i + j, p, q, nu_c, nv_c, nu_s, nv_s, rep, on_knots, clustered)
        if j == 1:  # the parity test shares the first surface's samples
            d0 = one_surface(1000 * i, p, q, nu_c, nv_c, nu_s, nv_s, rep, on_knots, clustered)
            d["us"], d["vs"] = d0["us"], d0["vs"]
        for qm in (q, G.plan_class(max(p, q))):
            out += G.tiles(d["ku"], d["kv"], p, q, nu_c, nv_c, d["us"], d["vs"], qm)
    return out


def test_each_path_is_reached():
    per_case = [case_tiles(i) for i in range(len(EDGE))]
    flat = [t for ts in per_case for t in ts]
    assert any(not t["staged"] for t in flat), "no case reads control rows from global memory"
    assert any(t["staged"] and t["passes"] >= 2 for t in flat), "no staged case with several gather passes"
    assert any(t["passes"] >= 3 for t in flat), "no case with more than 128 control columns"
    assert max(t["passes"] for t in flat) == 4
    assert any(t["staged"] and t["passes"] == 1 for t in flat)


def test_named_cases_take_their_paths():
    def find(p, q, nu_c, nv_c):
        for i, e in enumerate(EDGE):
            if e[:4] == (p, q, nu_c, nv_c):
                return case_tiles(i)
        raise KeyError((p, q, nu_c, nv_c))
    assert all(not t["staged"] for t in find(7, 7, 20, 48))
    t = find(3, 3, 12, 200)
    assert all(t_["ncols"] > 128 and t_["passes"] >= 3 and not t_["staged"] for t_ in t)
    t = find(1, 3, 20, 100)
    assert all(t_["staged"] and t_["passes"] == 2 for t_ in t)
    t = find(1, 7, 3, 248)
    assert max(t_["ncols"] for t_ in t) > 192


def test_workload_tiles_stay_on_the_common_paths():
    """The uneven batch's own tiles are staged and single-pass: the extra
    cases above are what covers the other paths."""
    from paper_2104_14547_amd import workloads as W
    b = W.uneven_batch(3, n_surf=256, with_upstream=False)
    for s in range(b.n):
        d = b.surface(s)
        for t in G.tiles(d["ku"], d["kv"], d["p"], d["q"], d["nu_c"], d["nv_c"], d["us"], d["vs"], 5):
            assert t["passes"] == 1
            assert t["ncols"] <= 64
