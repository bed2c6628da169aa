"""Per-surface parity cases shared by the GPU tests and the CPU checks of
which kernel paths they reach (seeded inputs only, none of the method's
arithmetic)."""
import numpy as np

from paper_2104_14547_amd import workloads as W


def one_surface(seed, p, q, nu_c, nv_c, nu_s, nv_s, repeat=0.0, on_knots=False, clustered=False):
    g = np.random.Generator(np.random.PCG64(seed))
    d = dict(p=p, q=q, nu_c=nu_c, nv_c=nv_c, nu_s=nu_s, nv_s=nv_s)
    d["ctrl"] = W.perturbed_lattice(g, nu_c, nv_c)
    d["w"] = g.uniform(0.5, 1.5, (nu_c, nv_c)).astype(np.float32)
    d["ku"] = W.clamped_random_knots(g, nu_c, p, repeat)
    d["kv"] = W.clamped_random_knots(g, nv_c, q, repeat)
    if clustered:
        n_int = nu_c - p - 1
        d["ku"][p + 1:p + 1 + n_int] = (0.4 + 2e-5 * np.arange(n_int)).astype(np.float32)
    d["us"] = W.uniform_grid(nu_s)
    d["vs"] = W.uniform_grid(nv_s)
    if on_knots:
        ku_in = np.unique(d["ku"])
        d["us"] = np.sort(np.concatenate([d["us"][:max(nu_s - len(ku_in), 0)], ku_in]))[:nu_s].astype(np.float32)
        kv_in = np.unique(d["kv"])
        d["vs"] = np.sort(np.concatenate([d["vs"][:max(nv_s - len(kv_in), 0)], kv_in]))[:nv_s].astype(np.float32)
    d["upstream"] = g.uniform(-0.1, 0.1, (nu_s, nv_s, 3)).astype(np.float32)
    return d


EDGE = [
    # (p, q, nu_c, nv_c, nu_s, nv_s, repeat, on_knots, clustered)
    (1, 1, 2, 2, 1, 1, 0.0, False, False),
    (1, 2, 3, 5, 7, 3, 0.0, False, False),
    (3, 3, 4, 4, 64, 64, 0.0, False, False),      # Bezier patch, exactly one column block
    (2, 3, 30, 40, 10, 13, 0.0, False, False),    # samples sparser than spans
    (5, 5, 6, 9, 130, 200, 0.3, False, False),    # ragged row tiles and column blocks
    (7, 7, 8, 9, 65, 129, 0.0, False, False),     # degree-7 class
    (3, 2, 9, 9, 257, 65, 0.3, True, False),      # samples on knots, repeated knots
    (4, 1, 12, 3, 33, 300, 0.4, True, False),
    (3, 3, 12, 12, 40, 40, 0.0, False, True),     # clustered knots
    (6, 2, 40, 48, 20, 250, 0.2, False, False),
    # kernel paths the workloads above never reach (checked by test_kernel_paths):
    (7, 7, 20, 48, 40, 48, 0.0, False, False),    # control rows read from global memory (block too narrow for p+1 rows)
    (3, 3, 10, 120, 30, 40, 0.0, False, False),   # sparse samples: two gather passes, global reads
    (3, 3, 12, 200, 20, 64, 0.1, False, False),   # four gather passes (> 128 control columns), global reads
    (2, 7, 9, 180, 17, 70, 0.0, False, False),    # degree-7 columns, three gather passes, ragged column block
    (1, 3, 20, 100, 40, 64, 0.0, False, False),   # two gather passes with control rows staged in LDS
    (1, 7, 3, 248, 5, 64, 0.0, False, False),     # the longest knot vector accepted (256 entries)
]
