"""Host-side emulation of the kernels' tile geometry (test helper).

A backward or forward tile is one wave over 64 consecutive sample columns.
Its control-column range runs from the first lane's v-span minus q to the
last active lane's v-span, so it spans ``nkeys + q`` columns, where
``nkeys = klast - kfirst + 1`` counts every span between the two, sampled or
not.  The kernels then choose, per tile:

* the staged row loop when ``320 // ncols >= p + 1`` control rows of the
  column range fit the wave's 320-entry LDS block, else the loop that reads
  control points from global memory;
* one flush-gather pass when ``nkeys + QM <= 64`` (QM is the compiled
  maximum degree in v: q for the uniform-batch kernels, 5 or 7 for the
  persistent plan kernels), else one pass per 64 control columns.

The spans come from the oracle's own span search, so this module restates
only the tiling rules, none of the method's arithmetic.
"""
import numpy as np

from oracle import oracle as O

WAVE = 64
BLOCK_CAP = 320


def tiles(ku, kv, p, q, nu_c, nv_c, us, vs, qm):
    """Per 64-column block: dict(ncols, nkeys, staged, passes)."""
    out = []
    kvd = np.asarray(kv, np.float64)
    spans = [O.find_span(kvd, q, float(x)) for x in np.asarray(vs, np.float32)]
    for c0 in range(0, len(vs), WAVE):
        blk = spans[c0:c0 + WAVE]
        nkeys = blk[-1] - blk[0] + 1
        ncols = nkeys + q
        staged = BLOCK_CAP // ncols >= p + 1
        wide = nkeys + qm > WAVE
        passes = (ncols + WAVE - 1) // WAVE if wide else 1
        out.append(dict(ncols=ncols, nkeys=nkeys, staged=staged, passes=passes))
    return out


def plan_class(max_degree):
    """Compiled maximum degree of the persistent kernels a plan uses."""
    return 5 if max_degree <= 5 else 7
