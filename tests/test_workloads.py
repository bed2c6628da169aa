"""The seeded generators: determinism, packing, and the stated recipes."""
import math

import numpy as np

from paper_2104_14547_amd import workloads as W


def test_deterministic_per_seed():
    a, b = W.batch_bicubic(1, n_surf=8), W.batch_bicubic(1, n_surf=8)
    for k in ("ctrl", "w", "ku", "kv", "us", "vs", "target"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = W.batch_bicubic(2, n_surf=8)
    assert not np.array_equal(a.ctrl, c.ctrl)


def test_single_bicubic_recipe():
    b = W.single_bicubic(0)
    s = b.surface(0)
    assert (s["p"], s["q"], s["nu_c"], s["nv_c"], s["nu_s"], s["nv_s"]) == (3, 3, 8, 8, 64, 64)
    assert np.allclose(s["ctrl"][:, :, 0], np.arange(8)[:, None] / 7)
    assert np.abs(s["ctrl"][..., 2]).max() <= 0.2
    assert s["w"].min() >= 0.5 and s["w"].max() <= 1.5
    assert list(s["ku"]) == [0, 0, 0, 0, np.float32(.2), np.float32(.4), np.float32(.6), np.float32(.8), 1, 1, 1, 1]
    assert s["us"][0] == 0 and s["us"][-1] == 1 and s["us"].dtype == np.float32


def test_packing_roundtrip():
    b = W.uneven_batch(3, n_surf=32)
    sub = b.subset([5, 2, 17])
    for new, old in enumerate([5, 2, 17]):
        x, y = sub.surface(new), b.surface(old)
        for k in ("ctrl", "w", "ku", "kv", "us", "vs", "upstream"):
            assert np.array_equal(x[k], y[k])


def test_uneven_batch_distribution():
    b = W.uneven_batch(3, n_surf=4096, with_upstream=False)
    s = b.shapes.astype(np.int64)
    assert s.shape == (4096, 6)
    assert set(np.unique(s[:, 0])) == {1, 2, 3, 4, 5} and set(np.unique(s[:, 1])) == {1, 2, 3, 4, 5}
    assert (s[:, 2] >= s[:, 0] + 1).all() and (s[:, 3] >= s[:, 1] + 1).all()
    assert s[:, 2].max() <= 48 and s[:, 4].min() >= 16 and s[:, 4].max() <= 256
    pts = int((s[:, 4] * s[:, 5]).sum())
    # E[side] = (256 - 16) / ln 16 for log-uniform sides
    expect = 4096 * ((256 - 16) / math.log(16)) ** 2
    assert abs(pts / expect - 1) < 0.05
    # knots: clamped, sorted, interior strictly inside (0,1), multiplicity <= degree
    rep = 0
    for i in range(0, 4096, 7):
        d = b.surface(i)
        for k, deg in ((d["ku"], d["p"]), (d["kv"], d["q"])):
            assert (np.diff(k) >= 0).all()
            inner = k[deg + 1:len(k) - deg - 1]
            assert ((inner > 0) & (inner < 1)).all()
            _, counts = np.unique(inner, return_counts=True)
            assert counts.max(initial=1) <= deg
            rep += int((counts > 1).sum())
    assert rep > 0


def test_fit_target_recipe():
    b = W.fit_target(2)
    s = b.surface(0)
    assert s["ctrl"].shape == (64, 64, 3) and s["target"].shape == (512, 512, 3)
    x = s["us"].astype(np.float64)
    np.testing.assert_allclose(s["target"][:, 7, 2], (np.sin(3 * x) * np.cos(3 * x[7])).astype(np.float32),
                               atol=1e-6)
    assert len(s["ku"]) == 68 and s["ku"][4] == np.float32(1 / 61)
