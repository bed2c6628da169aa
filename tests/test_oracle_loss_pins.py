"""Pins for the oracle's point-set losses (Sec. 4, eqs. ChamferDistance and
HausdorffDistance), from facts the definitions fix:

* the float32 nearest-point decision agrees with an FP64 brute force except
  at near-ties, and is exact (first index on ties) on integer lattices where
  float32 arithmetic is exact;
* CD(P, P) = HD(P, P) = 0; both are symmetric in (P, Q);
* a cloud against its own copy shifted by t (small against the spacing):
  every nearest partner is the shifted copy, CD = (n + m)|t|, HD = 2|t|,
  dCD/dP_i = 2 t/|t|;
* central finite differences of CD and HD with respect to P where the
  nearest partners do not change;
* a hand-worked three-point example.
"""
import numpy as np
import pytest

from oracle import oracle as O


def test_nearest_matches_fp64_brute_force_away_from_ties():
    g = np.random.default_rng(1)
    for dim in (2, 3):
        P = g.uniform(-1, 1, (400, dim)).astype(np.float32)
        Q = g.uniform(-1, 1, (300, dim)).astype(np.float32)
        idx, d2 = O.nearest(P, Q)
        D = ((P[:, None, :].astype(np.float64) - Q[None, :, :]) ** 2).sum(-1)
        ref = D.argmin(1)
        differ = idx != ref
        # a differing choice must be a near-tie in exact arithmetic
        assert np.all(np.abs(D[np.arange(len(P)), idx] - D[np.arange(len(P)), ref])[differ] < 1e-6)
        assert differ.mean() < 0.01
        np.testing.assert_allclose(d2, D[np.arange(len(P)), idx], rtol=1e-6)


def test_nearest_exact_on_integer_lattice_first_index_wins():
    P = np.array([[0, 0, 0], [2, 0, 0], [5, 5, 5]], np.float32)
    # Q0 and Q1 tie for P0 (distance 1); Q2 is P1 itself; Q3/Q4 tie for P2
    Q = np.array([[1, 0, 0], [-1, 0, 0], [2, 0, 0], [5, 5, 7], [5, 7, 5]], np.float32)
    idx, d2 = O.nearest(P, Q)
    assert idx.tolist() == [0, 2, 3]
    assert d2.tolist() == [1.0, 0.0, 4.0]


def test_identity_and_symmetry():
    g = np.random.default_rng(2)
    P = g.uniform(0, 1, (120, 3)).astype(np.float32)
    Q = g.uniform(0, 1, (90, 3)).astype(np.float32)
    cd, hd, gcd, ghd = O.chamfer_hausdorff(P, P)
    assert cd == 0.0 and hd == 0.0
    assert not gcd.any() and not ghd.any()
    a = O.chamfer_hausdorff(P, Q)
    b = O.chamfer_hausdorff(Q, P)
    assert a[0] == pytest.approx(b[0], rel=1e-14)
    assert a[1] == pytest.approx(b[1], rel=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_shifted_copy_closed_form(dim):
    # a lattice with spacing 1 and a shift of length 0.05
    grid = np.stack(np.meshgrid(*[np.arange(6)] * dim, indexing="ij"), -1).reshape(-1, dim).astype(np.float64)
    t = np.array([0.03, -0.04, 0.0][:dim]) if dim == 2 else np.array([0.03, 0.0, -0.04])
    P = grid.astype(np.float32)
    Q = (grid + t).astype(np.float32)
    tt = (Q.astype(np.float64) - P.astype(np.float64))  # the shift after rounding, per point
    cd, hd, gcd, ghd = O.chamfer_hausdorff(P, Q)
    lens = np.linalg.norm(tt, axis=1)
    assert cd == pytest.approx(2 * lens.sum(), rel=1e-12)
    assert hd == pytest.approx(2 * lens.max(), rel=1e-12)
    np.testing.assert_allclose(gcd, -2 * tt / lens[:, None], rtol=1e-12)
    # two unit vectors -t/|t|: on the farthest point and on the nearest point of the farthest target
    assert np.linalg.norm(ghd, axis=1).sum() == pytest.approx(2.0, rel=1e-12)
    assert np.count_nonzero(np.linalg.norm(ghd, axis=1)) in (1, 2)


def test_hand_worked_example():
    # P = {(0,0), (4,0)}, Q = {(0,3), (4,1)}:
    #   P0 -> Q0 (3), P1 -> Q1 (1); Q0 -> P0 (3), Q1 -> P1 (1)
    #   CD = 3 + 1 + 3 + 1 = 8, HD = 3 + 3 = 6
    P = np.array([[0, 0], [4, 0]], np.float32)
    Q = np.array([[0, 3], [4, 1]], np.float32)
    cd, hd, gcd, ghd = O.chamfer_hausdorff(P, Q)
    assert cd == 8.0 and hd == 6.0
    np.testing.assert_array_equal(gcd, [[0, -2], [0, -2]])
    np.testing.assert_array_equal(ghd, [[0, -2], [0, 0]])


@pytest.mark.parametrize("dim", [2, 3])
def test_finite_differences(dim):
    g = np.random.default_rng(3 + dim)
    P = g.uniform(0, 1, (40, dim)).astype(np.float32)
    Q = g.uniform(0, 1, (55, dim)).astype(np.float32)
    cd, hd, gcd, ghd = O.chamfer_hausdorff(P, Q)
    h = 2.0 ** -14  # the step actually taken (after float32 rounding) is used below
    for i in range(0, 40, 7):
        for x in range(dim):
            Pp, Pm = P.copy(), P.copy()
            Pp[i, x] += np.float32(h)
            Pm[i, x] -= np.float32(h)
            step = float(Pp[i, x]) - float(Pm[i, x])
            fp, fm = O.chamfer_hausdorff(Pp, Q), O.chamfer_hausdorff(Pm, Q)
            # only where the nearest / farthest choices stay the same on both sides
            if (O.nearest(Pp, Q)[0] == O.nearest(Pm, Q)[0]).all() and \
                    (O.nearest(Q, Pp)[0] == O.nearest(Q, Pm)[0]).all():
                assert (fp[0] - fm[0]) / step == pytest.approx(gcd[i, x], abs=2e-5)
                ap, am = O.nearest(Pp, Q)[1], O.nearest(Pm, Q)[1]
                bp, bm = O.nearest(Q, Pp)[1], O.nearest(Q, Pm)[1]
                if ap.argmax() == am.argmax() and bp.argmax() == bm.argmax():
                    assert (fp[1] - fm[1]) / step == pytest.approx(ghd[i, x], abs=2e-5)
