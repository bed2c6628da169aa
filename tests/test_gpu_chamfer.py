"""GPU parity of nurbs_nearest and nurbs_chamfer against the oracle's
nearest-neighbour and Chamfer/Hausdorff functions (Sec. 4, eqs.
ChamferDistance and HausdorffDistance), through the C ABI.

Bars: nearest indices and their float32 squared distances bit-exact (both
sides take the decision in float32 with the same formula, first index on
ties); CD and HD within 1e-5 relative (FP64 sums returned as float32);
gradients within 1e-4 of each gradient's largest magnitude.  Cases: both
dimensions, query sets small enough that the target set is split over
workgroups (the merge path) and large enough that it is not, ragged tails
(sizes not multiples of 256 or 1024), exact ties on a lattice, one point,
identical sets, B > 1.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2104_14547_amd as nd  # noqa: E402
from paper_2104_14547_amd import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def H(t):
    return t.detach().cpu().numpy()


def check_pair(P, Q, cd, hd, gcd, ghd):
    ref_cd, ref_hd, ref_gcd, ref_ghd = O.chamfer_hausdorff(P, Q)
    assert abs(float(cd) - ref_cd) <= 1e-5 * max(ref_cd, 1e-30), (float(cd), ref_cd)
    assert abs(float(hd) - ref_hd) <= 1e-5 * max(ref_hd, 1e-30), (float(hd), ref_hd)
    for got, want in ((gcd, ref_gcd), (ghd, ref_ghd)):
        got = H(got).astype(np.float64)
        scale = np.abs(want).max()
        err = np.abs(got - want).max()
        assert err <= 1e-4 * scale if scale > 0 else err == 0.0, err


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n,m", [(100, 5000), (1000, 777), (5000, 300), (2100, 2100), (1, 1), (1, 600), (600, 1)])
def test_nearest_bit_exact(dim, n, m):
    P, Q = W.point_sets(seed=n * 7 + m + dim, B=2, n=n, m=m, dim=dim)
    idx, d2 = nd.api.nearest(T(P), T(Q))
    for b in range(2):
        ri, rd = O.nearest(P[b], Q[b])
        np.testing.assert_array_equal(H(idx[b]), ri)
        np.testing.assert_array_equal(H(d2[b]), rd)


@pytest.mark.parametrize("dim", [2, 3])
def test_nearest_lattice_ties(dim):
    P, Q = W.point_sets(seed=11, B=1, n=3000, m=1500, dim=dim, lattice=True)
    idx, d2 = nd.api.nearest(T(P), T(Q))
    ri, rd = O.nearest(P[0], Q[0])
    np.testing.assert_array_equal(H(idx[0]), ri)
    np.testing.assert_array_equal(H(d2[0]), rd)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n,m", [(4096, 4096), (300, 2500), (2500, 300)])
def test_chamfer_hausdorff_parity(dim, n, m):
    B = 3
    P, Q = W.point_sets(seed=n + 3 * m + dim, B=B, n=n, m=m, dim=dim)
    cd, hd, gcd, ghd = nd.api.chamfer_hausdorff(T(P), T(Q))
    for b in range(B):
        check_pair(P[b], Q[b], cd[b], hd[b], gcd[b], ghd[b])


def test_chamfer_lattice_ties_and_degenerate():
    P, Q = W.point_sets(seed=12, B=1, n=2000, m=1000, dim=3, lattice=True)
    cd, hd, gcd, ghd = nd.api.chamfer_hausdorff(T(P), T(Q))
    check_pair(P[0], Q[0], cd[0], hd[0], gcd[0], ghd[0])
    # identical sets: both losses and their gradients vanish
    cd, hd, gcd, ghd = nd.api.chamfer_hausdorff(T(P), T(P))
    assert float(cd[0]) == 0.0 and float(hd[0]) == 0.0
    assert float(gcd.abs().max()) == 0.0 and float(ghd.abs().max()) == 0.0
    # one point each
    p1, q1 = np.array([[[0.0, 0.0, 0.0]]], np.float32), np.array([[[3.0, 4.0, 0.0]]], np.float32)
    cd, hd, gcd, ghd = nd.api.chamfer_hausdorff(T(p1), T(q1))
    assert float(cd[0]) == 10.0 and float(hd[0]) == 10.0
    # the pair is nearest in both directions, so its unit vector counts twice
    np.testing.assert_allclose(H(gcd[0, 0]), [-1.2, -1.6, 0.0], rtol=1e-6)
    np.testing.assert_allclose(H(ghd[0, 0]), [-1.2, -1.6, 0.0], rtol=1e-6)


def test_chamfer_deterministic_and_autograd():
    P, Q = W.point_sets(seed=13, B=1, n=1500, m=4000, dim=3)
    a = nd.api.chamfer_hausdorff(T(P), T(Q))
    b = nd.api.chamfer_hausdorff(T(P), T(Q))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    Pt = T(P).requires_grad_(True)
    loss = nd.api.chamfer_loss(Pt, T(Q)).sum() * 2.0
    loss.backward()
    assert torch.equal(Pt.grad, 2.0 * a[2])
