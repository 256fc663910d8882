"""Pins for the great-circle ground distance of the CPU oracle (no GPU).

Sec. 3 of the paper leaves the ground distance open and Sec. 2 motivates
vessel trajectories; the oracle's FFDO_HAVERSINE cell is the central
angle between (latitude, longitude) points in radians, by the haversine
formula in FP64.  It is tied here to things other than itself:

* closed forms: points on the equator are |dlon| apart (taken the short way
  round), points on a meridian |dlat|, a pole is pi/2 from the equator and
  antipodal points are pi apart;
* an independent formula: atan2(|u x v|, u . v) on the unit vectors u, v,
  in numpy FP64 (well conditioned at every angle);
* the Frechet distance and DTW on these cells against brute force over
  all couplings with the independent formula's matrix;
* invariances: rotation about the polar axis (a longitude shift),
  reflection in the equator, swapping the curves (bit-exact);
* the triangle inequality of the discrete Frechet distance;
* planted mistakes (no cosine factor, the full instead of the half angle,
  one latitude's cosine squared) fail the closed forms or the formula.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
import workloads

H = oracle.HAVERSINE


def pt(lat, lon):
    return np.array([[lat, lon]], dtype=np.float32)


def cell(a, b):
    """The oracle's cell: the distance of two one-point curves."""
    return oracle.dfd(a, b, H, "table")


def unit(c):
    c = np.asarray(c, dtype=np.float64)
    lat, lon = c[..., 0], c[..., 1]
    return np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], axis=-1)


def angle_matrix(p, q):
    """Central angles by atan2(|u x v|, u . v) (not the haversine formula)."""
    u, v = unit(p)[:, None, :], unit(q)[None, :, :]
    cr = np.cross(u, v)
    return np.arctan2(np.sqrt((cr * cr).sum(-1)), (u * v).sum(-1))


def test_equator_and_meridian():
    rng = np.random.default_rng(700)
    for _ in range(200):
        a, b = rng.uniform(-np.pi, np.pi, size=2).astype(np.float32)
        d = abs(float(a) - float(b))
        exp = d if d <= np.pi else 2 * np.pi - d
        assert cell(pt(0, a), pt(0, b)) == pytest.approx(exp, rel=1e-13, abs=1e-15)
        la, lb = rng.uniform(-1.5, 1.5, size=2).astype(np.float32)
        lon = np.float32(rng.uniform(-np.pi, np.pi))
        assert cell(pt(la, lon), pt(lb, lon)) == pytest.approx(abs(float(la) - float(lb)), rel=1e-13, abs=1e-15)


def test_poles_and_antipodes():
    half = np.float32(np.pi / 2)  # float32 pi/2 exceeds pi/2 by about 4.4e-8
    rng = np.random.default_rng(701)
    for lon in rng.uniform(-np.pi, np.pi, size=20).astype(np.float32):
        assert cell(pt(half, 0.3), pt(0, lon)) == pytest.approx(np.pi / 2, abs=1e-7)
        assert cell(pt(half, lon), pt(-half, 1.0)) == pytest.approx(np.pi, abs=1e-7)
        lat = np.float32(rng.uniform(-1.5, 1.5))
        anti = np.float32(lon + np.pi if lon < 0 else lon - np.pi)
        assert cell(pt(lat, lon), pt(-lat, anti)) == pytest.approx(np.pi, abs=1e-6)
    assert cell(pt(0.7, -2.0), pt(0.7, -2.0)) == 0.0


def test_independent_formula():
    rng = np.random.default_rng(702)
    # uniform on the sphere, and close pairs (steps of 1e-3 .. 1e-7 rad)
    z = rng.uniform(-1, 1, size=400)
    a = np.stack([np.arcsin(z), rng.uniform(-np.pi, np.pi, size=400)], 1).astype(np.float32)
    b = np.stack([np.arcsin(rng.uniform(-1, 1, size=400)), rng.uniform(-np.pi, np.pi, size=400)], 1)
    near = (a + rng.standard_normal((400, 2)) * 10.0 ** rng.uniform(-7, -3, size=(400, 1))).astype(np.float32)
    for other in (b.astype(np.float32), near):
        for k in range(400):
            got = cell(a[k:k + 1], other[k:k + 1])
            exp = angle_matrix(a[k:k + 1], other[k:k + 1])[0, 0]
            # the haversine form loses accuracy only next to the antipode
            tol = 1e-7 if exp > 3.0 else 1e-12 * max(exp, 1e-3)
            assert abs(got - exp) <= tol, (k, got, exp)


def test_frechet_equals_brute_force():
    rng = np.random.default_rng(703)
    for _ in range(60):
        n, m = (int(v) for v in rng.integers(1, 7, size=2))
        p = workloads.geo_walk(rng, n, 0.05).astype(np.float32)
        q = workloads.geo_walk(rng, m, 0.05).astype(np.float32)
        exp = brute.brute_from_matrix(angle_matrix(p, q).tolist())
        for method in ("table", "rolling", "recursive"):
            assert oracle.dfd(p, q, H, method) == pytest.approx(exp, rel=1e-12, abs=1e-15)


def test_dtw_equals_brute_force():
    """DTW (Appendix B) on great-circle cells: the smallest sum of angles
    over all couplings, with the independent formula's matrix."""
    rng = np.random.default_rng(708)
    for _ in range(40):
        n, m = (int(v) for v in rng.integers(1, 7, size=2))
        p = workloads.geo_walk(rng, n, 0.05).astype(np.float32)
        q = workloads.geo_walk(rng, m, 0.05).astype(np.float32)
        exp = brute.brute_dtw_from_matrix(angle_matrix(p, q).tolist())
        assert oracle.dtw(p, q, H) == pytest.approx(exp, rel=1e-12, abs=1e-15)


def test_invariances_and_symmetry():
    rng = np.random.default_rng(704)
    for _ in range(40):
        # coordinates on a 2^-10 grid, so that shifting the longitude by a
        # multiple of 1/8 is exact in float32
        p, q = (np.round(workloads.geo_walk(rng, L, 0.02) * 1024).astype(np.float32) / 1024
                for L in (30, 25))
        d = oracle.dfd(p, q, H)
        assert oracle.dfd(q, p, H) == d
        refl = [np.stack([-c[:, 0], c[:, 1]], 1) for c in (p, q)]
        assert oracle.dfd(*refl, H) == d
        # rotation about the axis: the FP64 cells change by rounding only
        s = np.float32(0.125 * int(rng.integers(-8, 8)))
        rot = [np.stack([c[:, 0], c[:, 1] + s], 1) for c in (p, q)]
        assert all(np.array_equal(r[:, 1] - s, c[:, 1]) for r, c in zip(rot, (p, q)))
        assert oracle.dfd(*rot, H) == pytest.approx(d, rel=1e-12, abs=1e-15)


def test_triangle_inequality():
    rng = np.random.default_rng(705)
    for _ in range(40):
        a, b, c = (workloads.geo_walk(rng, int(rng.integers(2, 40)), 0.03).astype(np.float32)
                   for _ in range(3))
        assert oracle.dfd(a, c, H) <= oracle.dfd(a, b, H) + oracle.dfd(b, c, H) + 1e-12


def test_pools_and_validation():
    P, po, Q, qo = workloads.geo_pairs(seed=706, npairs=12, lo=2, hi=90)
    got = oracle.dfd_batch(P, po, Q, qo, H, nthreads=3)
    for k in range(12):
        assert got[k] == oracle.dfd(P[po[k]:po[k + 1]], Q[qo[k]:qo[k + 1]], H)
    with pytest.raises(Exception):
        oracle.dfd(np.zeros((3, 3), np.float32), np.zeros((2, 3), np.float32), H)
    with pytest.raises(Exception):
        oracle.dfd_f32_replica(P[:4], Q[:4], H)


@pytest.mark.parametrize("mistake", ["no_cos", "full_angle", "one_cos"])
def test_pins_catch_planted_mistakes(mistake):
    def mutant(a, b):
        (la, oa), (lb, ob) = np.asarray(a, np.float64)[0], np.asarray(b, np.float64)[0]
        if mistake == "full_angle":
            h = np.sin(lb - la) ** 2 + np.cos(la) * np.cos(lb) * np.sin(ob - oa) ** 2
        else:
            cc = 1.0 if mistake == "no_cos" else np.cos(la) ** 2
            h = np.sin((lb - la) / 2) ** 2 + cc * np.sin((ob - oa) / 2) ** 2
        return 2 * np.arcsin(np.sqrt(min(h, 1.0)))
    rng = np.random.default_rng(707)
    caught = 0
    for _ in range(50):
        a = pt(*rng.uniform([-1.4, -3], [1.4, 3]))
        b = pt(*rng.uniform([-1.4, -3], [1.4, 3]))
        caught += abs(mutant(a, b) - angle_matrix(a, b)[0, 0]) > 1e-9
        caught += abs(mutant(pt(0, a[0, 1]), pt(0, b[0, 1])) - cell(pt(0, a[0, 1]), pt(0, b[0, 1]))) > 1e-9
    assert caught > 0
