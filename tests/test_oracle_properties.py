"""Property-based pins for the CPU oracle (hypothesis; no GPU).

Random curves of any shape, dimension and value range must satisfy what the
definitions imply, for both measures: the Frechet value is one of the cell
distances and lies between the end-point bound and the largest cell; both
measures are symmetric bit for bit; the squared-metric Frechet value is the
square of the Euclidean one; repeating a point leaves the Frechet value
unchanged; DTW lies between the Frechet value and (n + m - 1) times it; on
tiny inputs both equal brute force over all couplings.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from oracle import brute

SETTINGS = settings(max_examples=120, deadline=None)


@st.composite
def curve_pair(draw, max_len=24):
    D = draw(st.integers(1, 4))
    n = draw(st.integers(1, max_len))
    m = draw(st.integers(1, max_len))
    kind = draw(st.sampled_from(["small_int", "unit", "wide"]))
    if kind == "small_int":
        elem = st.integers(-4, 4).map(float)
    elif kind == "unit":
        elem = st.floats(-1.0, 1.0, width=32, allow_nan=False, allow_infinity=False)
    else:
        elem = st.floats(-1e6, 1e6, width=32, allow_nan=False, allow_infinity=False)
    p = np.array(draw(st.lists(elem, min_size=n * D, max_size=n * D)), dtype=np.float32).reshape(n, D)
    q = np.array(draw(st.lists(elem, min_size=m * D, max_size=m * D)), dtype=np.float32).reshape(m, D)
    return p, q


@SETTINGS
@given(curve_pair())
def test_frechet_is_a_cell_value_between_bounds(pq):
    p, q = pq
    for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
        d = brute.ground_matrix(p, q, squared=metric == oracle.SQEUCLIDEAN)
        v = oracle.dfd(p, q, metric, "rolling")
        assert v in set(d.ravel().tolist())
        assert max(d[0, 0], d[-1, -1]) <= v <= d.max()
        # every row and every column is visited by any coupling
        assert v >= d.min(axis=1).max() and v >= d.min(axis=0).max()


@SETTINGS
@given(curve_pair())
def test_symmetry_and_squared_metric(pq):
    p, q = pq
    for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
        assert oracle.dfd(p, q, metric, "rolling") == oracle.dfd(q, p, metric, "rolling")
        assert oracle.dtw(p, q, metric) == oracle.dtw(q, p, metric)
    e = oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")
    s = oracle.dfd(p, q, oracle.SQEUCLIDEAN, "rolling")
    assert abs(e * e - s) <= 4e-16 * s + 1e-300


@SETTINGS
@given(curve_pair(), st.data())
def test_repeating_a_point_keeps_the_frechet_value(pq, data):
    p, q = pq
    i = data.draw(st.integers(0, p.shape[0] - 1))
    p2 = np.insert(p, i, p[i], axis=0)
    assert oracle.dfd(p2, q, oracle.EUCLIDEAN, "rolling") == oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")


@SETTINGS
@given(curve_pair())
def test_dtw_between_frechet_bounds(pq):
    p, q = pq
    n, m = p.shape[0], q.shape[0]
    for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
        f = oracle.dfd(p, q, metric, "rolling")
        w = oracle.dtw(p, q, metric)
        assert f * (1 - 1e-12) <= w <= (n + m - 1) * f * (1 + 1e-12) + 1e-300


@settings(max_examples=60, deadline=None)
@given(curve_pair(max_len=5))
def test_tiny_inputs_equal_brute_force(pq):
    p, q = pq
    for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
        sq = metric == oracle.SQEUCLIDEAN
        assert oracle.dfd(p, q, metric, "recursive") == brute.brute(p, q, squared=sq)
        assert oracle.dtw(p, q, metric) == brute.brute_dtw(p, q, squared=sq)
