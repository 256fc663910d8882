"""C-ABI checks that need no GPU: the library loads, exports every function
include/ffd.h declares, and a planning-only context validates arguments and
sizes workspaces."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_05708_amd import ffd
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "ffd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffd_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert "ffd_distance" in names and "ffd_batch" in names and "ffd_cross" in names
    lib = ctypes.CDLL(ffd.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ffd.EXPORTS)


def test_version_and_status_text():
    assert "gfx950" in ffd.ffd_version()
    assert ffd.lib.ffd_strerror(ffd.FFD_E_INVALID).decode() == "invalid argument"
    assert ffd.lib.ffd_strerror(12345).decode() == "unknown status"


def test_create_without_gpu_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    assert ffd.lib.ffd_create(0, ctypes.byref(h)) == ffd.FFD_E_DEVICE
    assert ffd.lib.ffd_create(0, None) == ffd.FFD_E_INVALID


@pytest.fixture
def planner():
    h = ffd.ffd_create_planner(256, 160 * 1024)
    yield h
    ffd.ffd_destroy(h)


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail or the planner stops first


def test_planner_create_validation():
    h = ctypes.c_void_p()
    assert ffd.lib.ffd_create_planner(0, 65536, ctypes.byref(h)) == ffd.FFD_E_INVALID
    assert ffd.lib.ffd_create_planner(256, 1024, ctypes.byref(h)) == ffd.FFD_E_INVALID
    assert ffd.lib.ffd_create_planner(256, 65536, None) == ffd.FFD_E_INVALID


def test_distance_argument_checks(planner):
    L = ffd.lib
    ok = L.ffd_distance(planner, FAKE, 5, FAKE, 7, 2, 0, FAKE, None)
    assert ok == ffd.FFD_E_DEVICE  # checks pass, then the planner refuses to launch
    assert L.ffd_distance(planner, None, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance(planner, FAKE, 0, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance(planner, FAKE, 5, FAKE, -1, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 0, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 2, 9, FAKE, None) == ffd.FFD_E_INVALID
    # up to 16 coordinates per point
    assert ffd.FFD_MAX_DIM == 16
    for dim in (5, 8, 9, 16):
        assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, dim, 0, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 17, 0, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    assert L.ffd_distance(None, FAKE, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    # int32 coordinates: squared Euclidean only
    assert L.ffd_distance_i32(planner, FAKE, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    assert L.ffd_distance_i32(planner, FAKE, 5, FAKE, 7, 2, 1, FAKE, None) == ffd.FFD_E_DEVICE
    assert "planning-only" in L.ffd_last_error(planner).decode()


def test_batch_argument_checks(planner):
    L = ffd.lib
    good = np.array([0, 3, 5, 9], dtype=np.int64)
    empty = np.array([0, 3, 3, 9], dtype=np.int64)
    shifted = np.array([1, 3, 5, 9], dtype=np.int64)
    ws = 1 << 20
    args = lambda po, qo, n=3, metric=0, dim=2, out=FAKE, wsb=ws: L.ffd_batch(
        planner, FAKE, _i64p(po), FAKE, _i64p(qo), n, dim, metric, out, FAKE, wsb, None)
    assert args(good, good) == ffd.FFD_E_DEVICE
    assert args(good, empty) == ffd.FFD_E_INVALID
    assert args(shifted, good) == ffd.FFD_E_INVALID
    assert args(good, good, metric=7) == ffd.FFD_E_INVALID
    assert args(good, good, dim=9) == ffd.FFD_E_DEVICE
    assert args(good, good, dim=17) == ffd.FFD_E_UNSUPPORTED
    assert args(good, good, out=None) == ffd.FFD_E_INVALID
    assert args(good, good, n=-1) == ffd.FFD_E_INVALID
    assert args(good, good, n=0) == ffd.FFD_OK  # no-op
    assert L.ffd_batch(planner, FAKE, None, FAKE, _i64p(good), 3, 2, 0, FAKE, FAKE, ws, None) == ffd.FFD_E_INVALID


def test_cross_argument_checks(planner):
    L = ffd.lib
    qo = np.array([0, 4, 9], dtype=np.int64)
    do = np.array([0, 2, 3, 8], dtype=np.int64)
    bad = np.array([0, 2, 1, 8], dtype=np.int64)
    assert L.ffd_cross(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(do), 3, 2, 0, FAKE, FAKE, 1 << 20, None) == ffd.FFD_E_DEVICE
    assert L.ffd_cross(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(bad), 3, 2, 0, FAKE, FAKE, 1 << 20, None) == ffd.FFD_E_INVALID
    assert L.ffd_cross_i32(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(do), 3, 2, 0, FAKE, FAKE, 1 << 20, None) == ffd.FFD_E_UNSUPPORTED
    assert L.ffd_cross(planner, FAKE, _i64p(qo), 0, FAKE, _i64p(do), 3, 2, 0, FAKE, FAKE, 0, None) == ffd.FFD_OK


def test_workspace_size_and_too_small_workspace(planner):
    P, p_off, Q, q_off = workloads.random_pairs(3, 500, 1, 3000, dim=2)
    need = ffd.ffd_workspace_size(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    # at least the plan entries and both offset arrays
    assert need >= 500 * 32 + 2 * 501 * 8
    L = ffd.lib
    # the size covers both the float and the exact plan; far less is refused
    r = L.ffd_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 500, 2, 0, FAKE, FAKE, 256, None)
    assert r == ffd.FFD_E_NOMEM
    # with enough workspace the checks pass and the planning-only context refuses to launch
    r = L.ffd_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 500, 2, 0, FAKE, FAKE, need, None)
    assert r == ffd.FFD_E_DEVICE
    with pytest.raises(ffd.FFDError):
        ffd.ffd_workspace_size(planner, 7, p_off, q_off, 2)
    Qs, qo, DB, do = workloads.cross_int(seed=1, nq=8, ndb=40, length=30)
    assert ffd.ffd_workspace_size(planner, ffd.FFD_OP_CROSS, qo, do, 2) > 0


def test_dtw_argument_checks_and_workspace(planner):
    """The DTW calls take their Frechet counterparts' arguments and checks;
    ffd_workspace_size covers their plans too."""
    L = ffd.lib
    assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 7, 2, 1, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_dtw_distance(planner, None, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 0, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 7, 2, 7, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_distance(None, FAKE, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_distance_i32(planner, FAKE, 5, FAKE, 7, 2, 0, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    assert L.ffd_dtw_distance_i32(planner, FAKE, 5, FAKE, 7, 2, 1, FAKE, None) == ffd.FFD_E_DEVICE
    good = np.array([0, 3, 5, 9], dtype=np.int64)
    empty = np.array([0, 3, 3, 9], dtype=np.int64)
    assert L.ffd_dtw_batch(planner, FAKE, _i64p(good), FAKE, _i64p(good), 3, 2, 0, FAKE, FAKE, 1 << 20,
                           None) == ffd.FFD_E_DEVICE
    assert L.ffd_dtw_batch(planner, FAKE, _i64p(good), FAKE, _i64p(empty), 3, 2, 0, FAKE, FAKE, 1 << 20,
                           None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_batch_i32(planner, FAKE, _i64p(good), FAKE, _i64p(good), 3, 2, 0, FAKE, FAKE, 1 << 20,
                               None) == ffd.FFD_E_UNSUPPORTED
    qo = np.array([0, 4, 9], dtype=np.int64)
    do = np.array([0, 2, 3, 8], dtype=np.int64)
    assert L.ffd_dtw_cross(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(do), 3, 2, 1, FAKE, FAKE, 1 << 20,
                           None) == ffd.FFD_E_DEVICE
    assert L.ffd_dtw_cross_i32(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(do), 3, 2, 1, FAKE, FAKE, 1 << 20,
                               None) == ffd.FFD_E_DEVICE
    # long curves whose boundary rows do not fit LDS need link buffers in both measures
    P, p_off, Q, q_off = workloads.random_pairs(4, 60, 1, 9000, dim=2)
    need = ffd.ffd_workspace_size(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    for fn in (L.ffd_batch, L.ffd_dtw_batch):
        assert fn(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 2, 0, FAKE, FAKE, need,
                  None) == ffd.FFD_E_DEVICE
        assert fn(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 2, 0, FAKE, FAKE, 256,
                  None) == ffd.FFD_E_NOMEM


def test_metric_checks(planner):
    L = ffd.lib
    for metric in (ffd.FFD_MANHATTAN, ffd.FFD_CHEBYSHEV):
        assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 2, metric, FAKE, None) == ffd.FFD_E_DEVICE
        assert L.ffd_distance_i32(planner, FAKE, 5, FAKE, 7, 2, metric, FAKE, None) == ffd.FFD_E_DEVICE
        assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 7, 2, metric, FAKE, None) == ffd.FFD_E_DEVICE
        assert L.ffd_dtw_distance_i32(planner, FAKE, 5, FAKE, 7, 2, metric, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 2, 5, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 2, -1, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_distance_i32(planner, FAKE, 5, FAKE, 7, 2, ffd.FFD_EUCLIDEAN, FAKE, None) == ffd.FFD_E_UNSUPPORTED


def test_great_circle_checks(planner):
    """FFD_HAVERSINE: (latitude, longitude) points for the float32 Frechet
    and DTW calls only; the workspace size covers their FP64 plans."""
    L = ffd.lib
    H = ffd.FFD_HAVERSINE
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 2, H, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 3, H, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance(planner, FAKE, 5, FAKE, 7, 1, H, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 7, 2, H, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_dtw_distance(planner, FAKE, 5, FAKE, 7, 3, H, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_distance_i32(planner, FAKE, 5, FAKE, 7, 2, H, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    assert L.ffd_dtw_distance_i32(planner, FAKE, 5, FAKE, 7, 2, H, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    P, p_off, Q, q_off = workloads.random_pairs(6, 60, 1, 9000, dim=2)
    need = ffd.ffd_workspace_size(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2, metric=H)
    assert L.ffd_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 2, H, FAKE, FAKE, need,
                       None) == ffd.FFD_E_DEVICE
    assert L.ffd_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 2, H, FAKE, FAKE, 256,
                       None) == ffd.FFD_E_NOMEM
    assert L.ffd_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 4, H, FAKE, FAKE, need,
                       None) == ffd.FFD_E_INVALID
    assert L.ffd_batch_i32(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 2, H, FAKE, FAKE, need,
                           None) == ffd.FFD_E_UNSUPPORTED
    qo = np.array([0, 4, 9], dtype=np.int64)
    assert L.ffd_cross(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(p_off), 60, 2, H, FAKE, FAKE, 1 << 30,
                       None) == ffd.FFD_E_DEVICE
    assert L.ffd_dtw_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 2, H, FAKE, FAKE, need,
                           None) == ffd.FFD_E_DEVICE
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2, metric=H, dtw=True)
    assert sm["rows_per_lane"] <= 4
    with pytest.raises(ffd.FFDError):
        ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2, metric=H, exact=True)


def test_levenshtein_argument_checks(planner):
    L = ffd.lib
    assert L.ffd_levenshtein_distance(planner, FAKE, 5, FAKE, 7, 1, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_levenshtein_distance(planner, None, 5, FAKE, 7, 1, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_levenshtein_distance(planner, FAKE, 0, FAKE, 7, 1, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_levenshtein_distance(planner, FAKE, 5, FAKE, 7, 5, FAKE, None) == ffd.FFD_E_DEVICE
    assert L.ffd_levenshtein_distance(planner, FAKE, 5, FAKE, 7, 17, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    # values are float32 integers: n + m must stay below 2^24
    assert L.ffd_levenshtein_distance(planner, FAKE, 1 << 23, FAKE, 1 << 23, 1, FAKE, None) == ffd.FFD_E_UNSUPPORTED
    big = np.array([0, 1 << 23], dtype=np.int64)
    assert L.ffd_levenshtein_batch(planner, FAKE, _i64p(big), FAKE, _i64p(big), 1, 1, FAKE, FAKE, 1 << 20,
                                   None) == ffd.FFD_E_UNSUPPORTED
    one = np.array([0, 1], dtype=np.int64)
    assert L.ffd_levenshtein_cross(planner, FAKE, _i64p(big), 1, FAKE, _i64p(big), 1, 1, FAKE, FAKE, 1 << 20,
                                   None) == ffd.FFD_E_UNSUPPORTED
    assert L.ffd_levenshtein_cross(planner, FAKE, _i64p(one), 1, FAKE, _i64p(big), 1, 1, FAKE, FAKE, 1 << 20,
                                   None) == ffd.FFD_E_DEVICE  # 1 + 2^23 is within the bound
    good = np.array([0, 3, 5, 9], dtype=np.int64)
    assert L.ffd_levenshtein_batch(planner, FAKE, _i64p(good), FAKE, _i64p(good), 3, 1, FAKE, FAKE, 1 << 20,
                                   None) == ffd.FFD_E_DEVICE
    qo = np.array([0, 4, 9], dtype=np.int64)
    assert L.ffd_levenshtein_cross(planner, FAKE, _i64p(qo), 2, FAKE, _i64p(good), 3, 1, FAKE, FAKE, 1 << 20,
                                   None) == ffd.FFD_E_DEVICE
    P, p_off, Q, q_off = workloads.random_pairs(5, 60, 1, 9000, dim=1)
    need = ffd.ffd_workspace_size(planner, ffd.FFD_OP_BATCH, p_off, q_off, 1)
    assert L.ffd_levenshtein_batch(planner, FAKE, _i64p(p_off), FAKE, _i64p(q_off), 60, 1, FAKE, FAKE, need,
                                   None) == ffd.FFD_E_DEVICE


def test_set_tuning_validation(planner):
    ffd.ffd_set_tuning(planner, 4, 2)
    ffd.ffd_set_tuning(planner, 0, 0)
    with pytest.raises(ffd.FFDError):
        ffd.ffd_set_tuning(planner, 3, 1)
    with pytest.raises(ffd.FFDError):
        ffd.ffd_set_tuning(planner, 4, 99)
    ffd.ffd_set_tuning(planner, 2, -1)  # single pairs: the pipelined kernel whenever it can run them
    with pytest.raises(ffd.FFDError):
        ffd.ffd_set_tuning(planner, 2, -2)
    ffd.ffd_set_tuning(planner, 0, 0)


def test_kernel_timing_checks(planner):
    # a planning-only context launches nothing, so it has nothing to time
    with pytest.raises(ffd.FFDError):
        ffd.ffd_set_kernel_timing(planner, True)
    ffd.ffd_set_kernel_timing(planner, False)
    assert ffd.ffd_kernel_time(planner) == (0.0, 0)


def test_serving_database_and_arena(planner):
    L = ffd.lib
    DB, dbo = workloads.serving_db(seed=9, count=300)
    db = ctypes.c_void_p()
    assert L.ffd_db_create(planner, FAKE, _i64p(dbo), 300, 2, ctypes.byref(db)) == ffd.FFD_OK
    try:
        bad = dbo.copy()
        bad[5] = bad[4]
        h = ctypes.c_void_p()
        assert L.ffd_db_create(planner, FAKE, _i64p(bad), 300, 2, ctypes.byref(h)) == ffd.FFD_E_INVALID
        assert L.ffd_db_create(planner, None, _i64p(dbo), 300, 2, ctypes.byref(h)) == ffd.FFD_E_INVALID
        assert L.ffd_db_create(planner, FAKE, _i64p(dbo), 300, 17, ctypes.byref(h)) == ffd.FFD_E_UNSUPPORTED
        assert L.ffd_db_create(planner, FAKE, _i64p(dbo), 300, 9, ctypes.byref(h)) == ffd.FFD_OK
        ffd.lib.ffd_db_destroy(h)
        n = ctypes.c_size_t()
        assert L.ffd_server_arena_size(db, 8, 8192, ctypes.byref(n)) == ffd.FFD_OK
        # the reordered database, the queries of 8 requests and their results at least
        assert n.value >= dbo[-1] * 2 * 4 + 8 * 8192 * 2 * 4 + 8 * 300 * 4
        small = ctypes.c_size_t()
        assert L.ffd_server_arena_size(db, 1, 100, ctypes.byref(small)) == ffd.FFD_OK
        assert small.value < n.value
        assert L.ffd_server_arena_size(db, 0, 100, ctypes.byref(small)) == ffd.FFD_E_INVALID
        assert L.ffd_server_arena_size(db, 8, 0, ctypes.byref(small)) == ffd.FFD_E_INVALID
        s = ctypes.c_void_p()
        assert L.ffd_server_create(db, FAKE, n.value - 1, 8, 8192, ctypes.byref(s)) == ffd.FFD_E_NOMEM
        assert L.ffd_server_create(db, FAKE, n.value, 8, 8192, ctypes.byref(s)) == ffd.FFD_E_DEVICE
        assert L.ffd_server_create(db, None, n.value, 8, 8192, ctypes.byref(s)) == ffd.FFD_E_INVALID
        t = ctypes.c_uint64()
        assert L.ffd_server_submit(None, FAKE, 5, 0, FAKE, ctypes.byref(t)) == ffd.FFD_E_INVALID
    finally:
        L.ffd_db_destroy(db)


def test_scratch_sizes_and_registration(planner):
    """Scratch sizes (ffd_workspace_size with FFD_OP_PAIR, FFD_OP_DECIDE,
    FFD_OP_KNN) and ffd_set_scratch argument checks; the library allocates
    no device memory, so long pairs and the search calls size their scratch
    through these."""
    # a pair that fits one wavefront needs none, a long one some
    assert ffd.ffd_workspace_size(planner, ffd.FFD_OP_PAIR, [0, 100], [0, 90], 2) == 0
    long_need = ffd.ffd_workspace_size(planner, ffd.FFD_OP_PAIR, [0, 6000], [0, 5000], 2)
    assert long_need > 0
    # more rows need more boundary rows
    assert ffd.ffd_workspace_size(planner, ffd.FFD_OP_PAIR, [0, 60000], [0, 5000], 2) > long_need
    with pytest.raises(ffd.FFDError):
        ffd.ffd_workspace_size(planner, ffd.FFD_OP_PAIR, [0, 10, 20], [0, 5, 9], 2)  # two curves
    P, p_off, Q, q_off = workloads.random_pairs(5, 40, 1, 900, dim=2)
    assert ffd.ffd_workspace_size(planner, ffd.FFD_OP_DECIDE, p_off, q_off, 2) > 2 * 41 * 8
    _, db_off = workloads.concat([np.zeros((int(k), 2), np.float32) for k in np.arange(20, 220)])
    knn = ffd.ffd_workspace_size(planner, ffd.FFD_OP_KNN, [0, 300], db_off, 2)
    assert knn > 200 * 8
    # several queries (ffd_knn_batch): per-(query, curve) arrays grow with nq
    knn3 = ffd.ffd_workspace_size(planner, ffd.FFD_OP_KNN, [0, 30, 60, 400], db_off, 2)
    assert knn3 > knn + 2 * 3 * 200 * 4
    assert ffd.ffd_workspace_size(planner, ffd.FFD_OP_KNN, [0], db_off, 2) == 0  # no query: nothing
    L = ffd.lib
    assert L.ffd_set_scratch(None, None, 0) == ffd.FFD_E_INVALID
    assert L.ffd_set_scratch(planner, None, 64) == ffd.FFD_E_INVALID
    assert L.ffd_set_scratch(planner, FAKE, 64) == ffd.FFD_OK
    assert L.ffd_set_scratch(planner, None, 0) == ffd.FFD_OK


def test_noalloc_size_limit_checked_on_the_host(planner):
    """ffd_batch_noalloc refuses a request larger than its static scratch
    before anything is launched (FFD_E_NOMEM, with the size it needs); a
    request that fits passes the checks (a planning-only context then
    reports FFD_E_DEVICE)."""
    L = ffd.lib
    P, p_off, Q, q_off = workloads.batched()
    po, qo = np.asarray(p_off, np.int64), np.asarray(q_off, np.int64)
    assert L.ffd_batch_noalloc(planner, FAKE, _i64p(po), FAKE, _i64p(qo), 4096, 2, 0, FAKE, None) == ffd.FFD_E_DEVICE
    big = np.arange(5, dtype=np.int64) * 32768
    assert L.ffd_batch_noalloc(planner, FAKE, _i64p(big), FAKE, _i64p(big), 4, 2, 0, FAKE, None) == ffd.FFD_E_NOMEM
    assert b"ffd_batch_noalloc has 33554432" in L.ffd_last_error(planner)
    # argument checks come first
    bad = np.array([0, 5, 5], dtype=np.int64)
    assert L.ffd_batch_noalloc(planner, FAKE, _i64p(bad), FAKE, _i64p(bad), 2, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
    assert L.ffd_batch_noalloc(None, FAKE, _i64p(po), FAKE, _i64p(qo), 4096, 2, 0, FAKE, None) == ffd.FFD_E_INVALID
