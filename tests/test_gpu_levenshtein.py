"""GPU parity of the Levenshtein distance (Appendix B, Algorithm B.2) through
the C ABI: bit-exact against the int64 oracle for every launch shape, in the
batch, cross and single-pair forms, with bands split over waves, long
sequences whose boundary rows do not fit LDS, and the edge cases (single
symbols, equal and disjoint sequences)."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2404_05708_amd import ffd
    c = ffd.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def syms(rng, n, D=1, alphabet=4):
    return rng.integers(0, alphabet, size=(n, D)).astype(np.int32)


@pytest.mark.parametrize("R", [0, 1, 2, 4, 8])
def test_random_shapes(ctx, R):
    rng = np.random.default_rng(500 + R)
    ctx.set_tuning(R, 0)
    try:
        for it in range(14):
            n, m, D = int(rng.integers(1, 800)), int(rng.integers(1, 800)), int(rng.integers(1, 3))
            p, q = syms(rng, n, D), syms(rng, m, D)
            say(f"case: levenshtein R={R} n={n} m={m} D={D}")
            assert ctx.levenshtein(dev(p), dev(q)).item() == oracle.lev(p, q), (n, m, D)
    finally:
        ctx.set_tuning(0, 0)


def test_edge_cases(ctx):
    rng = np.random.default_rng(510)
    for n, m in [(1, 1), (1, 500), (500, 1), (64, 64), (512, 80), (513, 79), (64 * 8 + 1, 17), (3000, 2000)]:
        p, q = syms(rng, n), syms(rng, m)
        say(f"case: levenshtein edge n={n} m={m}")
        assert ctx.levenshtein(dev(p), dev(q)).item() == oracle.lev(p, q)
        assert ctx.last_errors() == 0
    p = syms(rng, 777)
    assert ctx.levenshtein(dev(p), dev(p)).item() == 0
    a, b = np.zeros((300, 1), np.int32), np.ones((450, 1), np.int32)
    assert ctx.levenshtein(dev(a), dev(b)).item() == 450


def test_extreme_symbol_values(ctx):
    """Symbols whose bit patterns are float specials (+-0, infinities, NaNs,
    denormals) stay distinct: the kernel compares bit patterns, never floats,
    and marks separators outside the symbol values."""
    special = np.array([0, -2 ** 31, 2 ** 31 - 1, -1, 0x7F800000, -0x00800000, 0x7FC00000, 0x7FC00001,
                        1, 0x00000001, 0x3F800000, 2 ** 24, 2 ** 24 + 1], dtype=np.int64).astype(np.int32)
    rng = np.random.default_rng(512)
    for n, m, D in [(40, 33, 1), (700, 650, 1), (90, 120, 2), (300, 200, 3), (130, 140, 4)]:
        p = special[rng.integers(0, len(special), size=(n, D))]
        q = special[rng.integers(0, len(special), size=(m, D))]
        say(f"case: levenshtein special symbols n={n} m={m} D={D}")
        assert ctx.levenshtein(dev(p), dev(q)).item() == oracle.lev(p, q)
    # +0 and -0 as float are the same value; as symbols they differ
    z, nz = np.zeros((5, 1), np.int32), np.full((5, 1), -2 ** 31, np.int32)
    assert ctx.levenshtein(dev(z), dev(nz)).item() == 5


def test_batch_cross_pairs_split_and_long(ctx):
    P, p_off, Q, q_off = workloads.symbol_pairs(seed=511, npairs=150, lo=1, hi=2500)
    say("case: levenshtein batch of 150 pairs")
    base = ctx.levenshtein_batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    np.testing.assert_array_equal(base, oracle.lev_batch(P, p_off, Q, q_off, nthreads=8))
    for R in (1, 2, 8):
        ctx.set_tuning(R, 0)
        ctx.set_split(1e-9)
        try:
            say(f"case: levenshtein batch split R={R}")
            got = ctx.levenshtein_batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
            assert ctx.last_errors() == 0
        finally:
            ctx.set_split(0.0)
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, base)
    for k in (0, 40, 149):
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        assert ctx.levenshtein(dev(p), dev(q)).item() == base[k]
    Qs, qo = workloads.concat([P[p_off[k]:p_off[k + 1]] for k in range(4)])
    DB, do = workloads.concat([Q[q_off[k]:q_off[k + 1]] for k in range(30)])
    say("case: levenshtein cross 4 x 30")
    cr = ctx.levenshtein_cross(dev(Qs), qo, dev(DB), do).cpu().numpy()
    np.testing.assert_array_equal(cr, oracle.lev_cross(Qs, qo, DB, do, nthreads=8))
    rng = np.random.default_rng(512)
    for n, m in [(700, 9000), (20000, 15000)]:
        p, q = syms(rng, n), syms(rng, m)
        say(f"case: levenshtein long pair n={n} m={m}")
        assert ctx.levenshtein(dev(p), dev(q)).item() == oracle.lev(p, q)
        assert ctx.last_errors() == 0


def test_symbol_workload_full_size_sampled(ctx):
    g = json.load(open(os.path.join(HERE, "golden", "expected.json")))["levenshtein"]
    P, p_off, Q, q_off = workloads.symbol_pairs()
    say("case: levenshtein symbol workload, 4096 pairs")
    got = ctx.levenshtein_batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    assert ctx.last_errors() == 0
    np.testing.assert_array_equal(got[np.array(g["sample_index"])], np.array(g["levenshtein"], dtype=np.int64))
