"""The phase schedule of the pipelined single-pair kernel, checked on the
CPU (no GPU): a model of which barrier phase writes and which reads every
value the kernel hands between waves -- the hand-off rings between the
computing waves of a workgroup, the column ring the helper wave fills, the
incoming link ring and the link rows between workgroups -- with the shape
constants read from the kernel's header.  Every value must be written in an
earlier phase than any phase that reads it (waves of a workgroup meet only
at the phase barrier), and no ring slot may be overwritten before its last
read.  A planted lag one group too short must fail."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2404_05708_amd", "csrc", "ffd_pipe_args.h")


def constants():
    text = open(HDR).read()
    out = {}
    for name in ("kPipeWaves", "kPipeLag", "kPipeRing", "kPipeGroup"):
        out[name] = int(re.search(r"constexpr int %s = (\d+);" % name, text).group(1))
    return out


def ring_write_step(j):
    """Lane 63 computes column j at step j + 63 and writes batches of four
    at the steps t with t % 4 == 2 (columns t - 66 .. t - 63)."""
    t = j + 63
    return t + ((2 - t) % 4)


def check(m, K, lag=None):
    W, L, RING, G = K["kPipeWaves"], K["kPipeLag"] if lag is None else lag, K["kPipeRing"], K["kPipeGroup"]
    gwork = (m - 1) // G + 6
    phase = lambda w, t: t // G + w * L     # phase of wave w's step t
    # hand-off ring of wave w, read by wave w + 1 at the start of its group
    for w in range(W - 1):
        for j in range(m):
            wr = phase(w, ring_write_step(j))
            rd = j // G + (w + 1) * L
            assert wr < rd, ("hand-off", m, w, j, wr, rd)
            over = phase(w, ring_write_step(j + RING))
            assert over > rd, ("hand-off overwrite", m, w, j)
    # the last step of a wave covers the ring write of the last column, and
    # the ring still holds it when the result is read
    assert ring_write_step(m - 1) <= G * gwork - 1
    assert (G * gwork - 1) - 63 < m - 1 + RING
    # column ring (2 RING entries, groups of G): the helper puts group h at
    # phase h - 2; wave w reads it at phase h - 1 + w L (one group ahead)
    QR = 2 * RING
    for h in range(0, (m + 63) // G + 2):
        put = h - 2
        for w in range(W):
            rd = max(h - 1, 0) + w * L
            assert put < rd, ("column ring", m, h, w)
            assert (h + QR // G) - 2 > rd, ("column ring overwrite", m, h, w)
    # negative columns (the +inf prefill, slots QR - 64 .. QR - 1) are read
    # up to step 63 and overwritten by group QR / G - 4
    assert (QR // G - 4) - 2 > 63 // G + (W - 1) * L
    # incoming link ring: group h taken by the helper at phase h - 1, read
    # by the first wave at phase h, slot reused by group h + RING / G
    for h in range(gwork):
        assert h - 1 < h and (h + RING // G) - 1 > h
    # outgoing link: the helper stores column j of the last wave's row at
    # phase j / G + 5 + (W - 1) L, after the ring write and before reuse,
    # and every column below m is stored within the phases of the pass
    phases = gwork + (W - 1) * L
    for j in range(m):
        st = j // G + 5 + (W - 1) * L
        assert phase(W - 1, ring_write_step(j)) < st, ("link store", m, j)
        assert phase(W - 1, ring_write_step(j + RING)) > st
        assert st <= phases - 1, ("link coverage", m, j)


@pytest.mark.parametrize("m", [2, 3, 15, 16, 17, 63, 64, 65, 100, 255, 256, 257, 700, 1000, 4097])
def test_pipe_schedule(m):
    check(m, constants())


def test_pipe_schedule_catches_a_short_lag():
    K = constants()
    with pytest.raises(AssertionError):
        check(700, K, lag=K["kPipeLag"] - 1)
