"""Pins for the oracle's 12-bit depth coding (Section V-A, Eq. 2 and Eq. 3):
hand-worked cases, the bit re-arrangement as a bijection, the continuity of
the folded LSBs (Fig. 6), and the quantiser's endpoints, monotonicity,
rounding and inverse."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "y12_cases.txt")


def golden_cases():
    out = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("->")
        f = lhs.split()
        out.append((f[0], f[1:], [int(v) for v in rhs.split()]))
    return out


@pytest.mark.parametrize("kind,args,want", golden_cases())
def test_golden(kind, args, want):
    if kind == "quant":
        zn, zf, mm = float(args[0]), float(args[1]), int(args[2])
        assert oracle.depth_codes(np.array([[mm]], np.uint16), zn, zf)[0, 0] == want[0]
    elif kind == "dequant":
        zn, zf, code = float(args[0]), float(args[1]), int(args[2])
        assert oracle.codes_depth(np.array([[code]], np.uint16), zn, zf)[0, 0] == want[0]
    else:
        c = np.array([int(v) for v in args], np.uint16).reshape(2, 2)
        Y, U, V = oracle.pack_y12(c)
        assert Y.reshape(-1).tolist() == want[:4]
        assert (int(U[0, 0]), int(V[0, 0])) == (want[4], want[5])
        assert np.array_equal(oracle.unpack_y12(Y, U, V), c)


def test_rearrangement_is_a_bijection():
    rng = np.random.default_rng(0)
    codes = rng.permutation(4096).astype(np.uint16).reshape(64, 64)
    assert np.array_equal(oracle.unpack_y12(*oracle.pack_y12(codes)), codes)
    # every byte pattern of the three planes is some code image: 4 * 8 + 8 + 8 bits
    # per 2x2 block on both sides
    Y = rng.integers(0, 256, (38, 70), dtype=np.uint8)
    U = rng.integers(0, 256, (19, 35), dtype=np.uint8)
    V = rng.integers(0, 256, (19, 35), dtype=np.uint8)
    c = oracle.unpack_y12(Y, U, V)
    assert c.max() <= 4095
    Y2, U2, V2 = oracle.pack_y12(c)
    assert np.array_equal(Y, Y2) and np.array_equal(U, U2) and np.array_equal(V, V2)


def test_folded_lsbs_are_continuous():
    # Fig. 6(c): the folded 8 LSBs of consecutive codes differ by at most one
    # and run up and down between 0 and 255 (a triangle wave of period 512)
    codes = np.arange(4096, dtype=np.uint16)
    blocks = np.repeat(np.repeat(codes.reshape(1, -1), 2, axis=0), 2, axis=1)
    Y, U, V = oracle.pack_y12(blocks)
    y = Y[0, ::2].astype(int)
    assert np.all(np.abs(np.diff(y)) <= 1)
    assert y.min() == 0 and y.max() == 255
    assert np.count_nonzero(np.diff(y) == 0) == 15        # one flat step at each MSB change
    # equal MSBs interleave to a value that increases with them
    u = U[0].astype(int)
    assert np.all(np.diff(u) >= 0) and u[0] == 0 and u[-1] == 255
    assert np.array_equal(U, V)


def exact_code(mm, zn, zf):
    """Eq. 2 in exact rational arithmetic (clipping planes as float32)."""
    z = Fraction(int(mm), 1000)
    fzn, fzf = Fraction(float(np.float32(zn))), Fraction(float(np.float32(zf)))
    return 4093 * (1 / z - 1 / fzf) / (1 / fzn - 1 / fzf) + 2


@pytest.mark.parametrize("zn,zf", [(0.5, 1.5), (0.3, 20.0), (1.0, 8.0)])
def test_quantiser_range_monotone_and_rounding(zn, zf):
    mm = np.arange(0, 65536, dtype=np.uint16).reshape(256, 256)
    codes = oracle.depth_codes(mm, zn, zf).reshape(-1).astype(int)
    assert codes[0] == 1 and codes[65535] == 0
    codes[65535] = 1            # the background signal; beyond z_far otherwise
    lo, hi = int(np.ceil(zn * 1000)), int(np.floor(zf * 1000))
    # the clipping planes and everything between them take codes 2..4095
    c = codes[lo:hi + 1]
    assert c.min() >= 2 and c.max() <= 4095
    assert codes[round(zn * 1000)] == 4095 and codes[round(zf * 1000)] == 2
    assert np.all(np.diff(codes[lo:hi + 1]) <= 0)          # farther -> smaller disparity code
    # beyond the planes the end codes continue while the rounded value stays
    # in 2..4095 (within half a code of the plane), then code 1
    far = codes[hi + 1:]
    n2 = int(np.count_nonzero(far == 2))
    assert np.all(far[:n2] == 2) and np.all(far[n2:] == 1)
    edge = hi + n2                                         # last millimetre coded 2
    assert exact_code(edge, zn, zf) >= Fraction(3, 2) > exact_code(edge + 1, zn, zf)
    near = codes[1:lo][::-1]
    n4 = int(np.count_nonzero(near == 4095))
    assert np.all(near[:n4] == 4095) and np.all(near[n4:] == 1)
    edge = lo - n4
    assert exact_code(edge, zn, zf) < Fraction(8191, 2) <= exact_code(edge - 1, zn, zf)
    # rounding within half a code of the exact rational value of Eq. 2
    for m in np.linspace(lo, hi, 97).astype(int):
        assert abs(codes[m] - exact_code(m, zn, zf)) <= Fraction(1, 2) + Fraction(1, 10 ** 9)


@pytest.mark.parametrize("zn,zf", [(0.5, 1.5), (0.3, 20.0), (1.0, 8.0)])
def test_dequantiser_inverts_the_quantiser(zn, zf):
    codes = np.arange(4096, dtype=np.uint16).reshape(64, 64)
    mm = oracle.codes_depth(codes, zn, zf).reshape(-1).astype(int)
    assert mm[0] == 65535 and mm[1] == 0
    d = mm[2:]
    assert np.all(np.diff(d) <= 0)
    assert d.min() == round(zn * 1000) and d.max() == round(zf * 1000)
    # decode -> encode -> decode is the identity on decoded values, and where a
    # code's bin spans several millimetres the code itself comes back
    back = oracle.depth_codes(mm.reshape(64, 64).astype(np.uint16), zn, zf).reshape(-1).astype(int)
    again = oracle.codes_depth(back.reshape(64, 64).astype(np.uint16), zn, zf).reshape(-1).astype(int)
    assert np.array_equal(again[2:], d)
    wide = np.zeros(4096, bool)
    wide[3:4095] = (mm[2:4094] - mm[4:4096]) >= 4
    if zf / zn > 5:
        assert wide.sum() > 100
    assert np.array_equal(back[wide], np.arange(4096)[wide])
