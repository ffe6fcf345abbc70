"""The class of caller-given ridge lists the library accepts (rd_validate_ridges, host only):
every list step 2 can produce passes, lists that could break the exact integer votes fail,
and over every direction code of the class a vote counter stays far below the bounds the
fused vote kernel relies on (16-bit counters, 32-bit band sums).  No GPU."""
import ctypes

import numpy as np
import pytest

from oracle import ridge_hough as O
from paper_1310_1371_amd import native as N
from paper_1310_1371_amd import synth


def _lib():
    return N.lib()


def _validate(xy, q, W, H):
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    q = np.ascontiguousarray(q, dtype=np.int16)
    return _lib().rd_validate_ridges(xy.ctypes.data, q.ctypes.data, len(xy), W, H)


def _all_oracle_codes():
    th = np.linspace(0.0, 2.0 * np.pi, 400_000, endpoint=False)
    qx, qy = O.direction_code(np.cos(th), np.sin(th))
    return np.unique(np.stack([qx, qy], 1), axis=0)


def _distinct_pixels(n, W=1024):
    i = np.arange(n)
    return np.stack([i % W, i // W], 1), W, int((n + W - 1) // W)


def test_every_code_of_step_one_is_accepted():
    codes = _all_oracle_codes()
    xy, W, H = _distinct_pixels(len(codes))
    assert _validate(xy, codes, W, H) == N.RD_OK


def test_oracle_ridge_lists_are_accepted():
    for f in (synth.config1(), synth.config2()):
        xs, ys, qx, qy, _ = O.ridges(f.image, f.params)
        H, W = f.image.shape
        assert _validate(np.stack([xs, ys], 1), np.stack([qx, qy], 1), W, H) == N.RD_OK


def test_negated_codes_are_rejected():
    codes = _all_oracle_codes()[::97]
    for q in -codes:
        assert _validate([[3, 4]], [q], 8, 8) == N.RD_E_INVALID, q


@pytest.mark.parametrize("q,ok", [
    ((16384, 0), True), ((0, 16384), True), ((-16384, 1), True), ((11585, 11585), True),
    ((16383, 0), True),                                 # 16383^2 = 2^28 - 32767
    ((16385, 0), False),                                # 16385^2 = 2^28 + 32769
    ((16384, 181), True), ((16384, 182), False),        # + 32761 and + 33124
    ((0, 0), False), ((-16384, 0), False), ((16384, -1), False), ((0, -16384), False),
    ((32767, 0), False), ((-32768, -32768), False)])
def test_code_predicate_cases(q, ok):
    """|q|^2 within 2^15 = 32768 of 2^28 and qy > 0 (or qy == 0, qx > 0); the squares are
    worked out by hand: (2^14 +- 1)^2 = 2^28 +- 2^15 + 1."""
    assert (_validate([[1, 1]], [q], 4, 4) == N.RD_OK) == ok


def test_repeats_and_off_frame_pixels_are_rejected():
    q = [[0, 16384], [16384, 0]]
    assert _validate([[2, 3], [3, 2]], q, 8, 8) == N.RD_OK
    assert _validate([[2, 3], [2, 3]], q, 8, 8) == N.RD_E_INVALID
    assert _validate([[2, 3], [8, 2]], q, 8, 8) == N.RD_E_INVALID
    assert _validate([[2, -1], [3, 2]], q, 8, 8) == N.RD_E_INVALID
    assert _validate(np.zeros((0, 2)), np.zeros((0, 2)), 8, 8) == N.RD_OK
    lib = _lib()
    assert lib.rd_validate_ridges(None, None, 0, 8, 8) == N.RD_OK
    assert lib.rd_validate_ridges(None, None, 1, 8, 8) == N.RD_E_INVALID
    assert lib.rd_validate_ridges(None, None, -1, 8, 8) == N.RD_E_INVALID


def test_counter_bound_over_the_accepted_class():
    """Every canonical integer code with |q|^2 within 2^15 of 2^28, both signs, at the
    largest level r = 127: the distinct offsets rho(127, q) bound any vote counter over a
    list of distinct pixels (a pixel votes once per sign and its two signs never meet at
    r >= 1).  The count stays below 4096, so two 8-tap bands of weights <= 2^15 sum below 2^31
    and the 16-bit counters cannot carry."""
    lo, hi = (1 << 28) - (1 << 15), (1 << 28) + (1 << 15)
    qx = np.arange(-16386, 16387, dtype=np.int64)
    rest_lo = lo - qx * qx
    rest_hi = hi - qx * qx
    ylo = np.ceil(np.sqrt(np.maximum(rest_lo, 0))).astype(np.int64)
    yhi = np.floor(np.sqrt(np.maximum(rest_hi, 0))).astype(np.int64)
    cx, cy = [], []
    for x, a, b in zip(qx.tolist(), ylo.tolist(), yhi.tolist()):
        for y in range(max(a - 1, 0), b + 2):
            n2 = x * x + y * y
            if lo <= n2 <= hi and (y > 0 or (y == 0 and x > 0)):
                cx.append(x)
                cy.append(y)
    cx, cy = np.array(cx), np.array(cy)
    assert len(cx) > 50_000
    offs = set()
    for sgn in (1, -1):
        ox = O.vote_offset(127, sgn * cx)
        oy = O.vote_offset(127, sgn * cy)
        offs.update(zip(ox.tolist(), oy.tolist()))
    n = len(offs)
    assert 2 * np.pi * 127 < n < 1200
    assert 16 * n * 2 ** 15 < 2 ** 31 and n < 1 << 16
