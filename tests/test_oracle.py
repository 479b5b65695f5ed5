"""Pins for the CPU oracle's pair counts (Eq. (1)) and quantizer (Section I.A).

Each test fixes the oracle against something other than itself: brute-force
enumeration of every pixel pair, a vectorised numpy formulation, closed forms
(totals, constant and checkerboard images), identities (transpose for opposite
offsets, marginals equal histograms, additivity over row strips) and
hand-derived fixtures in tests/golden/.
"""

import json
import os
import random

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- quantizer

def test_quantizer_hand_fixture():
    with open(os.path.join(GOLDEN, "quantizer_hand.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        for v, q in case["pairs"]:
            assert oracle.quantize(v, case["N"], case["lo"], case["hi"]) == q, (case, v)


QUANT_CASES = [  # (bits, N, lo, hi)
    (8, 8, 0, 255), (8, 32, 0, 255), (8, 16, 0, 255), (8, 256, 0, 255), (8, 7, 13, 200),
    (8, 5, 0, 0), (8, 3, 255, 255), (8, 100, 50, 60), (8, 1, 0, 255),
    (16, 64, 0, 65535), (16, 257, 1000, 60000), (16, 4096, 0, 65535), (16, 13, 0, 65535),
    (16, 4096, 7, 700),
]


@pytest.mark.parametrize("bits,N,lo,hi", QUANT_CASES)
def test_quantizer_exhaustive_properties(bits, N, lo, hi):
    """Over every input value: clamping outside [lo, hi]; monotone; range
    [0, N); the first value reaching level t is lo + ceil(t*D/N) (D = hi-lo+1),
    which also fixes every level's population to floor(D/N) or ceil(D/N)."""
    vals = np.arange(1 << bits)
    q = oracle.quantize_array(vals, N, lo, hi)
    assert q.min() >= 0 and q.max() <= N - 1
    assert np.all(q[vals < lo] == 0)
    assert np.all(q[vals > hi] == N - 1)
    assert np.all(np.diff(q) >= 0)
    D = hi - lo + 1
    inr = q[lo:hi + 1]
    for t in range(1, N):
        first = lo + -(-t * D // N)              # ceil(t*D/N), Python big ints
        if first <= hi:
            assert inr[first - lo] >= t and (first == lo or inr[first - lo - 1] < t), t
        else:
            assert np.all(inr < t)
    if N <= D:
        pop = np.bincount(inr, minlength=N)
        assert set(np.unique(pop)) <= {D // N, -(-D // N)}
        assert q[lo] == 0 and q[hi] == N - 1


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5, 8])
def test_quantizer_power_of_two_is_shift(k):
    """With [lo, hi] the whole 8- or 16-bit range and N = 2^k the reduction is a right shift."""
    v8 = np.arange(256)
    assert np.array_equal(oracle.quantize_array(v8, 1 << k, 0, 255), v8 >> (8 - k))
    v16 = np.arange(0, 65536, 7)
    assert np.array_equal(oracle.quantize_array(v16, 1 << (k + 4), 0, 65535), v16 >> (12 - k))


# ---------------------------------------------------------------- brute force

def brute_force(img, N, lo, hi, offsets):
    """Eq. (1) by enumerating every ordered pair of pixel positions (p1, p2) and
    keeping those displaced by exactly (dx, dy).  O((W*H)^2): tiny images only."""
    H, W = img.shape
    lv = oracle.quantize_array(img, N, lo, hi)
    pos = [(x, y) for y in range(H) for x in range(W)]
    out = np.zeros((len(offsets), N, N), dtype=np.int64)
    for k, (dx, dy) in enumerate(offsets):
        for (x1, y1) in pos:
            for (x2, y2) in pos:
                if x2 - x1 == dx and y2 - y1 == dy:
                    out[k, lv[y1, x1], lv[y2, x2]] += 1
    return out


def test_golden_hand_counts():
    with open(os.path.join(GOLDEN, "hand_4x3.json")) as f:
        fx = json.load(f)
    img = np.array(fx["image"], dtype=np.uint8)
    P = oracle.glcm(img, fx["N"], fx["lo"], fx["hi"], fx["offsets"])
    for k, (dx, dy) in enumerate(fx["offsets"]):
        assert P[k].tolist() == fx["counts"][f"{dx},{dy}"], (dx, dy)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_vs_brute_force(seed):
    r = random.Random(seed)
    W, H = r.randint(1, 8), r.randint(1, 8)
    dtype = np.uint8 if seed % 2 == 0 else np.uint16
    top = np.iinfo(dtype).max
    lo = r.randint(0, top // 2)
    hi = r.randint(lo, top)
    N = r.randint(1, 9)
    g = synth.rng(1000 + seed)
    # concentrate values around [lo, hi] so every level and both clamps occur
    img = g.integers(max(0, lo - 3), min(top, hi + 3) + 1, size=(H, W)).astype(dtype)
    offsets = [(r.randint(-4, 4), r.randint(-4, 4)) for _ in range(r.randint(1, 5))]
    got = oracle.glcm(img, N, lo, hi, offsets)
    assert np.array_equal(got, brute_force(img, N, lo, hi, offsets))


def test_oracle_strided_view_matches_copy():
    g = synth.rng(7)
    big = g.integers(0, 256, size=(37, 53), dtype=np.uint8)
    view = big[3:30, 5:44]          # row stride 53 elements, width 39
    offs = [(1, 0), (-2, 3), (0, 1), (4, 4)]
    assert np.array_equal(oracle.glcm(view, 16, 0, 255, offs),
                          oracle.glcm(np.ascontiguousarray(view), 16, 0, 255, offs))


# ---------------------------------------------------------------- vectorised formulation

def numpy_glcm(img, N, lo, hi, offsets):
    """Independent formulation: level lookup table over the value domain,
    array slicing for the overlapping rectangles, bincount of i*N + j."""
    top = np.iinfo(img.dtype).max
    lut = oracle.quantize_array(np.arange(top + 1), N, lo, hi)
    lv = lut[img]
    H, W = img.shape
    out = np.zeros((len(offsets), N, N), dtype=np.int64)
    for k, (dx, dy) in enumerate(offsets):
        w, h = W - abs(dx), H - abs(dy)
        if w <= 0 or h <= 0:
            continue
        x0, y0 = max(0, -dx), max(0, -dy)
        a = lv[y0:y0 + h, x0:x0 + w]
        b = lv[y0 + dy:y0 + dy + h, x0 + dx:x0 + dx + w]
        out[k] = np.bincount((a * N + b).ravel(), minlength=N * N).reshape(N, N)
    return out


@pytest.mark.parametrize("case", [
    ("uniform", np.uint8, 300, 257, 32, 0, 255, [(1, 0), (-1, 1), (0, 1), (1, 1)]),
    ("smooth", np.uint8, 256, 384, 8, 0, 255, [(1, 0), (-4, 4), (4, 0), (-2, -3)]),
    ("smooth", np.uint16, 200, 128, 64, 0, 65535, synth.offsets_for([1, 2, 4])),
    ("uniform", np.uint16, 64, 99, 50, 1000, 50000, [(0, 0), (3, -1), (70, 0), (0, 64)]),
])
def test_oracle_vs_numpy(case):
    kind, dtype, H, W, N, lo, hi, offs = case
    img = (synth.uniform(H, W, 11, dtype) if kind == "uniform"
           else synth.smooth(H, W, 4.0, 12, dtype))
    assert np.array_equal(oracle.glcm(img, N, lo, hi, offs), numpy_glcm(img, N, lo, hi, offs))


# ---------------------------------------------------------------- closed forms and identities

@pytest.mark.parametrize("W,H", [(1, 1), (1, 9), (9, 1), (17, 5), (64, 33)])
def test_total_count(W, H):
    img = synth.uniform(H, W, 3)
    offs = [(dx, dy) for dx in range(-5, 6, 2) for dy in range(-3, 4)]
    P = oracle.glcm(img, 8, 0, 255, offs)
    for k, (dx, dy) in enumerate(offs):
        assert int(P[k].sum()) == max(0, W - abs(dx)) * max(0, H - abs(dy))


def test_transpose_for_opposite_offsets():
    img = synth.smooth(96, 80, 3.0, 5)
    offs = [(1, 0), (-1, 1), (0, 1), (1, 1), (3, -2), (0, 0)]
    P = oracle.glcm(img, 16, 0, 255, offs)
    Q = oracle.glcm(img, 16, 0, 255, [(-dx, -dy) for dx, dy in offs])
    for k in range(len(offs)):
        assert np.array_equal(Q[k], P[k].T)


def test_constant_image_single_bin():
    img = synth.constant(64, 48, 128)
    offs = synth.offsets_for([1, 2])
    P = oracle.glcm(img, 32, 0, 255, offs)
    for k, (dx, dy) in enumerate(offs):
        assert P[k, 16, 16] == (48 - abs(dx)) * (64 - abs(dy))
        assert np.count_nonzero(P[k]) == 1


def test_constant_4096_closed_form():
    """4096^2 image of value 128 at N=32, d=1 at the four angles: bin (16,16)
    holds 4095*4096 for the axis offsets and 4095^2 for the diagonals."""
    img = synth.constant(4096, 4096, 128)
    P = oracle.glcm(img, 32, 0, 255, synth.offsets_for([1]))
    assert [int(P[k, 16, 16]) for k in range(4)] == [16773120, 16769025, 16773120, 16769025]


def checker_expected(W, H, dx, dy, A, B, N):
    """Closed form for a two-level checkerboard (a at even x+y, b at odd)."""
    P = np.zeros((N, N), dtype=np.int64)
    w, h = W - abs(dx), H - abs(dy)
    if w <= 0 or h <= 0:
        return P
    x0, y0 = max(0, -dx), max(0, -dy)
    wh = w * h
    s = 0 if wh % 2 == 0 else (1 if (x0 + y0) % 2 == 0 else -1)
    E = (wh + s) // 2                  # first pixels with even x+y
    if (dx + dy) % 2 == 0:
        P[A, A] += E
        P[B, B] += wh - E
    else:
        P[A, B] += E
        P[B, A] += wh - E
    return P


@pytest.mark.parametrize("W,H", [(8, 8), (7, 9), (1, 5), (13, 1), (31, 17)])
def test_checkerboard_closed_form(W, H):
    a, b, N = 40, 200, 8
    A, B = a * N // 256, b * N // 256
    img = synth.checkerboard(H, W, a, b)
    offs = [(dx, dy) for dx in range(-3, 4) for dy in range(-3, 4)]
    P = oracle.glcm(img, N, 0, 255, offs)
    for k, (dx, dy) in enumerate(offs):
        assert np.array_equal(P[k], checker_expected(W, H, dx, dy, A, B, N)), (dx, dy)


def test_marginals_are_histograms():
    img = synth.smooth(70, 90, 2.0, 9)
    N = 16
    lut = oracle.quantize_array(np.arange(256), N, 0, 255)
    lv = lut[img]
    H, W = img.shape
    for dx, dy in [(1, 0), (-1, 1), (2, 3), (-3, -2), (0, 0)]:
        P = oracle.glcm(img, N, 0, 255, [(dx, dy)])[0]
        x0, y0 = max(0, -dx), max(0, -dy)
        w, h = W - abs(dx), H - abs(dy)
        first = lv[y0:y0 + h, x0:x0 + w]
        second = lv[y0 + dy:y0 + dy + h, x0 + dx:x0 + dx + w]
        assert np.array_equal(P.sum(axis=1), np.bincount(first.ravel(), minlength=N))
        assert np.array_equal(P.sum(axis=0), np.bincount(second.ravel(), minlength=N))
        if (dx, dy) == (0, 0):
            assert np.array_equal(np.diag(P), np.bincount(lv.ravel(), minlength=N))
            assert np.count_nonzero(P - np.diag(np.diag(P))) == 0


@pytest.mark.parametrize("strip", [1, 3, 16, 29])
def test_strip_additivity_with_halo(strip):
    """Row strips that carry halo rows above and below and count only pairs
    whose first pixel lies in their own rows add up to the whole image: the
    2-D reading of the chunk bounds of Eq. (7)-(9)."""
    img = synth.smooth(61, 45, 3.0, 21, np.uint16, noise_frac=0.05)
    offs = [(1, 0), (-2, 2), (0, 4), (3, -1), (-1, -3)]
    up = max(0, max(-dy for _, dy in offs))
    down = max(0, max(dy for _, dy in offs))
    H = img.shape[0]
    whole = oracle.glcm(img, 64, 0, 65535, offs).astype(np.int64)
    acc = np.zeros_like(whole)
    for y0 in range(0, H, strip):
        y1 = min(H, y0 + strip)
        a, b = max(0, y0 - up), min(H, y1 + down)
        acc += oracle.glcm(img[a:b], 64, 0, 65535, offs, rows=(y0 - a, y1 - a))
    assert np.array_equal(acc, whole)


def test_offset_beyond_image_is_all_zero():
    img = synth.uniform(5, 6, 1)
    P = oracle.glcm(img, 4, 0, 255, [(6, 0), (0, 5), (-7, 2), (100, -100)])
    assert not P.any()
