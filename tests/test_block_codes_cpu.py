"""CPU replay of the block-code kernel's arithmetic (no GPU).

The block kernel (d = 1 directions) votes two codes per 2x2 block,
    code 1 = 11 a + 4 b + d + 5,   code 2 = 11 a + 4 b + e + 5,
finds the blocks whose differences b - a, d - a, e - a leave [-1, 2] with an
exact byte-wise test on packed levels (each digit X - a + 1 biased by 0x40, so
no byte borrows from the next), takes those votes back and counts their four
pairs one by one, and finally decodes the code counts.  This
test replays exactly that arithmetic in numpy (32-bit wrap-around included) and
checks:
  * the byte test flags exactly the blocks outside the window;
  * every code, of any level combination with the sentinel, lies inside the
    code table (16 N + 6 bins), so no vote or take-back leaves it;
  * the decoded counts plus the corrections equal the oracle's four GLCMs on
    smooth, noisy, constant, checkerboard and ragged images.
"""

import numpy as np
import pytest

import oracle
import synth

OFFS = [(1, 0), (-1, 1), (0, 1), (1, 1)]


def pack(levels):
    """[..., 16] bytes -> [..., 4] uint32 little-endian dwords (pixel 4m + j in byte j)."""
    v = levels.astype(np.uint64).reshape(levels.shape[:-1] + (4, 4))
    return (v[..., 0] | (v[..., 1] << 8) | (v[..., 2] << 16) | (v[..., 3] << 24)).astype(np.uint64)


def replay(q, N):
    """Counts of the four d = 1 GLCMs as the block kernel computes them, from a
    level image q (H x W, levels in [0, N))."""
    H, W = q.shape
    chunks = (W + 15) // 16
    Wp = chunks * 16
    # levels with the sentinel N past the right edge and below the last row
    L = np.full((H + 1, Wp + 1), N, dtype=np.int64)
    L[:H, :W] = q
    a = L[:H, :Wp]
    b = L[:H, 1:Wp + 1]
    d = L[1:H + 1, :Wp]
    e = L[1:H + 1, 1:Wp + 1]
    nbins = 16 * N + 6
    k1 = 11 * a + 4 * b + d + 5
    k2 = 11 * a + 4 * b + e + 5
    assert k1.min() >= 0 and k1.max() < nbins and k2.min() >= 0 and k2.max() < nbins
    c1 = np.bincount(k1.ravel(), minlength=nbins).astype(np.int64)
    c2 = np.bincount(k2.ravel(), minlength=nbins).astype(np.int64)

    # the window test, per lane chunk of 16 pixels as 4 packed dwords: digits
    # X - a + 1 + 0x40 for X = b, d, e, in window iff 0x40..0x43
    shp = (H, chunks, 16)
    m32 = np.uint64(0xFFFFFFFF)
    lb = (pack(a.reshape(shp)) - np.uint64(0x41414141)) & m32
    db = (pack(b.reshape(shp)) - lb) & m32
    dd = (pack(d.reshape(shp)) - lb) & m32
    de = (pack(e.reshape(shp)) - lb) & m32
    o = ((~(db & dd & de) & np.uint64(0x40404040)) | ((db | dd | de) & np.uint64(0x3C3C3C3C))) & m32
    flagged = np.zeros(shp, dtype=bool)
    for j in range(4):
        flagged[..., j::4] = ((o >> np.uint64(8 * j)) & np.uint64(0xFF)) != 0
    flagged = flagged.reshape(H, Wp)
    outside = ~(((b - a) >= -1) & ((b - a) <= 2) & ((d - a) >= -1) & ((d - a) <= 2) &
                ((e - a) >= -1) & ((e - a) <= 2))
    assert np.array_equal(outside, flagged), "the byte test differs from the window"

    # corrections: take back both codes, count the four pairs into the
    # block GLCMs with a sentinel row and column
    n1 = N + 1
    fb = np.zeros((4, n1, n1), dtype=np.int64)
    fa, fbb, fd, fe = a[flagged], b[flagged], d[flagged], e[flagged]
    np.subtract.at(c1, k1[flagged], 1)
    np.subtract.at(c2, k2[flagged], 1)
    np.add.at(fb[0], (fa, fbb), 1)
    np.add.at(fb[1], (fbb, fd), 1)
    np.add.at(fb[2], (fa, fd), 1)
    np.add.at(fb[3], (fa, fe), 1)
    assert c1.min() >= 0 and c2.min() >= 0

    # decode
    for bin_ in np.nonzero(c1[:16 * N])[0]:
        av = bin_ >> 4
        bv = av + ((bin_ >> 2) & 3) - 1
        dv = av + (bin_ & 3) - 1
        c = c1[bin_]
        if 0 <= bv < N:
            fb[0, av, bv] += c
        if 0 <= bv < N and 0 <= dv < N:
            fb[1, bv, dv] += c
        if 0 <= dv < N:
            fb[2, av, dv] += c
    for bin_ in np.nonzero(c2[:16 * N])[0]:
        av = bin_ >> 4
        ev = av + (bin_ & 3) - 1
        if 0 <= ev < N:
            fb[3, av, ev] += c2[bin_]
    return fb[:, :N, :N]


CASES = [
    ("smooth", lambda: synth.smooth(96, 200, 8.0, 11), 32),
    ("smooth_sigma2", lambda: synth.smooth(80, 130, 2.0, 12), 32),
    ("noise", lambda: synth.uniform(40, 67, 13), 32),
    ("constant", lambda: synth.constant(33, 50, 255), 32),
    ("checker", lambda: synth.checkerboard(31, 45, 0, 255), 32),
    ("smooth_n8", lambda: synth.smooth(64, 100, 4.0, 14), 8),
    ("ragged_tiny", lambda: synth.uniform(3, 5, 15), 5),
    # levels 0..6 at N = 32: differences of -6..6, many borrows between bytes
    ("narrow_levels", lambda: (synth.uniform(90, 77, 18) % 56).astype(np.uint8), 32),
    ("one_row", lambda: synth.smooth(1, 70, 3.0, 16), 16),
    ("one_col", lambda: synth.smooth(50, 1, 3.0, 17), 16),
]


@pytest.mark.parametrize("name,make,N", CASES, ids=[c[0] for c in CASES])
def test_block_codes_equal_oracle(name, make, N):
    img = make()
    q = (img.astype(np.int64) * N) // 256
    got = replay(q, N)
    want = oracle.glcm(img, N, 0, 255, OFFS).astype(np.int64)
    assert np.array_equal(got, want)


def test_every_code_inside_table_for_all_level_combinations():
    for N in (1, 2, 7, 32, 54, 62):
        lv = np.arange(N + 1)
        a, b, d, e = np.meshgrid(lv, lv, lv, lv, indexing="ij")
        k1 = 11 * a + 4 * b + d + 5
        k2 = 11 * a + 4 * b + e + 5
        assert k1.min() >= 0 and k1.max() < 16 * N + 6
        assert k2.min() >= 0 and k2.max() < 16 * N + 6
        # biased digits of the window test: no borrow, bit 7 clear
        x = lv[:, None] - lv[None, :] + 0x41
        assert x.min() >= 0 and x.max() < 0x80
