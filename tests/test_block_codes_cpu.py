"""CPU replay of the block-code kernel's arithmetic (no GPU).

The block kernel (d = 1 directions) votes two codes per 2x2 block,
    code 1 = 11 a + b + 4 d + 5,   code 2 = 11 a + e + 1,
finds the blocks whose differences b - a, d - a, e - a leave [-1, 2] with a
byte-wise test on packed levels (3 subtractions and a mask per 4 pixels, where
a negative digit borrows from the byte above it, so every pixel from the lowest
set byte of a dword upwards is corrected), takes those votes back and counts
their four pairs one by one, and finally decodes the code counts.  This
test replays exactly that arithmetic in numpy (32-bit wrap-around included) and
checks:
  * every block outside the window is found (no block escapes the correction);
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
    k1 = 11 * a + b + 4 * d + 5
    k2 = 11 * a + e + 1
    assert k1.min() >= 0 and k1.max() < nbins and k2.min() >= 0 and k2.max() < nbins
    c1 = np.bincount(k1.ravel(), minlength=nbins).astype(np.int64)
    c2 = np.bincount(k2.ravel(), minlength=nbins).astype(np.int64)

    # the byte test, per lane chunk of 16 pixels as 4 packed dwords
    shp = (H, chunks, 16)
    La = pack(a.reshape(shp))
    Rb1 = pack((b + 1).reshape(shp))
    Ld1 = pack((d + 1).reshape(shp))
    Re1 = pack((e + 1).reshape(shp))
    m32 = np.uint64(0xFFFFFFFF)
    o = (((Rb1 - La) & m32) | ((Ld1 - La) & m32) | ((Re1 - La) & m32)) & np.uint64(0xFCFCFCFC)
    # a borrow only moves the bytes above the one it comes from, so every
    # pixel from the lowest set byte of a dword upwards is corrected
    flagged = np.zeros(shp, dtype=bool)
    seen = np.zeros(o.shape, dtype=bool)
    for j in range(4):
        byte = (o >> np.uint64(8 * j)) & np.uint64(0xFF)
        seen |= byte != 0
        flagged[..., j::4] = seen
    flagged = flagged.reshape(H, Wp)
    outside = ~(((b - a) >= -1) & ((b - a) <= 2) & ((d - a) >= -1) & ((d - a) <= 2) &
                ((e - a) >= -1) & ((e - a) <= 2))
    assert not np.any(outside & ~flagged), "a block outside the window was not found"

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
        bv = av + (bin_ & 3) - 1
        dv = av + ((bin_ >> 2) & 3) - 1
        c = c1[bin_]
        if 0 <= bv < N:
            fb[0, av, bv] += c
        if 0 <= bv < N and 0 <= dv < N:
            fb[1, bv, dv] += c
        if 0 <= dv < N:
            fb[2, av, dv] += c
    for bin_ in np.nonzero(c2)[0]:
        av, de = divmod(int(bin_), 12)
        ev = av + de - 1
        if de <= 3 and av < N and 0 <= ev < N:
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
    for N in (1, 2, 7, 32, 54):
        lv = np.arange(N + 1)
        a, b, d, e = np.meshgrid(lv, lv, lv, lv, indexing="ij")
        k1 = 11 * a + b + 4 * d + 5
        k2 = 11 * a + e + 1
        assert k1.min() >= 0 and k1.max() < 16 * N + 6
        assert k2.min() >= 0 and k2.max() < 16 * N + 6
