"""Pins of the oracle's histogram, GLCM variants and Haralick statistics
against things other than the oracle itself: library routines (bincount,
weighted covariance, scipy's entropy), exact rational arithmetic, closed forms
of special matrices, and identities between the oracle's own functions that a
dropped term, a wrong index or a transposed operand would break."""

from fractions import Fraction

import numpy as np
import pytest
import scipy.stats

import oracle
import synth

RNG = np.random.default_rng(171006189)


def q_numpy(img, N, lo, hi):
    v = img.astype(np.int64)
    return np.where(v < lo, 0, np.where(v > hi, N - 1, (v - lo) * N // (hi - lo + 1)))


# ---------------------------------------------------------------- histogram

def test_histogram_u8_full_range_is_bincount():
    img = RNG.integers(0, 256, size=(37, 53), dtype=np.uint8)
    assert np.array_equal(oracle.histogram(img, 256, 0, 255), np.bincount(img.ravel(), minlength=256))


def test_histogram_u16_top_byte():
    img = RNG.integers(0, 65536, size=(29, 31), dtype=np.uint16)
    assert np.array_equal(oracle.histogram(img, 256, 0, 65535), np.bincount(img.ravel() >> 8, minlength=256))


@pytest.mark.parametrize("N,lo,hi", [(8, 0, 255), (5, 17, 200), (32, 3, 3), (1, 0, 255), (256, 100, 120)])
def test_histogram_vs_bincount_of_levels(N, lo, hi):
    img = RNG.integers(0, 256, size=(41, 23), dtype=np.uint8)
    want = np.bincount(q_numpy(img, N, lo, hi).ravel(), minlength=N)
    got = oracle.histogram(img, N, lo, hi)
    assert np.array_equal(got, want) and got.sum() == img.size


def test_histogram_strided_view():
    big = RNG.integers(0, 256, size=(40, 70), dtype=np.uint8)
    view = big[3:31, 5:62]
    assert np.array_equal(oracle.histogram(view, 16, 0, 255), oracle.histogram(view.copy(), 16, 0, 255))


@pytest.mark.parametrize("dx,dy", [(1, 0), (0, 1), (1, 1), (3, 2)])
def test_glcm_marginals_are_histograms(dx, dy):
    img = synth.smooth(45, 38, 2.0, 77)
    H, W = img.shape
    P = oracle.glcm(img, 16, 0, 255, [(dx, dy)])[0]
    assert np.array_equal(P.sum(axis=1), oracle.histogram(img[:H - dy, :W - dx], 16, 0, 255))
    assert np.array_equal(P.sum(axis=0), oracle.histogram(img[dy:, dx:], 16, 0, 255))


def test_zero_offset_diagonal_is_histogram():
    img = RNG.integers(0, 256, size=(19, 27), dtype=np.uint8)
    P = oracle.glcm(img, 32, 0, 255, [(0, 0)])[0]
    assert np.array_equal(np.diag(P), oracle.histogram(img, 32, 0, 255))
    assert P.sum() == np.trace(P)


# ---------------------------------------------------------------- symmetric

@pytest.mark.parametrize("d", [(1, 0), (-1, 1), (0, 2), (3, -1)])
def test_symmetric_counts_both_directions(d):
    img = RNG.integers(0, 256, size=(33, 29), dtype=np.uint8)
    P = oracle.glcm(img, 8, 0, 255, [d])
    both = oracle.glcm(img, 8, 0, 255, [d]).astype(np.int64) + oracle.glcm(img, 8, 0, 255, [(-d[0], -d[1])])
    S = oracle.symmetric(P)
    assert np.array_equal(S, both)
    assert np.array_equal(S[0], S[0].T)


def test_symmetric_wraps_modulo_two_to_32():
    P = np.zeros((1, 3, 3), dtype=np.uint32)
    P[0, 1, 1] = 2**31 + 5
    P[0, 0, 2] = 7
    S = oracle.symmetric(P)[0]
    assert S[1, 1] == 10 and S[0, 2] == 7 and S[2, 0] == 7 and S.sum() == 24


# ---------------------------------------------------------------- normalize

def test_normalize_hand_example():
    P = np.array([[1, 2], [3, 2]], dtype=np.uint32)
    assert np.array_equal(oracle.normalize(P), [[0.125, 0.25], [0.375, 0.25]])


def test_normalize_is_correctly_rounded_quotient():
    P = RNG.integers(0, 2**32, size=(3, 5, 5), dtype=np.uint64).astype(np.uint32)
    P[1] = RNG.integers(0, 4, size=(5, 5))
    got = oracle.normalize(P)
    for k in range(3):
        T = int(P[k].astype(np.uint64).sum())
        for v, g in zip(P[k].ravel(), got[k].ravel()):
            assert g == float(Fraction(int(v), T))


def test_normalize_empty_and_sum():
    P = np.zeros((2, 4, 4), dtype=np.uint32)
    P[1] = RNG.integers(0, 1000, size=(4, 4))
    got = oracle.normalize(P)
    assert not got[0].any()
    assert abs(got[1].sum() - 1.0) < 1e-14


# ---------------------------------------------------------------- average

def test_average_of_one_is_normalize():
    P = RNG.integers(0, 50, size=(6, 7, 7)).astype(np.uint32)
    assert np.array_equal(oracle.average(P, 1), oracle.normalize(P))


def test_average_of_opposite_offsets_is_normalized_symmetric():
    img = synth.smooth(40, 36, 3.0, 5)
    P = oracle.glcm(img, 16, 0, 255, [(1, 1), (-1, -1), (2, 0), (-2, 0)])
    got = oracle.average(P, 2)
    want = oracle.normalize(oracle.symmetric(P[0::2]))
    assert np.allclose(got, want, rtol=1e-15, atol=1e-18)


def test_average_matches_exact_rationals():
    P = RNG.integers(0, 2**20, size=(8, 4, 4)).astype(np.uint32)
    P[5] = 0  # an empty member contributes zeros but still counts in the mean
    m = 4
    got = oracle.average(P, m)
    for g in range(2):
        for i in range(4):
            for j in range(4):
                exact = sum((Fraction(int(P[k, i, j]), int(P[k].sum())) for k in range(g * m, g * m + m)
                             if P[k].sum()), Fraction(0)) / m
                assert abs(Fraction(got[g, i, j]) - exact) <= abs(exact) * Fraction(1, 2**50)


def test_average_rejects_ragged_groups():
    with pytest.raises(ValueError):
        oracle.average(np.zeros((5, 2, 2), dtype=np.uint32), 2)


# ---------------------------------------------------------------- Haralick f1..f13

def entropy(v):
    v = np.asarray(v, dtype=np.float64).ravel()
    return float(scipy.stats.entropy(v)) if v.sum() > 0 else 0.0


def haralick_numpy(P):
    """The thirteen statistics through library routines: bincount for the sum
    and difference distributions, weighted covariance, scipy's entropy."""
    P = P.astype(np.float64)
    p = P / P.sum()
    N = p.shape[0]
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    px, py = p.sum(axis=1), p.sum(axis=0)
    w = p.ravel()
    C = np.cov(np.vstack([I.ravel(), J.ravel()]), aweights=w, bias=True) if np.count_nonzero(w) > 1 else np.zeros((2, 2))
    ps = np.bincount((I + J).ravel(), weights=w, minlength=2 * N - 1)
    pd = np.bincount(np.abs(I - J).ravel(), weights=w, minlength=N)
    ts, td = np.arange(2 * N - 1), np.arange(N)
    f6 = float(np.dot(ts, ps))
    hx, hy, hxy = entropy(px), entropy(py), entropy(p)
    nz = p > 0
    hxy1 = float(-(p[nz] * np.log(np.outer(px, py)[nz])).sum())
    hxy2 = entropy(np.outer(px, py))
    single = np.count_nonzero(px) == 1 or np.count_nonzero(py) == 1
    return np.array([
        float((p ** 2).sum()),
        float(np.dot(((I - J) ** 2).ravel(), w)),
        1.0 if single else C[0, 1] / np.sqrt(C[0, 0] * C[1, 1]),
        C[0, 0] if not single or np.count_nonzero(px) > 1 else 0.0,
        float(np.dot(1.0 / (1.0 + (I - J).ravel() ** 2), w)),
        f6,
        float(np.dot((ts - f6) ** 2, ps)),
        entropy(ps),
        hxy,
        float(np.cov(td, aweights=pd, bias=True)) if np.count_nonzero(pd) > 1 else 0.0,
        entropy(pd),
        (hxy - hxy1) / max(hx, hy) if max(hx, hy) > 0 else 0.0,
        float(np.sqrt(max(0.0, 1.0 - np.exp(-2.0 * (hxy2 - hxy))))),
    ])


@pytest.mark.parametrize("seed", range(6))
def test_haralick_vs_library_routines(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 24))
    P = rng.integers(0, 1000, size=(N, N)).astype(np.uint32)
    P[rng.random((N, N)) < 0.5] = 0
    P[0, 0] += 1
    got, want = oracle.haralick(P), haralick_numpy(P)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-12), np.c_[got, want]


def test_haralick_on_image_glcms():
    img = synth.smooth(64, 64, 4.0, 11)
    P = oracle.glcm(img, 32, 0, 255, [(1, 0), (-1, 1), (0, 1), (1, 1)])
    got = oracle.haralick(P)
    for k in range(4):
        assert np.allclose(got[k], haralick_numpy(P[k]), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("a,b", [(0, 0), (3, 1), (0, 6)])
def test_haralick_single_bin(a, b):
    P = np.zeros((7, 7), dtype=np.uint32)
    P[a, b] = 123
    d2 = (a - b) ** 2
    want = [1, d2, 1, 0, 1 / (1 + d2), a + b, 0, 0, 0, 0, 0, 0, 0]
    assert np.allclose(oracle.haralick(P), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [2, 5, 16])
def test_haralick_uniform_matrix(N):
    P = np.full((N, N), 3, dtype=np.uint32)
    ps = np.convolve(np.full(N, 1 / N), np.full(N, 1 / N))  # sum of two independent uniform levels
    pd = np.r_[1 / N, 2 * (N - np.arange(1, N)) / N ** 2]  # their absolute difference
    td = np.arange(N)
    mud = np.dot(td, pd)
    idm = sum((N - abs(d)) / (1 + d * d) for d in range(-(N - 1), N)) / N ** 2
    want = [1 / N ** 2, (N * N - 1) / 6, 0, (N * N - 1) / 12, idm, N - 1, (N * N - 1) / 6,
            entropy(ps), 2 * np.log(N), np.dot((td - mud) ** 2, pd), entropy(pd), 0, 0]
    assert np.allclose(oracle.haralick(P), want, rtol=1e-12, atol=1e-7)


@pytest.mark.parametrize("N", [2, 8, 32])
def test_haralick_uniform_diagonal(N):
    P = np.diag(np.full(N, 9)).astype(np.uint32)
    L = np.log(N)
    want = [1 / N, 0, 1, (N * N - 1) / 12, 1, N - 1, (N * N - 1) / 3, L, L, 0, 0, -1, np.sqrt(1 - 1 / N ** 2)]
    assert np.allclose(oracle.haralick(P), want, rtol=1e-12, atol=1e-12)


def test_haralick_independent_product():
    ca, cb = RNG.integers(1, 50, size=9), RNG.integers(1, 50, size=9)
    P = np.outer(ca, cb).astype(np.uint32)
    a, b = ca / ca.sum(), cb / cb.sum()
    t = np.arange(9)
    f = oracle.haralick(P)
    var_a = np.dot((t - np.dot(t, a)) ** 2, a)
    assert abs(f[2]) < 1e-12 and abs(f[11]) < 1e-12 and f[12] < 1e-6
    assert np.isclose(f[8], entropy(a) + entropy(b), rtol=1e-12)
    assert np.isclose(f[0], (a ** 2).sum() * (b ** 2).sum(), rtol=1e-12)
    assert np.isclose(f[3], var_a, rtol=1e-12)
    assert np.isclose(f[5], np.dot(t, a) + np.dot(t, b), rtol=1e-12)


def test_haralick_transpose():
    P = RNG.integers(0, 100, size=(12, 12)).astype(np.uint32)
    f, ft = oracle.haralick(P), oracle.haralick(np.ascontiguousarray(P.T))
    same = [c for c in range(13) if c != 3]
    assert np.allclose(f[same], ft[same], rtol=1e-12, atol=1e-14)
    p = P / P.sum()
    py = p.sum(axis=0)
    t = np.arange(12)
    assert np.isclose(ft[3], np.dot((t - np.dot(t, py)) ** 2, py), rtol=1e-12)


def test_haralick_agrees_with_five_features():
    P = RNG.integers(0, 30, size=(5, 10, 10)).astype(np.uint32)
    P[2] = 0
    f13, f5 = oracle.haralick(P), oracle.features(P)
    # features: contrast, energy, entropy, homogeneity, correlation
    assert np.allclose(f13[:, [1, 0, 8, 4, 2]], f5, rtol=1e-12, atol=0)
    assert not f13[2].any()


# ---------------------------------------------------------------- f14, maximal correlation coefficient

def mcc_symmetric(P):
    """The same statistic through a different route: Q is similar to the
    symmetric S = B B^T with B(i, k) = p(i, k) / sqrt(px(i) py(k)), whose
    eigenvalues numpy's symmetric solver gives."""
    p = P.astype(np.float64) / P.sum()
    px, py = p.sum(axis=1), p.sum(axis=0)
    d = np.sqrt(np.outer(px, py))
    B = np.divide(p, d, out=np.zeros_like(p), where=d > 0)
    ev = np.sort(np.linalg.eigvalsh(B @ B.T))[::-1]
    return np.sqrt(max(0.0, ev[1])) if len(ev) > 1 else 0.0


@pytest.mark.parametrize("a,b", [(3, 1), (1, 3), (5, 5), (7, 0), (2, 9)])
def test_mcc_two_by_two(a, b):
    P = np.array([[a, b], [b, a]], dtype=np.uint32)
    # (near 0 the square root turns eigenvalue rounding of 1e-16 into 1e-8)
    assert abs(oracle.haralick_mcc(P) - abs(a - b) / (a + b)) < 1e-7


def test_mcc_closed_forms():
    assert abs(oracle.haralick_mcc(np.diag(np.full(9, 4)).astype(np.uint32)) - 1.0) < 1e-12
    ca, cb = RNG.integers(1, 60, size=11), RNG.integers(1, 60, size=11)
    assert oracle.haralick_mcc(np.outer(ca, cb).astype(np.uint32)) < 1e-6  # independent: 0
    blocks = np.zeros((8, 8), dtype=np.uint32)  # two independent components
    blocks[:3, :3] = np.outer(RNG.integers(1, 9, 3), RNG.integers(1, 9, 3))
    blocks[3:, 3:] = np.outer(RNG.integers(1, 9, 5), RNG.integers(1, 9, 5))
    assert abs(oracle.haralick_mcc(blocks) - 1.0) < 1e-9
    assert oracle.haralick_mcc(np.zeros((5, 5), dtype=np.uint32)) == 0.0
    assert oracle.haralick_mcc(np.full((1, 1), 3, dtype=np.uint32)) == 0.0


@pytest.mark.parametrize("seed", range(5))
def test_mcc_vs_symmetric_route_and_transpose(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 14))
    P = rng.integers(0, 200, size=(N, N)).astype(np.uint32)
    P[rng.random((N, N)) < 0.4] = 0
    P[int(rng.integers(0, N))] = 0  # an empty row
    P[0, 0] += 1
    m = oracle.haralick_mcc(P)
    assert abs(m - mcc_symmetric(P)) < 1e-9
    assert abs(m - oracle.haralick_mcc(np.ascontiguousarray(P.T))) < 1e-9
    assert 0.0 <= m <= 1.0 + 1e-12
