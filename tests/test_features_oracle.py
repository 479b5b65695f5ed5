"""Pins for the oracle's Haralick statistics (cited in the introduction).

Closed forms for constant, checkerboard, uniform and uniform-diagonal
matrices; a 2x2 family with an exact correlation; and library routines that
compute the same quantities another way (scipy's entropy, numpy's weighted
covariance).
"""

import math

import numpy as np
import pytest
import scipy.stats

import oracle
import synth

IDX = dict(contrast=0, energy=1, entropy=2, homogeneity=3, correlation=4)


def close(a, b, rel=1e-12, abs_=1e-12):
    return abs(a - b) <= max(abs_, rel * abs(b))


def test_empty_glcm_is_all_zero():
    assert np.array_equal(oracle.features(np.zeros((3, 4, 4), np.uint32)), np.zeros((3, 5)))


def test_constant_image_features():
    P = oracle.glcm(synth.constant(50, 40, 77), 16, 0, 255, synth.offsets_for([1]))
    f = oracle.features(P)
    for k in range(4):
        assert f[k].tolist() == [0.0, 1.0, 0.0, 1.0, 1.0]


@pytest.mark.parametrize("dxdy_odd", [True, False])
def test_checkerboard_features(dxdy_odd):
    a, b, N = 16, 240, 16
    A, B = a * N // 256, b * N // 256           # 1 and 15
    img = synth.checkerboard(20, 31, a, b)      # both offsets below cover an even count
    off = (1, 0) if dxdy_odd else (1, 1)
    f = oracle.features(oracle.glcm(img, N, 0, 255, [off]))[0]
    if dxdy_odd:
        expect = [(A - B) ** 2, 0.5, math.log(2), 1 / (1 + (A - B) ** 2), -1.0]
    else:
        expect = [0.0, 0.5, math.log(2), 1.0, 1.0]
    for got, want in zip(f, expect):
        assert close(got, want), (f, expect)


@pytest.mark.parametrize("N", [2, 3, 8, 32])
def test_uniform_matrix_features(N):
    P = np.full((N, N), 7, dtype=np.uint32)
    f = oracle.features(P)
    homog = (N + 2 * sum((N - k) / (1 + k * k) for k in range(1, N))) / N ** 2
    expect = [(N * N - 1) / 6, 1 / N ** 2, 2 * math.log(N), homog, 0.0]
    for got, want in zip(f, expect):
        assert close(got, want, abs_=1e-13), (N, f, expect)


@pytest.mark.parametrize("N", [2, 5, 64])
def test_uniform_diagonal_features(N):
    P = np.diag(np.full(N, 3, dtype=np.uint32))
    f = oracle.features(P)
    expect = [0.0, 1 / N, math.log(N), 1.0, 1.0]
    for got, want in zip(f, expect):
        assert close(got, want), (N, f, expect)


@pytest.mark.parametrize("a,b", [(5, 1), (1, 5), (3, 3), (1000, 1), (0, 9)])
def test_two_by_two_correlation(a, b):
    """P = [[a, b], [b, a]] has equal marginals 1/2, 1/2 and correlation (a-b)/(a+b)."""
    P = np.array([[a, b], [b, a]], dtype=np.uint32)
    f = oracle.features(P)
    assert close(f[IDX["correlation"]], (a - b) / (a + b))
    assert close(f[IDX["contrast"]], 2 * b / (2 * a + 2 * b))


def test_single_occupied_row_gives_correlation_one():
    P = np.zeros((6, 6), np.uint32)
    P[2, :] = [1, 4, 0, 2, 9, 3]
    assert oracle.features(P)[IDX["correlation"]] == 1.0
    P = np.zeros((6, 6), np.uint32)
    P[:, 4] = [1, 4, 0, 2, 9, 3]
    assert oracle.features(P)[IDX["correlation"]] == 1.0


@pytest.mark.parametrize("seed", range(6))
def test_features_vs_library_routines(seed):
    """Entropy via scipy.stats.entropy (natural log), correlation via numpy's
    frequency-weighted covariance, energy and contrast via plain numpy."""
    N = [4, 8, 16, 32, 64, 13][seed]
    img = synth.smooth(120, 100, 1.0 + seed, 40 + seed) if seed % 2 else synth.uniform(120, 100, 40 + seed)
    P = oracle.glcm(img, N, 0, 255, [(1, 0)])[0]
    f = oracle.features(P)
    p = P.astype(np.float64) / P.sum()
    assert close(f[IDX["entropy"]], scipy.stats.entropy(p.ravel()), rel=1e-10)
    assert close(f[IDX["energy"]], float(np.dot(p.ravel(), p.ravel())), rel=1e-10)
    ii, jj = np.indices((N, N))
    assert close(f[IDX["contrast"]], float(((ii - jj) ** 2 * p).sum()), rel=1e-10)
    assert close(f[IDX["homogeneity"]], float((p / (1 + (ii - jj) ** 2)).sum()), rel=1e-10)
    c = np.cov(ii.ravel(), jj.ravel(), fweights=P.ravel().astype(np.int64), bias=True)
    assert close(f[IDX["correlation"]], c[0, 1] / math.sqrt(c[0, 0] * c[1, 1]), rel=1e-9)


def test_features_transpose_invariant():
    img = synth.smooth(90, 70, 2.5, 77)
    P = oracle.glcm(img, 16, 0, 255, [(2, 1)])[0]
    assert np.allclose(oracle.features(P), oracle.features(np.ascontiguousarray(P.T)), rtol=1e-12, atol=0)
