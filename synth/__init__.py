"""Seeded synthetic images shared by the tests, the benchmark and the smoke check.

This module only draws pixels. It holds none of the co-occurrence arithmetic
(no quantization, no pair visiting, no counting), so both the HIP path and the
CPU oracle can take their inputs from it without sharing any of the method.

The paper measures on two sample photographs that are not available: one with
small gray-level changes (Fig. 1(a)) and one with large changes (Fig. 1(b)),
Section II.A. They are replaced here by:

* ``smooth``  - white Gaussian noise blurred with a Gaussian of std ``sigma``
                pixels (periodic boundary, exact Gaussian transfer function in
                the Fourier domain), min-max rescaled to the full dtype range;
                stands in for Fig. 1(a).
* ``uniform`` - i.i.d. uniform pixels over the dtype range; stands in for
                Fig. 1(b).
* ``constant`` - one value everywhere, the worst case for same-address votes.
* ``checkerboard`` - two values on alternating pixels, for closed forms.

Every generator takes an explicit seed and uses numpy's PCG64.
"""

from __future__ import annotations

import hashlib

import numpy as np

BASE_SEED = 171006189

# Direction table of Eq. (2): with row-major storage the second pixel of a pair
# lies +d, +d*(W-1), +d*W, +d*(W+1) elements after the first one for
# theta = 0, 45, 90, 135 degrees.  As (dx, dy) with y pointing down the rows
# these are (d,0), (-d,d), (0,d), (d,d).  Kept here as plain input data.
THETA_TABLE = {0: (1, 0), 45: (-1, 1), 90: (0, 1), 135: (1, 1)}


def offsets_for(distances, angles=(0, 45, 90, 135)):
    """Offsets (dx, dy) for every distance in ``distances`` times every angle."""
    out = []
    for d in distances:
        for a in angles:
            ux, uy = THETA_TABLE[a]
            out.append((ux * d, uy * d))
    return out


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _maxval(dtype) -> int:
    return int(np.iinfo(dtype).max)


def uniform(h: int, w: int, seed: int, dtype=np.uint8) -> np.ndarray:
    """i.i.d. uniform pixels over the whole range of ``dtype``."""
    return rng(seed).integers(0, _maxval(dtype) + 1, size=(h, w), dtype=dtype)


def gaussian_blur_periodic(z: np.ndarray, sigma: float) -> np.ndarray:
    """Blur with a Gaussian of std ``sigma`` pixels on a periodic grid.

    Multiplies the spectrum by exp(-2 pi^2 sigma^2 |f|^2), the Fourier transform
    of the unit-mass Gaussian.  Float32 FFTs keep 8192^2 fields cheap."""
    import scipy.fft as sf

    h, w = z.shape
    fy = np.fft.fftfreq(h).astype(np.float32)[:, None]
    fx = np.fft.rfftfreq(w).astype(np.float32)[None, :]
    gain = np.exp(np.float32(-2.0 * np.pi ** 2 * sigma * sigma) * (fx * fx + fy * fy))
    spec = sf.rfft2(z, workers=-1)
    spec *= gain
    return sf.irfft2(spec, s=(h, w), workers=-1)


def smooth(h: int, w: int, sigma: float, seed: int, dtype=np.uint8,
           noise_frac: float = 0.0) -> np.ndarray:
    """Blurred Gaussian noise, min-max rescaled to [0, max(dtype)].

    ``noise_frac`` > 0 adds i.i.d. normal noise of std ``noise_frac * max``
    after the rescale (then clip and round), as in the multispectral bands."""
    g = rng(seed)
    z = g.standard_normal((h, w), dtype=np.float32)
    b = gaussian_blur_periodic(z, sigma).astype(np.float64)
    top = float(_maxval(dtype))
    lo, hi = b.min(), b.max()
    b = (b - lo) * (top / (hi - lo)) if hi > lo else np.zeros_like(b)
    if noise_frac > 0:
        b += g.normal(0.0, noise_frac * top, size=(h, w))
    return np.clip(np.rint(b), 0, top).astype(dtype)


def constant(h: int, w: int, value: int, dtype=np.uint8) -> np.ndarray:
    return np.full((h, w), value, dtype=dtype)


def checkerboard(h: int, w: int, a: int, b: int, dtype=np.uint8) -> np.ndarray:
    """Pixel (x, y) is ``a`` where x + y is even, else ``b``."""
    yy, xx = np.indices((h, w))
    return np.where((xx + yy) % 2 == 0, a, b).astype(dtype)


def sha256(arr: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# Named workloads.  Each returns plain numpy inputs plus the call parameters.
# ---------------------------------------------------------------------------

def small_uniform_512():
    """512x512 uint8 i.i.d. uniform, N=8 over [0,255], one offset (1,0)."""
    img = uniform(512, 512, BASE_SEED + 0)
    return dict(name="512x512-u8-uniform-N8-K1", images=[img], N=8, lo=0, hi=255,
                offsets=[(1, 0)])


def square_4096(kind: str):
    """4096x4096 uint8, N=32 over [0,255], d=1 at the four angles.

    ``kind`` is ``uniform``, ``smooth`` (sigma = 8 px) or ``constant`` (128)."""
    s = BASE_SEED + 1
    if kind == "uniform":
        img = uniform(4096, 4096, s)
    elif kind == "smooth":
        img = smooth(4096, 4096, 8.0, s)
    elif kind == "constant":
        img = constant(4096, 4096, 128)
    else:
        raise ValueError(kind)
    return dict(name=f"4096x4096-u8-{kind}-N32-K4", images=[img], N=32, lo=0, hi=255,
                offsets=offsets_for([1]))


def multispectral_band(band: int, size: int = 8192):
    """One band of the 8-band uint16 stack: smooth field with sigma drawn
    uniformly in [2, 32] px, plus i.i.d. noise of std 5% of the range."""
    s = BASE_SEED + 2 + 1000 * band
    sigma = float(rng(s + 999).uniform(2.0, 32.0))
    return smooth(size, size, sigma, s, dtype=np.uint16, noise_frac=0.05), sigma


def multispectral(size: int = 8192, bands: int = 8):
    imgs = [multispectral_band(b, size)[0] for b in range(bands)]
    return dict(name=f"{bands}x{size}x{size}-u16-multispectral-N64-K12", images=imgs,
                N=64, lo=0, hi=65535, offsets=offsets_for([1, 2, 4]))


def batch_tiles(count: int = 4096, seed_offset: int = 3):
    """The batched workload: ``count`` uint8 tiles whose width and height are
    drawn independently as floor(exp(uniform(ln 32, ln 513))) (log-uniform in
    [32, 512]); the first half i.i.d. uniform, the second half smooth
    (sigma = 4 px); then the order is shuffled.  N = 16, d = 1 at the four
    angles."""
    g = rng(BASE_SEED + seed_offset)
    sides = np.floor(np.exp(g.uniform(np.log(32.0), np.log(513.0), size=(count, 2)))).astype(int)
    tiles = []
    for i in range(count):
        h, w = int(sides[i, 0]), int(sides[i, 1])
        s = BASE_SEED + seed_offset + 10 + i
        tiles.append(uniform(h, w, s) if i < count // 2 else smooth(h, w, 4.0, s))
    order = g.permutation(count)
    tiles = [tiles[i] for i in order]
    return dict(name=f"{count}-tiles-u8-32to512-N16-K4", images=tiles, N=16, lo=0, hi=255,
                offsets=offsets_for([1]))


def serving_pool(size: int = 8192):
    """The two pool images requests are cropped from: smooth (sigma = 8 px)
    and i.i.d. uniform noise, both uint8 size x size."""
    s = BASE_SEED + 4
    return {"smooth": smooth(size, size, 8.0, s), "noise": uniform(size, size, s + 1)}


def serving_requests(count: int = 1000, size: int = 8192, seed_offset: int = 5):
    """The serving workload's requests: a square crop with side uniform in
    [256, size] at a uniform position of the smooth or the noise pool image
    (probability 1/2 each), N drawn from {8, 16, 32, 64, 256}, the offsets a
    uniform non-empty subset (mask in [1, 4095]) of d in {1, 2, 4} at the four
    angles, statistics requested with probability 1/2."""
    g = rng(BASE_SEED + seed_offset)
    all12 = offsets_for([1, 2, 4])
    out = []
    for _ in range(count):
        side = int(g.integers(256, size + 1))
        kind = "smooth" if g.integers(0, 2) == 0 else "noise"
        y0 = int(g.integers(0, size - side + 1))
        x0 = int(g.integers(0, size - side + 1))
        N = int(g.choice([8, 16, 32, 64, 256]))
        mask = int(g.integers(1, 4096))
        offs = [all12[b] for b in range(12) if mask >> b & 1]
        out.append(dict(kind=kind, side=side, y0=y0, x0=x0, N=N, offsets=offs, features=bool(g.integers(0, 2))))
    return out


def glcm_like_counts(count: int = 16384, N: int = 16, seed_offset: int = 6):
    """Synthetic co-occurrence counts shaped like those of the batch tiles:
    ``count`` matrices of N x N uint32, entry (i, j) Poisson with mean
    T * exp(-(i - j)^2 / (2 s^2)) / Z, T (pairs of a tile) log-uniform in
    [3000, 260000], s (neighbour spread in levels) uniform in [0.3, 6]; one
    matrix in 64 is left empty."""
    g = rng(BASE_SEED + seed_offset)
    T = np.exp(g.uniform(np.log(3000.0), np.log(260000.0), size=count))
    s = g.uniform(0.3, 6.0, size=count)
    d = np.subtract.outer(np.arange(N), np.arange(N)).astype(np.float64)
    shape = np.exp(-(d[None] ** 2) / (2.0 * s[:, None, None] ** 2))
    lam = shape / shape.sum(axis=(1, 2), keepdims=True) * T[:, None, None]
    P = g.poisson(lam).astype(np.uint32)
    P[::64] = 0
    return dict(name=f"{count}-glcm-like-N{N}", counts=P)
