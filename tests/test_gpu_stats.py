"""GPU parity of the 1-D histogram and the GLCM variants against the oracle,
through the C ABI: histograms and symmetric matrices bit for bit, normalised
and averaged matrices equal to the oracle's fp64 value rounded to fp32, and
Haralick's thirteen statistics (fp64 on the device, stored as fp32) within
1e-5 relative of the oracle, plus 1e-6 absolute on f3, f12 and f13 (cancellations near zero)."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_1710_06189_amd")

RNG = np.random.default_rng(20171006)
ALL12 = [(d * a, d * b) for d in (1, 2, 4) for a, b in ((1, 0), (-1, 1), (0, 1), (1, 1))]


def host(t):
    torch.cuda.synchronize()
    if t.dtype == torch.float32:
        return t.cpu().numpy()
    return t.view(torch.int32).cpu().numpy().view(np.uint32)


def dev(a):
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda().view(torch.uint32)
    return torch.from_numpy(a).cuda()


# ---------------------------------------------------------------- histogram

HIST_CASES = [
    # (H, W, dtype, N, lo, hi)
    (1, 1, np.uint8, 8, 0, 255),
    (37, 53, np.uint8, 32, 0, 255),        # shift quantizer, ragged chunks
    (29, 1000, np.uint8, 5, 17, 200),      # magic-number quantizer
    (3, 4099, np.uint8, 256, 0, 255),
    (1, 70001, np.uint8, 16, 0, 255),      # one long row
    (2049, 3, np.uint8, 7, 0, 255),        # many short rows
    (61, 77, np.uint16, 64, 0, 65535),
    (40, 515, np.uint16, 1000, 0, 65535),  # levels beyond a byte
    (33, 65, np.uint16, 4096, 1000, 60000),
    (50, 50, np.uint8, 4096, 0, 255),      # more levels than values
    (8, 8, np.uint8, 1, 0, 255),
]


@pytest.mark.parametrize("H,W,dt,N,lo,hi", HIST_CASES)
def test_histogram_matches_oracle(H, W, dt, N, lo, hi):
    top = 256 if dt == np.uint8 else 65536
    img = RNG.integers(0, top, size=(H, W), dtype=dt)
    print(f"[hist] {H}x{W} {np.dtype(dt).name} N={N}", flush=True)
    got = host(G.glcm_histogram(dev(img), N, lo, hi))
    assert np.array_equal(got, oracle.histogram(img, N, lo, hi))


@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
@pytest.mark.parametrize("pitch", [301, 320])
def test_histogram_views(dt, pitch):
    """Views with odd pitches and offsets take the per-pixel loads; a 16-byte
    pitch with a 16-byte aligned offset keeps the chunk loads."""
    hi = 255 if dt == np.uint8 else 65535
    base = RNG.integers(0, hi + 1, size=(90, pitch), dtype=dt)
    t = dev(base)
    for (y0, x0, h, w) in [(0, 1, 90, 299), (3, 5, 80, 17), (1, 0, 89, 300), (7, 13, 1, 250), (2, 16, 70, 280)]:
        view = t[y0:y0 + h, x0:x0 + w]
        got = host(G.glcm_histogram(view, 24, 0, hi))
        assert np.array_equal(got, oracle.histogram(base[y0:y0 + h, x0:x0 + w], 24, 0, hi))


@pytest.mark.parametrize("N", [32, 256])
def test_histogram_full_size(N):
    img = synth.smooth(4096, 4096, 8.0, 171006190)
    print(f"[hist] 4096x4096 smooth N={N}", flush=True)
    got = host(G.glcm_histogram(dev(img), N, 0, 255))
    assert np.array_equal(got, oracle.histogram(img, N, 0, 255))
    assert int(got.sum()) == 4096 * 4096


def test_histogram_equals_glcm_marginals():
    img = synth.smooth(500, 700, 4.0, 3)
    t = dev(img)
    P = host(G.glcm_compute(t, 32, 0, 255, [(1, 0), (0, 1)]))
    assert np.array_equal(P[0].sum(axis=1), host(G.glcm_histogram(t[:, :-1].contiguous(), 32, 0, 255)))
    assert np.array_equal(P[1].sum(axis=0), host(G.glcm_histogram(t[1:], 32, 0, 255)))


def test_histogram_with_plan_and_errors():
    img = RNG.integers(0, 256, size=(100, 130), dtype=np.uint8)
    plan = G.glcm_plan_create(np.uint8, 16, [(1, 0)], 64, 64)
    try:
        got = host(G.glcm_histogram(dev(img), 16, 0, 255, plan=plan))  # the plan's size limits do not apply
        assert np.array_equal(got, oracle.histogram(img, 16, 0, 255))
        with pytest.raises(G.GlcmError):
            G.glcm_histogram(dev(img), 8, 0, 255, plan=plan)  # N differs from the plan's
    finally:
        plan.close()
    with pytest.raises(ValueError):
        G.glcm_histogram(torch.from_numpy(img), 16)  # host tensor
    lib = G._lib()
    import ctypes
    out = torch.empty(16, dtype=torch.uint32, device="cuda")
    rc = lib.glcm_histogram(None, ctypes.c_void_p(img.ctypes.data), 130, 100, 130, 0, 16, 0, 255,
                            ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -3  # host image: not served


# ---------------------------------------------------------------- variants

def image_glcms(N, K=4, size=(300, 400), seed=0, kind="smooth"):
    img = synth.smooth(*size, 4.0, seed) if kind == "smooth" else synth.uniform(*size, seed)
    return oracle.glcm(img, N, 0, 255, ALL12[:K])


def random_counts(K, N, high, density=0.6):
    P = RNG.integers(0, high, size=(K, N, N), dtype=np.uint64).astype(np.uint32)
    P[RNG.random((K, N, N)) > density] = 0
    return P


VARIANT_INPUTS = [
    ("image N=8", lambda: image_glcms(8)),
    ("image N=33 noise", lambda: image_glcms(33, kind="uniform", seed=4)),
    ("image N=256", lambda: image_glcms(256, K=2, size=(500, 500), seed=2)),
    ("random N=7", lambda: random_counts(50, 7, 1000)),
    ("random N=16 batch", lambda: random_counts(4096, 16, 2 ** 16)),
    ("random large counts", lambda: random_counts(6, 9, 2 ** 32)),
    ("single level", lambda: np.full((3, 1, 1), 5, dtype=np.uint32)),
]


@pytest.mark.parametrize("name,make", VARIANT_INPUTS, ids=[v[0] for v in VARIANT_INPUTS])
def test_symmetrize_normalize(name, make):
    P = make()
    P[0] = 0  # an empty matrix
    t = dev(P)
    assert np.array_equal(host(G.glcm_symmetrize(t)), oracle.symmetric(P))
    assert np.array_equal(host(G.glcm_normalize(t)), oracle.normalize(P).astype(np.float32))
    inplace = t.clone()
    G.glcm_symmetrize(inplace, out=inplace)
    assert np.array_equal(host(inplace), oracle.symmetric(P))


@pytest.mark.parametrize("m", [1, 2, 4, 12])
def test_average(m):
    P = np.concatenate([image_glcms(16, K=12, seed=5), random_counts(12, 16, 5000)])
    P[3] = 0
    got = host(G.glcm_average(dev(P), m))
    assert np.array_equal(got, oracle.average(P, m).astype(np.float32))


# Statistics that are a cancellation near zero for nearly independent
# matrices and so need an absolute term besides the relative one: f3, the
# correlation (a covariance over a product of deviations); f12, a difference
# of two entropies over a third; f13, the square root of 1 - exp(-2 (HXY2 -
# HXY)), which turns a rounding-level difference of entropies into its
# square root.  Every other statistic is held to 1e-5 relative alone (exact
# zeros must come out as zeros).
NEAR_ZERO_STATS = [2, 11, 12]


def assert_stats_close(got, want):
    tol = 1e-5 * np.abs(want)
    tol[..., NEAR_ZERO_STATS] += 1e-6
    bad = np.abs(got.astype(np.float64) - want) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], got[bad][:5], want[bad][:5])


@pytest.mark.parametrize("name,make", VARIANT_INPUTS, ids=[v[0] for v in VARIANT_INPUTS])
def test_haralick(name, make):
    P = make()
    P[0] = 0
    got = host(G.glcm_haralick(dev(P)))
    assert got.shape == (P.shape[0], 13)
    assert_stats_close(got, oracle.haralick(P))
    assert not got[0].any()


def test_haralick_special_matrices():
    N = 24
    mats = np.zeros((5, N, N), dtype=np.uint32)
    mats[0, 3, 17] = 99                      # single bin off the diagonal
    mats[1] = 7                              # uniform
    mats[2][np.arange(N), np.arange(N)] = 3  # uniform diagonal
    mats[3] = np.outer(RNG.integers(1, 40, N), RNG.integers(1, 40, N)).astype(np.uint32)  # independent
    mats[4, :, 5] = RNG.integers(1, 100, N)  # column marginal on one level
    got = host(G.glcm_haralick(dev(mats)))
    assert_stats_close(got, oracle.haralick(mats))
    assert got[4, 2] == 1.0


def test_haralick_largest_levels_and_limit():
    P = random_counts(2, 1024, 50, density=0.01)
    assert_stats_close(host(G.glcm_haralick(dev(P))), oracle.haralick(P))
    with pytest.raises(G.GlcmError) as e:
        G.glcm_haralick(torch.zeros((1, 1025, 1025), dtype=torch.uint32, device="cuda"))
    assert e.value.status == -3


def test_variants_compose_with_compute():
    """The direction-averaged, symmetric statistics of an image: counts from
    glcm_compute, then the post-processing calls, all on the device."""
    img = synth.smooth(600, 800, 6.0, 8)
    t = dev(img)
    P = G.glcm_compute(t, 32, 0, 255, ALL12)
    Pc = oracle.glcm(img, 32, 0, 255, ALL12)
    S = G.glcm_symmetrize(P)
    assert np.array_equal(host(G.glcm_average(S, 4)), oracle.average(oracle.symmetric(Pc), 4).astype(np.float32))
    assert_stats_close(host(G.glcm_haralick(S)), oracle.haralick(oracle.symmetric(Pc)))


def test_post_processing_graph_replays():
    """The four post-processing calls only queue kernels, so they are captured
    in a graph and replayed; the input is rewritten in place between replays
    (eager work, synchronised) and every replay is checked against the oracle."""
    P = random_counts(64, 16, 3000)
    P[5] = 0
    t = dev(P)
    sym = torch.empty_like(t)
    nrm = torch.empty((64, 16, 16), dtype=torch.float32, device="cuda")
    avg = torch.empty((16, 16, 16), dtype=torch.float32, device="cuda")
    har = torch.empty((64, 13), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()

    def run(stream):
        G.glcm_symmetrize(t, out=sym, stream=stream)
        G.glcm_normalize(t, out=nrm, stream=stream)
        G.glcm_average(t, 4, out=avg, stream=stream)
        G.glcm_haralick(sym, out=har, stream=stream)

    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(side)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        run(side)
    torch.cuda.synchronize()
    for rep in range(4):
        new = random_counts(64, 16, 3000 + 500 * rep)
        new[(rep * 7) % 64] = 0
        t.copy_(dev(new))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        S = oracle.symmetric(new)
        assert np.array_equal(host(sym), S), f"replay {rep}: symmetric matrices"
        assert np.array_equal(host(nrm), oracle.normalize(new).astype(np.float32)), f"replay {rep}: normalised"
        assert np.array_equal(host(avg), oracle.average(new, 4).astype(np.float32)), f"replay {rep}: averaged"
        assert_stats_close(host(har), oracle.haralick(S))


def test_histogram_on_streams_with_one_plan():
    """Histograms of different images on two streams through one plan are
    ordered after each other (the plan's partials are shared) and all match."""
    imgs = [RNG.integers(0, 256, size=(700, 900), dtype=np.uint8) for _ in range(6)]
    ts = [dev(im) for im in imgs]
    plan = G.glcm_plan_create(np.uint8, 64, [(0, 0)], 1024, 1024)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()  # the uploads are done before the side streams read the images
    try:
        outs = [G.glcm_histogram(t, 64, 0, 255, plan=plan, stream=streams[i % 2]) for i, t in enumerate(ts)]
        torch.cuda.synchronize()
        for o, im in zip(outs, imgs):
            assert np.array_equal(host(o), oracle.histogram(im, 64, 0, 255))
    finally:
        plan.close()


MCC_INPUTS = [v for v in VARIANT_INPUTS if v[0] in ("image N=8", "image N=33 noise", "random N=7",
                                                       "random N=16 batch", "single level")] + [
    ("diag and blocks", lambda: np.stack([np.diag(np.full(12, 5)).astype(np.uint32),
                                          np.kron(np.eye(3, dtype=np.uint32), np.full((4, 4), 2, dtype=np.uint32))])),
    ("two by two", lambda: np.array([[[3, 1], [1, 3]], [[0, 7], [7, 0]], [[5, 5], [5, 5]]], dtype=np.uint32)),
    ("N=64 sparse", lambda: random_counts(3, 64, 40, density=0.05)),
]


@pytest.mark.parametrize("name,make", MCC_INPUTS, ids=[v[0] for v in MCC_INPUTS])
def test_haralick_mcc(name, make):
    """f14 against the oracle (numpy's eigenvalues of Q): within 1e-5 rel +
    1e-6 abs (near 0 both sides are the square root of an eigenvalue at
    rounding level, about 1e-8, which the absolute term covers)."""
    P = make()
    if P.shape[0] > 1:
        P[0] = 0
    got = host(G.glcm_haralick_mcc(dev(P))).astype(np.float64)
    want = oracle.haralick_mcc(P)
    bad = np.abs(got - want) > 1e-5 * np.abs(want) + 1e-6
    assert not bad.any(), (np.argwhere(bad)[:5], got[bad][:5], want[bad][:5])
    if P.shape[0] > 1:
        assert got[0] == 0.0
    with pytest.raises(G.GlcmError) as e:
        G.glcm_haralick_mcc(torch.zeros((1, 65, 65), dtype=torch.uint32, device="cuda"))
    assert e.value.status == -3


def test_post_processing_rejects_overlaps_and_bad_groups():
    """Argument errors with real device buffers: partial overlaps, K not a
    multiple of m, m beyond 64 (nothing is queued; the status is EINVAL)."""
    import ctypes
    lib = G._lib()
    buf = torch.zeros(3 * 8 * 8 + 64, dtype=torch.int32, device="cuda")
    p = buf.data_ptr()
    vp = ctypes.c_void_p
    # symmetric output shifted by one word into the input: rejected; exactly in place: accepted
    assert lib.glcm_symmetrize(vp(p), 3, 8, vp(p + 4), None) == -1
    assert lib.glcm_symmetrize(vp(p), 3, 8, vp(p), None) == 0
    assert lib.glcm_normalize(vp(p), 3, 8, vp(p + 64), None) == -1
    assert lib.glcm_haralick(vp(p), 3, 8, vp(p + 8), None) == -1
    assert lib.glcm_haralick_mcc(vp(p), 3, 8, vp(p + 8), None) == -1
    other = torch.zeros(1024, dtype=torch.float32, device="cuda")
    assert lib.glcm_average(vp(p), 3, 8, 2, vp(other.data_ptr()), None) == -1   # K % m != 0
    assert lib.glcm_average(vp(p), 130, 8, 65, vp(other.data_ptr()), None) == -1  # m > 64
    torch.cuda.synchronize()


def test_histogram_u16_largest_levels_full_size():
    img = synth.smooth(2048, 2048, 6.0, 4242, dtype=np.uint16)
    print("[hist] 2048x2048 u16 N=4096", flush=True)
    got = host(G.glcm_histogram(dev(img), 4096, 0, 65535))
    assert np.array_equal(got, oracle.histogram(img, 4096, 0, 65535))
