"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Covers the workloads the library is measured on (512^2 uint8 N=8; 4096^2 uint8
N=32 with four d=1 offsets on uniform, smooth and constant images; uint16
multispectral bands, N=64, twelve offsets), every kernel variant forced through
plans, replica / workgroup / band sweeps, ragged and degenerate shapes, strided
and misaligned views, exhaustive quantizer inputs and large N.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_1710_06189_amd")


def to_device(img: np.ndarray) -> torch.Tensor:
    if img.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(img).view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def to_host(out: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return out.view(torch.int32).cpu().numpy().view(np.uint32)


def gpu_glcm(img, N, lo, hi, offs, plan=None, t=None):
    if t is None:
        t = to_device(img)
    out = torch.empty((len(offs), N, N), dtype=torch.uint32, device="cuda")
    return to_host(G.glcm_compute(t, N, lo, hi, offs, plan=plan, out=out))


def check(img, N, lo, hi, offs, plan=None, t=None, label=""):
    print(f"[parity] {label} shape={img.shape} dtype={img.dtype} N={N} lo={lo} hi={hi} K={len(offs)}", flush=True)
    got = gpu_glcm(img, N, lo, hi, offs, plan=plan, t=t)
    want = oracle.glcm(img, N, lo, hi, offs)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        k, i, j = bad[0]
        raise AssertionError(f"{label}: {len(bad)} bins differ, first at k={k} i={i} j={j}: "
                             f"gpu {got[k, i, j]} oracle {want[k, i, j]}")
    return got


def test_status_word_clear_after_suite_start():
    t = to_device(synth.uniform(64, 64, 1))
    check(synth.uniform(64, 64, 1), 8, 0, 255, [(1, 0)], t=t, label="warmup")


def test_small_uniform_512():
    w = synth.small_uniform_512()
    check(w["images"][0], w["N"], w["lo"], w["hi"], w["offsets"], label=w["name"])


@pytest.mark.parametrize("kind", ["uniform", "smooth", "constant"])
def test_square_4096(kind):
    w = synth.square_4096(kind)
    got = check(w["images"][0], w["N"], w["lo"], w["hi"], w["offsets"], label=w["name"])
    if kind == "constant":
        assert [int(got[k, 16, 16]) for k in range(4)] == [16773120, 16769025, 16773120, 16769025]


SHAPES = [(1, 1), (1, 37), (37, 1), (15, 16), (16, 15), (17, 33), (64, 63), (65, 129), (1023, 3), (3, 1025),
          (1040, 77), (2000, 31), (4097, 5)]


@pytest.mark.parametrize("W,H", SHAPES)
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_ragged_shapes(W, H, dtype):
    img = synth.smooth(H, W, 2.0, 100 + W + H, dtype) if W > 2 and H > 2 else synth.uniform(H, W, 3, dtype)
    offs = synth.offsets_for([1, 2, 4]) + [(0, 0), (-3, -1), (4, -4)]
    top = int(np.iinfo(dtype).max)
    check(img, 16, 0, top, offs, label=f"ragged {W}x{H}")


@pytest.mark.parametrize("offs", [
    [(5, 0)], [(0, 9)], [(-7, 3)], [(16, 16), (-16, 1)], [(100, 0), (0, 100), (-100, -100)],
    [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)],
])
def test_offsets_any(offs):
    img = synth.smooth(130, 300, 3.0, 7)
    check(img, 24, 10, 240, offs, label=f"offsets {offs}")


@pytest.mark.parametrize("flags,name", [
    (G.FLAG_FORCE_GENERIC, "generic"), (G.FLAG_FORCE_PARTITIONED, "partitioned"),
    (G.FLAG_FORCE_GLOBAL, "global"), (G.FLAG_FORCE_SLABS, "slabs"), (G.FLAG_FORCE_L2, "l2"), (0, "auto"),
])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("merge", [0, 1])
def test_forced_paths(flags, name, dtype, merge):
    img = synth.smooth(517, 731, 5.0, 11, dtype)
    offs = synth.offsets_for([1, 2, 4])
    top = int(np.iinfo(dtype).max)
    plan = G.glcm_plan_create(dtype, 32, offs, 731, 517, flags)
    try:
        if plan.tuning.path != 3:
            plan.set_tuning(merge=merge)
        check(img, 32, 0, top, offs, plan=plan, label=f"path {name} {plan.tuning.as_dict()}")
        check(img, 32, 0, top, offs, plan=plan, label=f"path {name} again")
    finally:
        plan.close()


@pytest.mark.parametrize("N,dtype,shape,offs", [
    (256, np.uint8, (700, 900), synth.offsets_for([1, 2, 4])),
    (256, np.uint8, (1, 1), [(1, 0)]),
    (512, np.uint16, (333, 1001), [(1, 0), (0, -3), (-5, 5)]),
    (1024, np.uint16, (257, 129), [(0, 0), (7, 7)]),
    (128, np.uint8, (64, 2100), synth.offsets_for([1]) + [(-64, 0), (2100, 0)]),
])
def test_l2_slice_path(N, dtype, shape, offs):
    """Pairs added straight into the per-XCD slices (large N), on aligned and
    misaligned views, twice on one plan (the slices are clean again after each
    call)."""
    H, W = shape
    top = int(np.iinfo(dtype).max)
    img = synth.smooth(H + 3, W + 5, 4.0, 31 + N, dtype) if H > 2 and W > 2 else synth.uniform(H + 3, W + 5, 3, dtype)
    plan = G.glcm_plan_create(dtype, N, offs, W + 5, H + 3, G.FLAG_FORCE_L2)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == "l2"
        t = to_device(img)
        for y0, x0 in ((0, 0), (3, 5), (1, 2)):
            view, sub = t[y0:y0 + H, x0:x0 + W], img[y0:y0 + H, x0:x0 + W]
            check(sub, N, 0, top, offs, plan=plan, t=view, label=f"l2 N={N} at ({y0},{x0})")
    finally:
        plan.close()


SLAB_LAYOUTS = [(1, 32), (2, 32), (4, 32), (8, 32), (16, 32), (2, 16), (4, 16), (8, 16), (16, 16), (32, 16)]
STRIP_LAYOUTS = [(4, 32), (8, 32), (16, 32), (32, 32), (4, 16), (8, 16), (16, 16), (32, 16)]


@pytest.mark.parametrize("kernel,R,bits", [("slabs", R, b) for R, b in SLAB_LAYOUTS] +
                         [("strips", R, b) for R, b in STRIP_LAYOUTS])
@pytest.mark.parametrize("wg", [256, 1024])
def test_replica_counter_and_workgroup_sweep(kernel, R, bits, wg):
    img = synth.smooth(300, 2100, 8.0, 12)
    offs = synth.offsets_for([1])
    plan = G.glcm_plan_create(np.uint8, 32, offs, 2100, 300, G.FLAG_FORCE_SLABS if kernel == "slabs" else 0)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == kernel
        t = plan.set_tuning(replicas=R, wg_size=wg, counter_bits=bits)
        assert t.replicas == R and t.wg_size == wg and t.counter_bits == bits
        check(img, 32, 0, 255, offs, plan=plan, label=f"{kernel} R={R} bits={bits} wg={wg} P={t.partitions}")
    finally:
        plan.close()


@pytest.mark.parametrize("K", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("R", [4, 16, 32])
def test_strip_pairs_any_offset_count(K, R):
    """16-bit pair layout with an odd number of GLCMs per partition and with
    several partitions; offsets include negated ones (stored transposed)."""
    pool = [(1, 0), (-1, -1), (0, 1), (1, 1), (-1, 1), (0, -1), (-1, 0)]
    offs = pool[:K]
    img = synth.smooth(203, 1100, 3.0, 70 + K)
    plan = G.glcm_plan_create(np.uint8, 32, offs, 1100, 203)
    try:
        t = plan.set_tuning(replicas=R, counter_bits=16)
        assert G.PATH_NAMES[t.path] == "strips"
        check(img, 32, 0, 255, offs, plan=plan, label=f"pairs K={K} R={R} P={t.partitions}")
    finally:
        plan.close()


def test_strip_layout_rejects_unsupported_copies():
    plan = G.glcm_plan_create(np.uint8, 32, [(1, 0)], 256, 256)
    try:
        for R, bits in [(1, 32), (2, 32), (64, 32), (2, 16), (64, 16)]:
            with pytest.raises(G.GlcmError):
                plan.set_tuning(replicas=R, counter_bits=bits)
    finally:
        plan.close()


def test_sixteen_bit_counters_near_the_bound():
    """A constant image puts every vote of a copy into one bin: the largest
    band the 16-bit slab counters accept, and one just beyond (falls back to 32)."""
    for H in (4096, 8192):  # 16 and 32 slabs of 2048 same-bin votes per copy: 32768, then 65536
        img = synth.constant(H, 4096, 77)
        offs = synth.offsets_for([1])
        plan = G.glcm_plan_create(np.uint8, 16, offs, 4096, H, G.FLAG_FORCE_SLABS)
        try:
            plan.set_tuning(replicas=2, counter_bits=16)
            check(img, 16, 0, 255, offs, plan=plan, label=f"c16 bound H={H}")
        finally:
            plan.close()


@pytest.mark.parametrize("W,H", [(4096, 4096), (16, 8192), (1024, 65535)])
def test_sixteen_bit_strip_counters_constant_image(W, H):
    """Every vote of a 16-bit strip counter in one bin, on the tallest bands
    (two GLCMs share each dword, so a wrap would also corrupt the other)."""
    img = synth.constant(H, W, 200)
    offs = synth.offsets_for([1])
    plan = G.glcm_plan_create(np.uint8, 16, offs, W, H)
    try:
        plan.set_tuning(replicas=8, counter_bits=16)
        check(img, 16, 0, 255, offs, plan=plan, label=f"strips c16 constant {W}x{H}")
    finally:
        plan.close()


@pytest.mark.parametrize("kernel,dists", [("slabs", [1, 2, 4]), ("strips", [1, 2]), ("strips", [1])])
@pytest.mark.parametrize("H", [1, 2, 3, 4, 5, 7, 9, 255, 257, 1029])
def test_band_heights(kernel, dists, H):
    """Heights that leave partial slabs, strips and bands in the row kernels."""
    img = synth.uniform(H, 1500, 13 + H)
    offs = synth.offsets_for(dists)
    plan = G.glcm_plan_create(np.uint8, 8, offs, 1500, H)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == kernel
        check(img, 8, 0, 255, offs, plan=plan, label=f"{kernel} d={dists} H={H}")
    finally:
        plan.close()


def force_strips(plan, R, bits, wg=512):
    """Moves a slab plan onto the strip kernel with R dwords per bin; None
    when that layout does not fit the LDS."""
    try:
        return plan.set_tuning(path=4, replicas=R, counter_bits=bits, wg_size=wg)
    except G.GlcmError:
        return None


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("N,dists", [(16, [3]), (32, [4]), (8, [1, 2, 4]), (16, [3, 4])])
@pytest.mark.parametrize("kind", ["smooth", "uniform"])
def test_strips_reach_four(dtype, N, dists, kind):
    """Offsets of reach 3 and 4 along the four directions, negated ones
    included, on the strip kernel's five-row ring (forced over the slab
    kernel): several layouts and workgroup sizes, a ragged image of several
    bands and strips, and a misaligned view of it read in place."""
    W, H = 1037, 301
    top = int(np.iinfo(dtype).max)
    img = synth.smooth(H, W, 3.0, 140 + N, dtype) if kind == "smooth" else synth.uniform(H, W, 141 + N, dtype)
    t = to_device(img)
    d = dists[-1]
    offs = synth.offsets_for(dists) + [(-d, 0), (d, -d), (0, 0)]
    plan = G.glcm_plan_create(dtype, N, offs, W, H)
    try:
        ran = 0
        for R, bits, wg in [(32, 16, 512), (16, 32, 256), (8, 16, 512), (4, 32, 1024)]:
            tu = force_strips(plan, R, bits, wg)
            if tu is None:
                continue
            assert G.PATH_NAMES[tu.path] == "strips" and tu.rows_per_wave == 0
            check(img, N, 0, top, offs, plan=plan, t=t, label=f"strips reach {d} R={R} bits={bits} wg={wg} {kind}")
            sub = img[2:, 3:3 + 1001]
            check(sub, N, 0, top, offs, plan=plan, t=t[2:, 3:3 + 1001], label=f"strips reach {d} R={R} in place")
            ran += 1
        assert ran >= 2
        back = plan.set_tuning(path=1, replicas=4, counter_bits=32, wg_size=1024)
        assert G.PATH_NAMES[back.path] == "slabs" and back.rows_per_wave == 4
        check(img, N, 0, top, offs, plan=plan, t=t, label=f"back on slabs reach {d}")
    finally:
        plan.close()


@pytest.mark.parametrize("H", [1, 2, 3, 4, 5, 6, 7, 9, 11, 255, 257, 1029])
def test_strips_reach_four_band_heights(H):
    """Heights that end a strip inside the five-row ring."""
    img = synth.uniform(H, 1500, 23 + H)
    offs = synth.offsets_for([1, 4])
    plan = G.glcm_plan_create(np.uint8, 8, offs, 1500, H)
    try:
        assert force_strips(plan, 32, 16) is not None
        check(img, 8, 0, 255, offs, plan=plan, label=f"strips reach 4 H={H}")
    finally:
        plan.close()


def test_strip_reach_rules():
    """Reach 3 and 4 stay on the slab kernel off the four directions; the
    strip kernel refuses them, and a plan off the row kernels keeps its path."""
    img = synth.smooth(200, 700, 3.0, 150)
    offs = [(1, 3), (2, 0)]
    plan = G.glcm_plan_create(np.uint8, 16, offs, 700, 200)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == "slabs"
        with pytest.raises(G.GlcmError):
            plan.set_tuning(path=4, replicas=32, counter_bits=16, wg_size=512)
        assert G.PATH_NAMES[plan.tuning.path] == "slabs"
        check(img, 16, 0, 255, offs, plan=plan, label="reach 3 off the directions")
    finally:
        plan.close()
    plan = G.glcm_plan_create(np.uint8, 300, [(4, 4)], 700, 200)
    try:
        before = plan.tuning.path
        assert G.PATH_NAMES[before] not in ("strips", "slabs")
        assert plan.set_tuning(path=4).path == before
    finally:
        plan.close()


@pytest.mark.parametrize("kind", ["smooth", "uniform"])
def test_autotune_reach_four(kind):
    """The autotuner times strip layouts of reach 4 beside the slabs and keeps
    one; the counts stay exact."""
    W, H = 2048, 512
    img = synth.smooth(H, W, 6.0, 155) if kind == "smooth" else synth.uniform(H, W, 156)
    offs = synth.offsets_for([4])
    t = to_device(img)
    plan = G.glcm_plan_create(np.uint8, 16, offs, W, H)
    try:
        chosen = plan.autotune(t, 0, 255, repeats=2)
        name = G.PATH_NAMES[chosen.path]
        print(f"[autotune] reach 4 {kind}: {chosen.as_dict()}", flush=True)
        assert name in ("strips", "slabs")
        check(img, 16, 0, 255, offs, plan=plan, t=t, label=f"autotuned reach 4 {name} {kind}")
    finally:
        plan.close()


@pytest.mark.parametrize("W", [1, 15, 16, 17, 1023, 1024, 1025, 2047, 3000])
@pytest.mark.parametrize("dists", [[1], [2], [1, 2]])
def test_strip_widths(W, dists):
    """Widths around the 16-pixel chunk and 1024-pixel strip boundaries."""
    img = synth.smooth(70, W, 3.0, 40 + W) if W > 2 else synth.uniform(70, W, 41)
    offs = synth.offsets_for(dists) + [(0, 0), (-dists[-1], 0), (dists[-1], -dists[-1])]
    check(img, 32, 0, 255, offs, label=f"strip widths W={W} d={dists}")


@pytest.mark.parametrize("W", [8, 24, 40, 1032, 2056])
def test_strip_u16_pitch_of_8_pixels(W):
    """uint16 rows whose pitch is a multiple of 8 but not 16 pixels: aligned
    for the strip kernel, with the last chunk ending inside the last row."""
    img = synth.smooth(37, W, 2.5, 60 + W, np.uint16)
    offs = synth.offsets_for([1, 2])
    plan = G.glcm_plan_create(np.uint16, 16, offs, W, 37)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == "strips"
        check(img, 16, 0, 65535, offs, plan=plan, label=f"u16 pitch W={W}")
    finally:
        plan.close()


def test_rows_per_wave_knob():
    plan = G.glcm_plan_create(np.uint8, 8, [(1, 0)], 64, 64, G.FLAG_FORCE_SLABS)
    try:
        assert plan.set_tuning(rows_per_wave=4).rows_per_wave == 4
        with pytest.raises(G.GlcmError):
            plan.set_tuning(rows_per_wave=3)
    finally:
        plan.close()
    plan = G.glcm_plan_create(np.uint8, 8, [(1, 0)], 64, 64)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == "strips" and plan.tuning.rows_per_wave == 0
        with pytest.raises(G.GlcmError):
            plan.set_tuning(rows_per_wave=4)
    finally:
        plan.close()


def test_strided_and_misaligned_views():
    base = synth.smooth(400, 700, 4.0, 14)
    tb = to_device(base)
    offs = synth.offsets_for([1, 4])
    for (y0, y1, x0, x1) in [(0, 400, 0, 640), (3, 397, 1, 699), (10, 300, 16, 656), (0, 399, 5, 6)]:
        view = tb[y0:y1, x0:x1]
        check(base[y0:y1, x0:x1], 32, 0, 255, offs, t=view, label=f"view {(y0, y1, x0, x1)}")


@pytest.mark.parametrize("N,lo,hi", [(8, 0, 255), (7, 13, 200), (256, 0, 255), (1, 0, 255), (100, 50, 60),
                                     (3, 255, 255), (32, 0, 127)])
def test_quantizer_exhaustive_u8(N, lo, hi):
    """Every 8-bit value occurs; offset (0,0) puts the level histogram on the diagonal."""
    img = np.arange(256, dtype=np.uint8).reshape(16, 16)
    img = np.concatenate([img, img[::-1, ::-1]], axis=0)
    check(img, N, lo, hi, [(0, 0), (1, 0), (0, 1)], label=f"quant u8 N={N}")


@pytest.mark.parametrize("N,lo,hi", [(64, 0, 65535), (257, 1000, 60000), (13, 0, 65535), (4096, 0, 65535),
                                     (4096, 7, 700), (300, 0, 299)])
def test_quantizer_exhaustive_u16(N, lo, hi):
    img = np.arange(65536, dtype=np.uint16).reshape(256, 256)
    want = oracle.glcm(img, N, lo, hi, [(0, 0)])
    got = gpu_glcm(img, N, lo, hi, [(0, 0)])
    assert np.array_equal(got, want), f"quant u16 N={N} lo={lo} hi={hi}"


@pytest.mark.parametrize("N", [256, 300, 1024])
def test_large_levels(N):
    img = synth.uniform(300, 257, 15, np.uint16)
    check(img, N, 0, 65535, [(1, 0), (-1, 1)], label=f"large N={N}")


def test_multispectral_band_reduced():
    img, sigma = synth.multispectral_band(0, size=1536)
    check(img, 64, 0, 65535, synth.offsets_for([1, 2, 4]), label=f"multispectral 1536^2 sigma={sigma:.1f}")


def test_multispectral_band_full():
    img, sigma = synth.multispectral_band(3)
    check(img, 64, 0, 65535, synth.offsets_for([1, 2, 4]), label=f"multispectral 8192^2 sigma={sigma:.1f}")


def test_repeated_calls_two_streams():
    img = synth.smooth(512, 1024, 6.0, 16)
    offs = synth.offsets_for([1])
    want = oracle.glcm(img, 32, 0, 255, offs)
    t = to_device(img)
    plan = G.glcm_plan_create(np.uint8, 32, offs, 1024, 512)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    try:
        for it in range(40):
            s = s1 if it % 3 else s2
            with torch.cuda.stream(s):
                outs.append(G.glcm_compute(t, 32, 0, 255, offs, plan=plan, stream=s))
        torch.cuda.synchronize()
        for o in outs:
            assert np.array_equal(to_host(o), want)
    finally:
        plan.close()


def test_offsets_outside_image_give_zero():
    img = synth.uniform(20, 30, 17)
    got = gpu_glcm(img, 8, 0, 255, [(30, 0), (0, 20), (-31, 5)])
    assert not got.any()


@pytest.mark.parametrize("case", ["smooth", "uniform", "constant", "checker", "sparse"])
def test_features_vs_oracle(case):
    N = 16
    if case == "smooth":
        img = synth.smooth(600, 500, 4.0, 18)
    elif case == "uniform":
        img = synth.uniform(600, 500, 18)
    elif case == "constant":
        img = synth.constant(60, 50, 99)
    elif case == "checker":
        img = synth.checkerboard(60, 51, 16, 240)
    else:
        img = synth.constant(64, 64, 0)
        img[10, 10] = 255
    offs = synth.offsets_for([1, 2])
    P = G.glcm_compute(to_device(img), N, 0, 255, offs)
    f = G.glcm_features(P)
    torch.cuda.synchronize()
    got = f.cpu().numpy().astype(np.float64)
    want = oracle.features(oracle.glcm(img, N, 0, 255, offs))
    zero = want == 0
    assert np.all(got[zero] == 0), (got, want)
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    assert np.all(rel[~zero] <= 1e-5), (case, got, want, rel)


def test_features_large_and_empty():
    rng = synth.rng(19)
    P = rng.integers(0, 1 << 15, size=(4, 256, 256)).astype(np.uint32)  # totals below 2^31
    P[1] = 0
    P[2, :, :] = 0
    P[2, 5, 7] = 0xFFFFFFFF
    t = torch.from_numpy(P.view(np.int32)).cuda()
    got = G.glcm_features(t).cpu().numpy().astype(np.float64)
    want = oracle.features(P)
    assert np.all(got[1] == 0)
    P[3, 0, 0] = 1 << 31                      # total above 2^32 - 1: documented NaN output
    P[3, 1, 1] = 1 << 31
    t3 = torch.from_numpy(P[3:].view(np.int32)).cuda()
    assert np.all(np.isnan(G.glcm_features(t3).cpu().numpy()))
    for k in (0, 2):
        for c in range(5):
            if want[k, c] == 0:
                assert got[k, c] == 0
            else:
                assert abs(got[k, c] - want[k, c]) <= 1e-5 * abs(want[k, c]), (k, c, got[k], want[k])


# ---------------------------------------------------------------- host-resident images (streamed tiles)

@pytest.mark.parametrize("tile_rows", [1, 7, 64, 1024])
@pytest.mark.parametrize("pinned", [False, True])
@pytest.mark.parametrize("serial", [False, True])
@pytest.mark.parametrize("merge", [0, 1])
def test_host_image_tiles(tile_rows, pinned, serial, merge):
    """Host images go up in row tiles with halo rows; each tile owns the pairs
    whose first pixel lies in its rows, so the sum over tiles is exact."""
    img = synth.smooth(301, 517, 3.0, 31, np.uint16, noise_frac=0.05)
    offs = synth.offsets_for([1, 2, 4]) + [(-2, -3), (3, -1)]
    flags = G.FLAG_SERIAL_UPLOAD if serial else 0
    plan = G.glcm_plan_create(np.uint16, 64, offs, 517, 301, flags)
    try:
        plan.set_tuning(tile_rows=tile_rows, merge=merge)
        src = torch.from_numpy(img.view(np.int16)).view(torch.uint16)
        if pinned:
            src = src.pin_memory()
        check(img, 64, 0, 65535, offs, plan=plan, t=src,
              label=f"host tiles={tile_rows} pinned={pinned} serial={serial}")
        check(img, 64, 0, 65535, offs, plan=plan, t=src, label="host again")
    finally:
        plan.close()


@pytest.mark.parametrize("offs,flags,path", [
    ([(0, -1)], 0, "strips"),
    ([(1, -1), (0, -2), (-2, -1)], 0, "strips"),
    ([(1, 1), (-2, -3)], 0, "slabs"),
    ([(0, -1), (-1, -1)], G.FLAG_FORCE_SLABS, "slabs"),
    ([(0, -4), (3, -2)], 0, "slabs"),
])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("tile_rows", [1, 6, 64])
def test_host_tiles_upward_offsets(offs, flags, path, dtype, tile_rows):
    """Offsets whose dy is negative, alone or larger than every positive dy:
    the strip and slab kernels count them from the upper pixel, so a tile needs
    max|dy| rows below it, whatever the positive offsets reach."""
    W, H = 203, 77
    img = synth.smooth(H, W, 2.0, 33, dtype) if dtype == np.uint8 else synth.smooth(H, W, 2.0, 33, dtype,
                                                                                    noise_frac=0.05)
    N, hi = (16, 255) if dtype == np.uint8 else (32, 65535)
    plan = G.glcm_plan_create(dtype, N, offs, W, H, flags)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == path, plan.tuning.as_dict()
        plan.set_tuning(tile_rows=tile_rows)
        src = torch.from_numpy(img if dtype == np.uint8 else img.view(np.int16))
        if dtype == np.uint16:
            src = src.view(torch.uint16)
        check(img, N, 0, hi, offs, plan=plan, t=src, label=f"host upward offs={offs} tiles={tile_rows} {path}")
    finally:
        plan.close()


def test_plan_cache_is_bounded():
    """100 calls with plan=None and 100 distinct offset sets (16 MiB of per-XCD
    accumulators each at N = 256, K = 4) keep at most 32 cached plans and
    512 MiB of device workspace; the results stay exact."""
    G.glcm_plan_cache_clear()
    img = synth.smooth(96, 80, 2.0, 41)
    t = to_device(img)
    free0 = torch.cuda.mem_get_info()[0]
    last = None
    for s in range(100):
        offs = [(1, 0), (0, 1), (s % 10 - 5, s // 10 - 5), (2, 2)]
        out = G.glcm_compute(t, 256, 0, 255, offs)
        n, b = G.glcm_plan_cache_stats()
        assert n <= 32 and b <= 512 << 20, (s, n, b)
        last = (offs, out)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    assert used < 700 << 20, f"device memory grew by {used >> 20} MiB"
    offs, out = last
    assert np.array_equal(to_host(out), oracle.glcm(img, 256, 0, 255, offs))
    G.glcm_plan_cache_clear()
    assert G.glcm_plan_cache_stats()[0] == 0


def test_host_numpy_strided_view():
    base = synth.uniform(200, 300, 32)
    view = base[5:190, 7:290]
    offs = synth.offsets_for([1])
    check(np.ascontiguousarray(view), 16, 0, 255, offs, t=view, label="numpy strided view")


def test_host_multispectral_band_streamed():
    img, sigma = synth.multispectral_band(1, size=2048)
    offs = synth.offsets_for([1, 2, 4])
    src = torch.from_numpy(img.view(np.int16)).view(torch.uint16).pin_memory()
    check(img, 64, 0, 65535, offs, t=src, label=f"multispectral 2048^2 streamed sigma={sigma:.1f}")


@pytest.mark.parametrize("merge", [0, 1])
def test_alternating_images_one_plan(merge):
    """Consecutive calls on one plan with different images: nothing carries over."""
    imgs = [synth.smooth(256, 1100, 2.0 + i, 50 + i) for i in range(3)] + [synth.constant(256, 1100, 200)]
    offs = synth.offsets_for([1, 2])
    wants = [oracle.glcm(im, 16, 0, 255, offs) for im in imgs]
    ts = [to_device(im) for im in imgs]
    plan = G.glcm_plan_create(np.uint8, 16, offs, 1100, 256)
    try:
        plan.set_tuning(merge=merge)
        outs = [G.glcm_compute(ts[i % 4], 16, 0, 255, offs, plan=plan) for i in range(24)]
        for i, o in enumerate(outs):
            assert np.array_equal(to_host(o), wants[i % 4]), i
    finally:
        plan.close()


@pytest.mark.parametrize("flags", [0, G.FLAG_FORCE_GENERIC])
def test_autotune_keeps_results(flags):
    img = synth.smooth(700, 1500, 6.0, 60)
    offs = synth.offsets_for([1, 2])
    plan = G.glcm_plan_create(np.uint8, 32, offs, 1500, 700, flags)
    try:
        t = plan.autotune(to_device(img), repeats=2)
        assert t.replicas >= 1 and t.wg_size in (256, 512, 1024)
        check(img, 32, 0, 255, offs, plan=plan, label=f"after autotune {t.as_dict()}")
    finally:
        plan.close()


@pytest.mark.parametrize("dtype,N,dists,path", [
    (np.uint8, 32, [1, 2], "strips"),     # 16 dwords per bin
    (np.uint8, 64, [1], "strips"),        # 8 dwords per bin, reach 1
    (np.uint8, 64, [2], "slabs"),         # 8 dwords per bin, reach 2
    (np.uint16, 64, [1, 2], "slabs"),     # 4 dwords per bin
    (np.uint16, 64, [1, 2, 4], "slabs"),  # beyond the strip kernel's reach
])
def test_strip_or_slab_default(dtype, N, dists, path):
    """The strip kernel is the default only with 16 or more dwords per bin, or
    8 at a reach of 1; otherwise the slab kernel (measured faster or equal).
    Both give the oracle's counts."""
    W, H = 1037, 93
    img = synth.smooth(H, W, 3.0, 90 + N, dtype) if dtype == np.uint8 else synth.smooth(H, W, 3.0, 90 + N, dtype,
                                                                                           noise_frac=0.05)
    hi = 255 if dtype == np.uint8 else 65535
    offs = synth.offsets_for(dists)
    plan = G.glcm_plan_create(dtype, N, offs, W, H)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == path, plan.tuning.as_dict()
        check(img, N, 0, hi, offs, plan=plan, label=f"default {path} N={N} d={dists}")
    finally:
        plan.close()


@pytest.mark.parametrize("kind", ["smooth", "uniform"])
def test_autotune_across_row_kernels(kind):
    """A plan whose offsets both row kernels reach: the autotuner times strip
    and slab layouts together and keeps one; the counts stay exact, and a
    plan created with FLAG_FORCE_SLABS stays on the slab kernel."""
    W, H = 2048, 512
    img = synth.smooth(H, W, 6.0, 95, np.uint16) if kind == "smooth" else synth.uniform(H, W, 96, np.uint16)
    offs = synth.offsets_for([2])
    t = torch.from_numpy(img.view(np.int16)).view(torch.uint16).cuda()
    for flags in (0, G.FLAG_FORCE_SLABS):
        plan = G.glcm_plan_create(np.uint16, 64, offs, W, H, flags)
        try:
            chosen = plan.autotune(t, 0, 65535, repeats=2)
            name = G.PATH_NAMES[chosen.path]
            print(f"[autotune] {kind} flags={flags}: {chosen.as_dict()}", flush=True)
            assert name in (("strips", "slabs") if flags == 0 else ("slabs",))
            check(img, 64, 0, 65535, offs, plan=plan, label=f"autotuned {name} {kind}")
        finally:
            plan.close()


def test_kernel_timing_flag():
    img = synth.uniform(512, 2048, 61)
    offs = synth.offsets_for([1])
    plan = G.glcm_plan_create(np.uint8, 16, offs, 2048, 512, G.FLAG_TIMING)
    try:
        t = to_device(img)
        for _ in range(3):
            check(img, 16, 0, 255, offs, plan=plan, t=t, label="timing")
        ms, n = plan.kernel_time()
        assert n == 3 and ms > 0
        assert plan.kernel_time() == (0.0, 0)
    finally:
        plan.close()


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("offs", [synth.offsets_for([1]), synth.offsets_for([1, 2, 4])])
def test_misaligned_views_read_in_place(dtype, offs):
    """Misaligned views (base or pitch not 16-byte aligned) of at least 2^16
    pixels are read in place by the strip and slab kernels, smaller ones by
    the per-pixel kernels: bit-exact whatever the byte offset of the rows,
    and the plan's workspace does not grow (no staging copy)."""
    top = int(np.iinfo(dtype).max)
    base = synth.smooth(520, 1100, 4.0, 41, dtype)
    t = to_device(base)
    plan = G.glcm_plan_create(dtype, 32, offs, 1100, 520)
    try:
        kernel = G.PATH_NAMES[plan.tuning.path]
        assert kernel in ("strips", "slabs")
        before = G.glcm_plan_workspace(plan)
        for y0, x0, h, w in ((1, 3, 500, 1001), (0, 1, 257, 1099), (7, 13, 300, 700), (2, 5, 40, 17),
                             (0, 7, 3, 1093), (11, 2, 509, 1), (5, 1, 1, 1024), (3, 9, 200, 1040)):
            sub = base[y0:y0 + h, x0:x0 + w]
            check(sub, 32, 0, top, offs, plan=plan, t=t[y0:y0 + h, x0:x0 + w],
                  label=f"{kernel} in place ({y0},{x0}) {h}x{w}")
        assert G.glcm_plan_workspace(plan) == before
    finally:
        plan.close()


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("N,dists", [(8, [1]), (16, [1, 2]), (64, [2]), (32, [1, 2, 4])])
def test_misaligned_views_every_layout(dtype, N, dists):
    """In-place reads on both row kernels and several layouts (copies,
    counter width), views starting at every byte offset of a dword."""
    top = int(np.iinfo(dtype).max)
    base = synth.smooth(300, 2100, 3.0, 42 + N, dtype)
    t = to_device(base)
    offs = synth.offsets_for(dists) + [(-dists[-1], 0), (0, -1)]
    plan = G.glcm_plan_create(dtype, N, offs, 2100, 300)
    try:
        kernel = G.PATH_NAMES[plan.tuning.path]
        for x0 in (1, 2, 3, 5, 6, 7):
            w = 2100 - x0 - (x0 * 37) % 50
            sub = base[x0:, x0:x0 + w]
            check(sub, N, 0, top, offs, plan=plan, t=t[x0:, x0:x0 + w], label=f"{kernel} N={N} view x0={x0} w={w}")
    finally:
        plan.close()


@pytest.mark.parametrize("N,K,W,path", [
    (256, 12, 4096, "partitioned"),    # 10 passes of 16-bit bins
    (1024, 2, 4096, "partitioned"),    # 26 passes: 13 per GLCM
    (1024, 4, 4096, "partitioned"),    # 52 passes: 13 per GLCM
    (1280, 1, 4096, "l2"),             # 21 passes for one GLCM
    (2048, 1, 4096, "l2"),
    (1024, 2, 70000, "l2"),            # rows too long for 16-bit bands: 52 passes of 32-bit bins
])
def test_large_n_path_choice(N, K, W, path):
    """LDS bin partitions while they cost at most 13 image passes per GLCM
    (counted as the kernel runs them), else pairs straight into the per-XCD
    L2 slices.  Plan creation only."""
    offs = synth.offsets_for([1, 2, 4])[:K]
    plan = G.glcm_plan_create(np.uint8, N, offs, W, 64)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == path, plan.tuning.as_dict()
    finally:
        plan.close()


@pytest.mark.parametrize("N,dtype,shape,offs", [
    (256, np.uint8, (60, 8200), synth.offsets_for([1, 2, 4])[:6]),   # bands of 7 rows (W > 4369)
    (256, np.uint8, (700, 300), synth.offsets_for([1, 2, 4])[:9]),
    (256, np.uint8, (301, 1500), synth.offsets_for([1, 2, 4])),        # 12 GLCMs: 10 passes of 16-bit bins
    (400, np.uint16, (130, 700), [(1, 0), (0, 1), (1, 1), (-1, 1), (2, 0)]),  # 5 GLCMs of 160000 bins: 10 passes
    (1024, np.uint8, (150, 900), [(1, 0), (-2, 2)]),                    # 2 GLCMs of 2^20 bins: 26 passes
    (1024, np.uint16, (90, 700), synth.offsets_for([1])),               # 4 GLCMs of 2^20 bins: 52 passes
    (400, np.uint16, (257, 1030), [(1, 0), (-2, 3), (0, -4)]),
    (256, np.uint8, (1, 70000), [(1, 0), (3, 0)]),                      # one row wider than 2^16
])
def test_partitioned_sixteen_bit_bins(N, dtype, shape, offs):
    """Bin partitions with 16-bit counters, two bins per dword: every band
    stays below 2^16 first pixels, so a constant image (all pairs in one bin
    per GLCM) must count exactly too."""
    H, W = shape
    top = int(np.iinfo(dtype).max)
    img = synth.smooth(H, W, 3.0, 51 + N, dtype) if H > 2 else synth.uniform(H, W, 52, dtype)
    plan = G.glcm_plan_create(dtype, N, offs, W, H)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == "partitioned"
        check(img, N, 0, top, offs, plan=plan, label=f"16-bit bins N={N} {W}x{H}")
        const = np.full((H, W), top // 3, dtype=dtype)
        check(const, N, 0, top, offs, plan=plan, label=f"16-bit bins constant N={N} {W}x{H}")
    finally:
        plan.close()
