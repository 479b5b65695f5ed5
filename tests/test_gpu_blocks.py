"""GPU parity of the block-code kernel (the four d = 1 directions), bit-exact
against the CPU oracle: the full-size 4096^2 workload on smooth, noisy and
constant images, ragged shapes and band heights, uint16, offset subsets,
opposite directions and repeats, host images in tiles, and the offsets it does
not take (which go to the other kernels)."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_1710_06189_amd")

D1 = [(1, 0), (-1, 1), (0, 1), (1, 1)]


def to_device(img):
    if img.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(img).view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def run(img, N, lo, hi, offs, flags=G.FLAG_FORCE_BLOCKS, tile=None, expect_path="blocks"):
    H, W = img.shape
    dt = G.U16 if img.dtype == np.uint16 else G.U8
    print(f"[blocks] shape={img.shape} dtype={img.dtype} N={N} K={len(offs)} tile={tile}", flush=True)
    plan = G.glcm_plan_create(dt, N, offs, W, H, flags)
    try:
        assert G.PATH_NAMES[plan.tuning.path] == expect_path, plan.tuning.as_dict()
        if tile is not None:
            plan.set_tuning(tile_rows=tile)
            src = torch.from_numpy(img if img.dtype == np.uint8 else img.view(np.int16))
            if img.dtype == np.uint16:
                src = src.view(torch.uint16)
        else:
            src = to_device(img)
        out = torch.empty((len(offs), N, N), dtype=torch.uint32, device="cuda")
        G.glcm_compute(src, N, lo, hi, offs, plan=plan, out=out)
        torch.cuda.synchronize()
        got = out.view(torch.int32).cpu().numpy().view(np.uint32)
    finally:
        plan.close()
    want = oracle.glcm(img, N, lo, hi, offs)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        k, i, j = bad[0]
        raise AssertionError(f"{len(bad)} bins differ, first k={k} i={i} j={j}: gpu {got[k, i, j]} "
                             f"oracle {want[k, i, j]}")


@pytest.mark.parametrize("kind", ["smooth", "uniform", "constant"])
def test_square_4096(kind):
    w = synth.square_4096(kind)
    run(w["images"][0], w["N"], w["lo"], w["hi"], w["offsets"])


SHAPES = [(1, 1), (1, 37), (37, 1), (15, 16), (16, 15), (17, 33), (64, 63), (65, 129), (1023, 3), (3, 1025),
          (1040, 77), (2000, 31), (4097, 5), (1025, 1025)]


@pytest.mark.parametrize("W,H", SHAPES)
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_ragged_shapes(W, H, dtype):
    img = synth.smooth(H, W, 3.0, 200 + W + H, dtype) if W > 2 and H > 2 else synth.uniform(H, W, 5, dtype)
    run(img, 32, 0, int(np.iinfo(dtype).max), D1)


@pytest.mark.parametrize("sigma", [1.0, 2.0, 4.0, 16.0])
@pytest.mark.parametrize("N", [2, 8, 16, 32, 50])
def test_smoothness_and_levels(sigma, N):
    run(synth.smooth(300, 700, sigma, int(sigma * 10) + N), N, 0, 255, D1)


@pytest.mark.parametrize("offs", [
    [(1, 0)], [(1, 1)], [(-1, 1), (0, 1)], [(-1, 0), (0, -1), (-1, -1), (1, -1)],
    D1 + [(-1, 0), (1, -1)], [(0, 1), (0, 1), (1, 0)], D1 * 3,
])
def test_offset_sets(offs):
    run(synth.smooth(257, 513, 4.0, 31), 24, 0, 255, offs)


def test_quantizer_general_u16():
    img = synth.smooth(200, 300, 3.0, 41, np.uint16, noise_frac=0.01)
    run(img, 13, 1000, 60000, D1)


@pytest.mark.parametrize("tile", [1, 7, 64])
def test_host_image_tiles(tile):
    run(synth.smooth(150, 333, 4.0, 51), 32, 0, 255, D1 + [(-1, 0)], tile=tile)


def test_band_partial_merge_takes_strips():
    """The block kernel merges into the per-XCD slices only; with the band-
    partial merge selected, the plan counts on the strip kernel."""
    img = synth.smooth(200, 300, 4.0, 71)
    plan = G.glcm_plan_create(G.U8, 32, D1, 300, 200, G.FLAG_FORCE_BLOCKS)
    try:
        plan.set_tuning(merge=1)
        out = G.glcm_compute(to_device(img), 32, 0, 255, D1, plan=plan)
        torch.cuda.synchronize()
        got = out.view(torch.int32).cpu().numpy().view(np.uint32)
    finally:
        plan.close()
    assert np.array_equal(got, oracle.glcm(img, 32, 0, 255, D1))


def test_other_offsets_take_other_kernels():
    run(synth.smooth(100, 200, 4.0, 61), 16, 0, 255, [(1, 0), (2, 0)], expect_path="strips")
    run(synth.smooth(100, 200, 4.0, 62), 64, 0, 255, D1, expect_path="strips")


@pytest.mark.parametrize("kind", ["smooth", "uniform"])
def test_misaligned_view_is_staged(kind):
    t = to_device(np.ascontiguousarray(synth.square_4096(kind)["images"][0][:1000, :1002]))
    view = t[:, 1:]  # base + 1 byte, pitch 1002: not 16-byte aligned
    plan = G.glcm_plan_create(G.U8, 32, D1, 1001, 1000, G.FLAG_FORCE_BLOCKS)
    try:
        out = G.glcm_compute(view, 32, 0, 255, D1, plan=plan)
        torch.cuda.synchronize()
        got = out.view(torch.int32).cpu().numpy().view(np.uint32)
    finally:
        plan.close()
    want = oracle.glcm(np.ascontiguousarray(view.cpu().numpy()), 32, 0, 255, D1)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kind", ["smooth", "uniform"])
def test_autotune_between_row_kernels_and_blocks(kind):
    """glcm_plan_autotune times the block-code kernel against the strip and
    slab layouts for a d = 1 plan; whichever it keeps, the counts stay exact."""
    w = synth.square_4096(kind)
    img = w["images"][0]
    t = to_device(img)
    plan = G.glcm_plan_create(G.U8, 32, D1, 4096, 4096)
    try:
        chosen = plan.autotune(t, 0, 255, repeats=3)
        name = G.PATH_NAMES[chosen.path]
        print(f"[autotune] {kind}: {chosen.as_dict()}", flush=True)
        assert name in ("strips", "slabs", "blocks")
        assert G.PATH_NAMES[plan.tuning.path] == name
        out = G.glcm_compute(t, 32, 0, 255, D1, plan=plan)
        torch.cuda.synchronize()
        got = out.view(torch.int32).cpu().numpy().view(np.uint32)
    finally:
        plan.close()
    assert np.array_equal(got, oracle.glcm(img, 32, 0, 255, D1))


def test_autotune_keeps_other_offsets_off_blocks():
    img = synth.smooth(300, 400, 4.0, 81)
    plan = G.glcm_plan_create(G.U8, 16, [(1, 0), (2, 0)], 400, 300)
    try:
        chosen = plan.autotune(to_device(img), 0, 255, repeats=2)
        assert G.PATH_NAMES[chosen.path] != "blocks"
    finally:
        plan.close()
