"""GPU parity of the batched engine (glcm_batch_compute, through the C ABI):
every image of a batch against the CPU oracle, bit-exact counts and features
within 1e-5 relative of the fp64 oracle; aligned and misaligned images, u8 and
u16, narrow and wide images, offsets counted transposed, plan reuse."""

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


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    if t.dtype == torch.float32:
        return t.cpu().numpy()
    return t.view(torch.int32).cpu().numpy().view(np.uint32)


def check_features(got, want, label):
    got = got.astype(np.float64)
    zero = want == 0
    assert np.all(got[zero] == 0), f"{label}: exact zeros not kept"
    rel = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
    assert np.all(rel <= 1e-5), f"{label}: features off by {rel.max():.3g}"


def run_batch(imgs, N, lo, hi, offs, views=None, features=True, plan=None):
    dt = imgs[0].dtype
    tens = views if views is not None else [to_device(im) for im in imgs]
    own = plan is None
    if own:
        plan = G.glcm_plan_create(dt, N, offs, max(im.shape[1] for im in imgs), max(im.shape[0] for im in imgs))
    try:
        print(f"[batch] T={len(imgs)} dtype={dt} N={N} K={len(offs)} offsets={offs}", flush=True)
        out, feats = G.glcm_batch_compute(tens, plan, lo, hi, features=features)
        got = host(out)
        fgot = host(feats) if feats is not None else None
    finally:
        if own:
            plan.close()
    for t, im in enumerate(imgs):
        want = oracle.glcm(im, N, lo, hi, offs)
        if not np.array_equal(got[t], want):
            bad = np.argwhere(got[t] != want)
            raise AssertionError(f"image {t} {im.shape}: {len(bad)} bins differ, first {tuple(bad[0])}")
        if fgot is not None:
            check_features(fgot[t], oracle.features(want), f"image {t} {im.shape}")
    return got, fgot


def test_batch_tiles_workload_sample():
    w = synth.batch_tiles(96)
    run_batch(w["images"], w["N"], w["lo"], w["hi"], w["offsets"])


@pytest.mark.parametrize("shapes", [
    [(1, 1), (1, 40), (40, 1), (2, 2), (17, 3)],
    [(32, 32), (512, 512), (33, 511), (511, 33), (100, 1000), (7, 2100)],
    [(64, 64)] * 7 + [(300, 1100)],
])
def test_batch_shapes(shapes):
    imgs = [synth.smooth(h, w, 2.0, 500 + i, np.uint8) if min(h, w) > 2 else synth.uniform(h, w, 500 + i)
            for i, (h, w) in enumerate(shapes)]
    run_batch(imgs, 16, 0, 255, synth.offsets_for([1]))


@pytest.mark.parametrize("offs", [
    [(1, 0)], [(0, 1), (1, 0), (-1, -1)], [(2, 0), (-2, 2), (0, 2), (2, 2)],
    [(0, 0), (-1, 0), (1, -1), (0, -2)],
])
def test_batch_offsets(offs):
    imgs = [synth.smooth(90 + 7 * i, 130 + 11 * i, 3.0, 600 + i) for i in range(6)]
    run_batch(imgs, 32, 0, 255, offs)


@pytest.mark.parametrize("N,lo,hi", [(8, 0, 255), (24, 10, 240), (43, 0, 255), (1, 0, 255)])
def test_batch_levels_u8(N, lo, hi):
    imgs = [synth.uniform(50, 70, 700), synth.smooth(120, 64, 4.0, 701)]
    run_batch(imgs, N, lo, hi, synth.offsets_for([1]))


@pytest.mark.parametrize("N,lo,hi", [(32, 0, 65535), (40, 1000, 60000)])
def test_batch_u16(N, lo, hi):
    imgs = [synth.smooth(80 + 13 * i, 48 + 40 * i, 3.0, 800 + i, np.uint16, noise_frac=0.05) for i in range(5)]
    run_batch(imgs, N, lo, hi, synth.offsets_for([2]))


def test_batch_misaligned_and_strided_views():
    base = synth.smooth(300, 700, 4.0, 900)
    tb = to_device(base)
    cuts = [(0, 300, 0, 640), (3, 297, 1, 699), (10, 200, 16, 656), (0, 299, 5, 6), (7, 100, 33, 300)]
    imgs = [base[y0:y1, x0:x1] for y0, y1, x0, x1 in cuts]
    views = [tb[y0:y1, x0:x1] for y0, y1, x0, x1 in cuts]
    run_batch(imgs, 16, 0, 255, synth.offsets_for([1]), views=views)


@pytest.mark.parametrize("dt,N,lo,hi", [(np.uint8, 32, 0, 255), (np.uint16, 24, 0, 4095)])
def test_batch_misaligned_wide_views(dt, N, lo, hi):
    """Views whose base and row pitch are not 16-byte aligned, wider than one
    wavefront's 1024 columns, with reach-2 offsets."""
    base = synth.smooth(150, 2300, 5.0, 950, dt, noise_frac=0.05)
    tb = to_device(base)
    cuts = [(0, 150, 1, 2300), (2, 149, 3, 1030), (5, 60, 7, 1029), (1, 90, 1001, 2299), (9, 10, 11, 12)]
    imgs = [base[y0:y1, x0:x1] for y0, y1, x0, x1 in cuts]
    views = [tb[y0:y1, x0:x1] for y0, y1, x0, x1 in cuts]
    run_batch(imgs, N, lo, hi, synth.offsets_for([2]), views=views)


def test_batch_without_features_and_plan_reuse():
    offs = synth.offsets_for([1])
    plan = G.glcm_plan_create(np.uint8, 16, offs, 512, 512)
    try:
        for T, seed in [(5, 1000), (40, 1100), (3, 1200)]:  # grows and reuses the descriptor staging
            imgs = [synth.uniform(20 + 9 * i, 30 + 5 * i, seed + i) for i in range(T)]
            got, f = run_batch(imgs, 16, 0, 255, offs, features=False, plan=plan)
            assert f is None
    finally:
        plan.close()


def test_batch_matches_per_image_calls():
    w = synth.batch_tiles(32)
    N, offs = w["N"], w["offsets"]
    plan = G.glcm_plan_create(np.uint8, N, offs, 512, 512)
    try:
        tens = [to_device(im) for im in w["images"]]
        out, feats = G.glcm_batch_compute(tens, plan)
        for t, x in enumerate(tens):
            P = G.glcm_compute(x, N, 0, 255, offs, plan=plan)
            F = G.glcm_features(P)
            assert np.array_equal(host(out[t].contiguous()), host(P))
            assert np.array_equal(host(feats[t].contiguous()), host(F))
    finally:
        plan.close()


@pytest.mark.parametrize("N,offs", [(16, [(1, 0)] * 5), (16, [(4, 0)]), (16, [(0, 3)]), (255, [(1, 0)] * 4)])
def test_batch_unsupported(N, offs):
    """More than 4 offsets, a reach beyond 2, or LDS copies that do not fit."""
    plan = G.glcm_plan_create(np.uint8, N, offs, 64, 64)
    try:
        with pytest.raises(G.GlcmError) as e:
            G.glcm_batch_compute([to_device(synth.uniform(8, 8, 1))], plan)
        assert e.value.status == -3
    finally:
        plan.close()


def test_batch_rejects_oversize_images():
    plan = G.glcm_plan_create(np.uint8, 16, [(1, 0)], 64, 64)
    try:
        with pytest.raises(G.GlcmError) as e:
            G.glcm_batch_compute([to_device(synth.uniform(65, 8, 1))], plan)
        assert e.value.status == -1
    finally:
        plan.close()


def test_batch_rejects_memory_the_kernel_cannot_read_or_write():
    """Tiles must lie in device memory of the current device, outputs too,
    and no output may overlap a tile: GLCM_EINVAL before anything is queued
    (a host pointer read by the kernel would fault the GPU)."""
    import ctypes
    lib = G._lib()
    offs = [(1, 0)]
    plan = G.glcm_plan_create(np.uint8, 16, offs, 64, 64)
    dev_img = to_device(synth.uniform(64, 64, 5))
    pageable = torch.from_numpy(synth.uniform(64, 64, 6))
    pinned = pageable.pin_memory()
    out = torch.zeros((2, 1, 16, 16), dtype=torch.uint32, device="cuda")
    feat = torch.zeros((2, 1, 5), dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(imgs, o=None, f=None):
        arr = (G.Tile * len(imgs))(*[G.Tile(t.data_ptr(), 64, 64, 64) for t in imgs])
        return lib.glcm_batch_compute(plan.handle, arr, len(imgs), 0, 255,
                                      ctypes.c_void_p((o if o is not None else out).data_ptr()),
                                      ctypes.c_void_p(f.data_ptr()) if f is not None else None, stream)
    try:
        assert call([dev_img, dev_img], f=feat) == 0
        torch.cuda.synchronize()
        want = oracle.glcm(dev_img.cpu().numpy(), 16, 0, 255, offs)
        assert np.array_equal(host(out)[1], want)
        out.zero_()
        assert call([dev_img, pageable]) == -1, "pageable host tile accepted"
        assert call([pinned, dev_img]) == -1, "pinned host tile accepted"
        big = torch.zeros(64 * 64 * 4, dtype=torch.uint8, device="cuda")
        big[: 64 * 64].copy_(dev_img.flatten())
        assert call([big, dev_img], o=big.view(torch.uint32)[512:1024]) == -1, "out over a tile accepted"
        assert call([dev_img, dev_img], f=out.view(torch.float32).flatten()[:10]) == -1, "features over out accepted"
        host_out = torch.zeros((2, 1, 16, 16), dtype=torch.int32).pin_memory()
        assert call([dev_img, dev_img], o=host_out) == -1, "host output accepted"
        torch.cuda.synchronize()
        assert not host(out).any(), "a rejected call wrote the output"
        # a prepared batch checks its tiles once and its outputs at every run
        arr = (G.Tile * 2)(G.Tile(dev_img.data_ptr(), 64, 64, 64), G.Tile(pageable.data_ptr(), 64, 64, 64))
        h = ctypes.c_void_p()
        assert lib.glcm_batch_prepare(plan.handle, arr, 2, ctypes.byref(h)) == -1
        pb = G.PreparedBatch([dev_img, dev_img], plan)
        try:
            assert lib.glcm_batch_run(pb.handle, 0, 255, ctypes.c_void_p(host_out.data_ptr()), None, stream) == -1
            assert lib.glcm_batch_run(pb.handle, 0, 255, ctypes.c_void_p(dev_img.data_ptr()), None, stream) == -1
            o2, _ = pb.run()
            assert np.array_equal(host(o2)[0], want)
        finally:
            pb.close()
    finally:
        plan.close()


def test_prepared_batch_runs_and_graph_replays():
    """A prepared batch equals glcm_batch_compute; captured in a graph it is
    replayed several times, with eager work on the same images in between
    (which changes their pixels), and every replay is checked against an
    eager run of the same pixels."""
    w = synth.batch_tiles(48)
    imgs = w["images"]
    N, offs = w["N"], w["offsets"]
    tens = [to_device(im) for im in imgs]
    plan = G.glcm_plan_create(np.uint8, N, offs, 512, 512)
    pb = G.PreparedBatch(tens, plan)
    try:
        ref_out, ref_f = G.glcm_batch_compute(tens, plan)
        out, f = pb.run(features=True)
        assert np.array_equal(host(out), host(ref_out)) and np.array_equal(host(f), host(ref_f))
        # capture one run into a graph on a side stream
        g_out = torch.empty_like(out)
        g_f = torch.empty_like(f)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            pb.run(out=g_out, features=g_f, stream=side)  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            pb.run(out=g_out, features=g_f, stream=side)
        torch.cuda.synchronize()
        for rep in range(4):
            for t in tens:  # eager work in between: new pixels in place
                t.copy_((t.to(torch.int32) * 7 + rep + 1).remainder(256).to(torch.uint8))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            e_out, e_f = G.glcm_batch_compute(tens, plan)
            assert np.array_equal(host(g_out), host(e_out)), f"replay {rep}: counts differ from the eager run"
            assert np.array_equal(host(g_f), host(e_f)), f"replay {rep}: statistics differ from the eager run"
        last = [t.cpu().numpy() for t in tens[:4]]
        for i, im in enumerate(last):
            assert np.array_equal(host(g_out)[i], oracle.glcm(im, N, 0, 255, offs))
    finally:
        pb.close()
        plan.close()


def test_batch_layouts_are_all_exact():
    """Every batch layout (LDS copies x shortest row run) gives the same counts
    and statistics, equal to the oracle."""
    w = synth.batch_tiles(40)
    imgs, N, offs = w["images"], w["N"], w["offsets"]
    tens = [to_device(im) for im in imgs]
    plan = G.glcm_plan_create(np.uint8, N, offs, 512, 512)
    try:
        ref_out, ref_f = G.glcm_batch_compute(tens, plan)
        ref_out, ref_f = host(ref_out), host(ref_f)
        for t in range(0, 40, 5):
            assert np.array_equal(ref_out[t], oracle.glcm(imgs[t], N, 0, 255, offs))
        for D in (4, 8, 16):
            for rows in (1, 3, 8, 32):
                bt = plan.set_batch_tuning(replicas=D, min_rows=rows)
                assert (bt.replicas, bt.min_rows, bt.wg_size) == (D, rows, 256)
                print(f"[batch layout] D={D} min_rows={rows}", flush=True)
                o, f = G.glcm_batch_compute(tens, plan)
                assert np.array_equal(host(o), ref_out), (D, rows)
                assert np.array_equal(host(f), ref_f), (D, rows)
        with pytest.raises(G.GlcmError):
            plan.set_batch_tuning(replicas=32)
        with pytest.raises(G.GlcmError):
            plan.set_batch_tuning(min_rows=300)
    finally:
        plan.close()


def test_batch_autotune_keeps_a_measured_layout():
    w = synth.batch_tiles(64)
    imgs, N, offs = w["images"], w["N"], w["offsets"]
    tens = [to_device(im) for im in imgs]
    plan = G.glcm_plan_create(np.uint8, N, offs, 512, 512)
    try:
        ref_out, ref_f = G.glcm_batch_compute(tens, plan)
        chosen = plan.batch_autotune(tens, repeats=2)
        assert chosen.replicas in (4, 8, 16) and chosen.min_rows in (4, 8, 16, 32) and chosen.wg_size in (256, 512)
        assert plan.batch_tuning.as_dict() == chosen.as_dict()
        o, f = G.glcm_batch_compute(tens, plan)
        assert np.array_equal(host(o), host(ref_out)) and np.array_equal(host(f), host(ref_f))
        for t in range(0, 64, 8):
            assert np.array_equal(host(o)[t], oracle.glcm(imgs[t], N, 0, 255, offs))
    finally:
        plan.close()


@pytest.mark.parametrize("dt,N,lo,hi", [(np.uint8, 16, 0, 255), (np.uint16, 24, 100, 60000)])
def test_batch_large_images_split_into_bands(dt, N, lo, hi):
    """Images above 2^20 pixels are counted as bands of rows by several
    workgroups and summed by k_batch_fin: band edges must neither drop nor
    double a pair, for offsets reaching two rows down or up (counted
    transposed), narrow and wide images, next to small whole images."""
    shapes = [(4200, 260), (1030, 1100), (129, 9000), (300, 301), (33, 35), (1, 70000)]
    imgs = [synth.smooth(h, w, 3.0, 900 + i, dt, noise_frac=0.05) for i, (h, w) in enumerate(shapes)]
    offs = [(1, 0), (-2, 2), (0, -2), (2, 1)]
    run_batch(imgs, N, lo, hi, offs)


def test_batch_misaligned_bands():
    base = to_device(synth.smooth(1500, 1301, 4.0, 950))
    views = [base[:, 1:], base[3:1450, 5:801], base[:500, 7:1000]]
    imgs = [v.cpu().numpy() for v in views]
    run_batch(imgs, 32, 0, 255, [(1, 0), (-1, 1), (0, 1), (1, 1)], views=views)


@pytest.mark.parametrize("wg", [256, 512])
@pytest.mark.parametrize("D", [4, 16])
def test_batch_workgroup_sizes(wg, D):
    w = synth.batch_tiles(160)
    imgs, N, offs = w["images"], w["N"], w["offsets"]
    imgs = imgs + [synth.smooth(1100, 1000, 4.0, 977)]  # one image split into bands
    plan = G.glcm_plan_create(np.uint8, N, offs, 1100, 1100)
    try:
        t = plan.set_batch_tuning(replicas=D, min_rows=8, wg_size=wg)
        assert (t.replicas, t.wg_size) == (D, wg)
        run_batch(imgs, N, w["lo"], w["hi"], offs, plan=plan)
    finally:
        plan.close()
