"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: tile assignment, key order and tile ranges bit-exact; images
max-abs 1e-4 over pixels with no decision within a relative 1e-5 (alpha) /
1e-4 (transmittance) of its threshold; gradients relative 1e-3 in L2 per
tensor (FP32 atomics make the summation order nondeterministic).
"""
import numpy as np
import pytest

from paper_2409_13055_amd import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle.oracle as O  # noqa: E402
from tests import gpu_util as U  # noqa: E402


def small_scene(seed=3, n=2000, D=3, tile_div=1):
    cams = [S.pinhole(130, 97, 110.0), S.pinhole(100, 76, 90.0, *S.look_at((0.35, -0.1, -0.5), (0.0, 0.0, 3.0)))]
    return S.make_scene(seed, n, D, cams, "box", log_scale_mu=-3.3, log_scale_sigma=0.6, logit_sigma=1.5)


def check_projection(sc, g, opts):
    P = O.Params.from_scene(sc)
    ref = O.project_views(P, sc.cameras, opts)
    rec = g["rec"].astype(np.float64)
    ext = U.gpu_extents(g["rec"])
    fl = ref["flags"]
    vis_o = ref["radius"] > 0
    vis_g = ext[:, 0] > 0
    boundary = (fl & (O.F_NEAR_RADIUS | O.F_NEAR_RECT | O.F_NEAR_PLANE)) != 0
    assert np.array_equal(vis_o[~boundary], vis_g[~boundary]), "culling differs"
    both = vis_o & vis_g
    r = ref["rec"]
    assert np.abs(rec[both, 0] - r[both, 0]).max() <= 1e-3
    assert np.abs(rec[both, 1] - r[both, 1]).max() <= 1e-3
    cscale = np.maximum(np.abs(r[both, 3]), np.abs(r[both, 5]))
    for gi, oi in ((2, 3), (3, 4), (4, 5)):
        assert (np.abs(rec[both, gi] - r[both, oi]) / cscale).max() <= 1e-4, f"conic {gi}"
    assert (np.abs(rec[both, 9] - r[both, 2]) / r[both, 2]).max() <= 1e-6, "depth"
    assert (np.abs(rec[both, 5] - r[both, 6]) / r[both, 6]).max() <= 1e-6, "opacity"
    assert np.abs(rec[both, 6:9] - r[both, 7:10]).max() <= 1e-5, "rgb"
    ok = both & ~boundary
    assert np.array_equal(ext[ok], ref["ext"][ok]), "rect half-extents"
    rect_area = (ref["rect"][:, 2] - ref["rect"][:, 0]) * (ref["rect"][:, 3] - ref["rect"][:, 1])
    assert np.array_equal(g["tiles"][ok], rect_area[ok]), "tiles touched"
    return int(boundary.sum())


def check_bins(sc, g, tile):
    rec = g["rec"]
    keys, ids, ranges = O.bin_sort(rec[:, 0:2], U.gpu_extents(rec), rec[:, 9], sc.cameras, tile)
    assert g["m"] == ids.shape[0]
    assert np.array_equal(g["ids"], ids)
    assert np.array_equal(g["ranges"], ranges)
    if g["keys"] is not None:
        assert np.array_equal(g["keys"], keys)


def check_image_pinned(sc, g, opts):
    ref = O.render(sc.cameras, opts, U.gpu_rec_to_oracle(g["rec"]), g["ids"], g["ranges"])
    ok = ref["pix_flags"] == 0
    assert ok.mean() > 0.999
    P = ref["t_final"].shape[0]
    img_g, img_o = g["image"], ref["image"]
    # per-view planar layout: pixel mask repeated per channel
    mask = np.concatenate([np.tile(ok[off:off + c.width * c.height], 3) for off, c in
                           zip(np.cumsum([0] + [c.width * c.height for c in sc.cameras])[:-1], sc.cameras)])
    assert mask.shape[0] == 3 * P
    assert np.abs(img_g - img_o)[mask].max() <= 1e-4
    if "t_final" in g:
        assert np.abs(g["t_final"] - ref["t_final"])[ok].max() <= 1e-4
        assert np.array_equal(g["n_contrib"][ok], ref["n_contrib"][ok])
    return ref


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_forward_backward_parity_two_views(tile):
    sc = small_scene()
    opts = O.Options(tile=tile)
    g = U.run_gpu(sc, tile=tile)
    check_projection(sc, g, opts)
    check_bins(sc, g, tile)
    check_image_pinned(sc, g, opts)
    # loss value
    loss_ref = O.l1_loss_per_view(g["image"], sc.targets, sc.cameras)
    np.testing.assert_allclose(g["loss"], loss_ref, rtol=1e-5)
    # image-space gradients (pinned lists, dL/dC from the GPU image)
    orec = U.gpu_rec_to_oracle(g["rec"])
    _, dl = O.l1_loss(g["image"], sc.targets, sc.cameras)
    g2_ref = O.render_backward(sc.cameras, opts, orec, g["ids"], g["ranges"], dl)
    for c in range(9):
        assert U.rel_l2(g["grad2d"][:, c], g2_ref[:, c]) <= 1e-3, (c, U.rel_l2(g["grad2d"][:, c], g2_ref[:, c]))
    # projection backward alone: oracle chain rule fed with the GPU's image-space gradients
    P = O.Params.from_scene(sc)
    U.compare_grads(g["grads"], O.project_backward(P, sc.cameras, opts, g["grad2d"]), 1e-3, "chain")
    # end to end against the oracle's own image-space gradients
    U.compare_grads(g["grads"], O.project_backward(P, sc.cameras, opts, g2_ref), 1e-3, "end-to-end")


@pytest.mark.parametrize("tile", [16, 32])
def test_wave_block_cull_on_needles(tile):
    """Strongly anisotropic splats at random orientations (log-scales N(-2.8, 1.3) per axis, so long
    needles cross many wavefront blocks diagonally) and opacities spread around alpha_min: the
    wave-level cull below the tile must drop no entry that a pixel would blend.  The oracle has no
    such cull, so a dropped entry shows as an image, transmittance or contributor-count mismatch."""
    cams = [S.pinhole(150, 113, 120.0), S.pinhole(97, 131, 80.0, *S.look_at((0.2, 0.3, -0.4), (0.0, 0.0, 3.0)))]
    sc = S.make_scene(29 + tile, 1500, 1, cams, "box", log_scale_mu=-2.8, log_scale_sigma=1.3,
                      logit_sigma=2.0, transparent_frac=0.3)
    opts = O.Options(tile=tile)
    g = U.run_gpu(sc, tile=tile)
    check_bins(sc, g, tile)
    orec = U.gpu_rec_to_oracle(g["rec"])
    ref = O.render(sc.cameras, opts, orec, g["ids"], g["ranges"])
    ok = ref["pix_flags"] == 0
    assert ok.mean() > 0.98, ok.mean()
    mask = np.concatenate([np.tile(ok[off:off + c.width * c.height], 3) for off, c in
                           zip(np.cumsum([0] + [c.width * c.height for c in cams])[:-1], cams)])
    assert np.abs(g["image"] - ref["image"])[mask].max() <= 1e-4
    assert np.abs(g["t_final"] - ref["t_final"])[ok].max() <= 1e-4
    assert np.array_equal(g["n_contrib"][ok], ref["n_contrib"][ok])
    _, dl = O.l1_loss(g["image"], sc.targets, cams)
    g2_ref = O.render_backward(cams, opts, orec, g["ids"], g["ranges"], dl)
    for c in range(9):
        assert U.rel_l2(g["grad2d"][:, c], g2_ref[:, c]) <= 1e-3, (c, U.rel_l2(g["grad2d"][:, c], g2_ref[:, c]))


def test_projection_segments_list_the_visible_pairs():
    """The projection's hand-off to the bin sort: per (view, 64 Gaussians) segment, the visible pairs
    in ascending id with their depth bits and a tile rect of the pair's tile count; together, in
    segment order, exactly the pairs with tiles_touched > 0 in (v*N+i) order."""
    sc = small_scene(seed=5, n=3001)
    g = U.run_gpu(sc, tile=16, backward=False)
    fr = g["frame"]
    n, V = sc.n, len(sc.cameras)
    S_ = (n + 63) // 64
    cnt = fr.vis_count.cpu().numpy().astype(np.int64)
    ent = fr.vis.cpu().numpy().view(np.uint32).reshape(V * S_, 64, 4)
    assert cnt.shape == (V * S_,) and cnt.min() >= 0 and cnt.max() <= 64
    got = np.concatenate([ent[s, :cnt[s]] for s in range(V * S_)])
    tiles = g["tiles"]
    vis = np.nonzero(tiles > 0)[0]
    assert np.array_equal(got[:, 2], vis.astype(np.uint32))
    seg_of = (vis // n) * S_ + (vis % n) // 64
    assert np.array_equal(np.repeat(np.arange(V * S_), cnt), seg_of)
    depth_bits = np.ascontiguousarray(g["rec"][vis, 9]).view(np.uint32)
    assert np.array_equal(got[:, 3], depth_bits)
    x0, x1, y0, y1 = got[:, 0] & 0xffff, got[:, 0] >> 16, got[:, 1] & 0xffff, got[:, 1] >> 16
    assert np.all(x1 > x0) and np.all(y1 > y0)
    assert np.array_equal((x1 - x0) * (y1 - y0), tiles[vis].astype(np.uint32))


def test_forward_independent_mode():
    """Whole FP64 pipeline (own projection, binning, sort) vs the GPU: differences are confined to
    rare discrete flips."""
    sc = S.make_config(1)
    opts = O.Options(tile=16)
    g = U.run_gpu(sc, backward=False)
    ref = O.forward(O.Params.from_scene(sc), sc.cameras, opts)
    d = np.abs(g["image"] - ref["image"]).reshape(3, -1).max(axis=0)
    assert (d > 1e-4).mean() < 0.005, (d > 1e-4).mean()
    assert np.median(d) < 1e-6


def test_checkpoint_recompute_matches_stored():
    sc = small_scene(seed=8, n=1500)
    a = U.run_gpu(sc, checkpoint=False)
    b = U.run_gpu(sc, checkpoint=True)
    assert np.array_equal(a["image"], b["image"])
    for k in a["grads"]:
        assert U.rel_l2(b["grads"][k], a["grads"][k]) <= 1e-5, k


def test_batched_equals_per_view():
    sc = small_scene(seed=9, n=1500)
    both = U.run_gpu(sc)
    parts = []
    for v, c in enumerate(sc.cameras):
        sv = S.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh_dc, sc.sh_rest, sc.sh_degree, [c],
                     [sc.targets[v]])
        parts.append(U.run_gpu(sv))
    npx = [c.width * c.height for c in sc.cameras]
    np.testing.assert_array_equal(both["image"], np.concatenate([p["image"] for p in parts]))
    for k in both["grads"]:
        assert U.rel_l2(both["grads"][k], parts[0]["grads"][k] + parts[1]["grads"][k]) <= 1e-5, k
    # batched ranges are the per-view ranges shifted by the earlier views' pair counts
    T0 = parts[0]["ranges"].shape[0]
    np.testing.assert_array_equal(both["ranges"][:T0], parts[0]["ranges"])
    r1 = parts[1]["ranges"].astype(np.int64)
    shifted = np.where(r1[:, 1:2] > 0, r1 + parts[0]["m"], 0)
    np.testing.assert_array_equal(both["ranges"][T0:], shifted)
    assert npx[0] > 0


def test_empty_and_degenerate_inputs():
    sc = small_scene(seed=4, n=64, D=0)
    sc.means[:, 2] = -5.0  # all behind the camera
    g = U.run_gpu(sc)
    assert g["m"] == 0
    assert np.all(g["image"] == 0.0) and np.all(g["t_final"] == 1.0) and np.all(g["n_contrib"] == 0)
    for k, v in g["grads"].items():
        assert np.all(v == 0.0), k
    # a single Gaussian; a zero quaternion culls
    sc1 = small_scene(seed=4, n=1, D=1)
    sc1.means[0] = (0.0, 0.0, 3.0)
    sc1.log_scales[0] = np.log(0.1)
    g1 = U.run_gpu(sc1)
    assert g1["m"] > 0
    check_image_pinned(sc1, g1, O.Options(tile=16))
    sc1.quats[0] = 0.0
    g0 = U.run_gpu(sc1)
    assert g0["m"] == 0


def test_capacity_overflow_is_reported_and_recovers():
    import torch as T
    from paper_2409_13055_amd import rasterizer as R
    sc = small_scene(seed=5, n=800)
    params = R.GaussianParams.from_scene(sc, "cuda")
    rast = R.Rasterizer(sc.cameras, params.n, params.sh_degree, device="cuda")
    rast.reserve(100)
    fr = rast.new_frame()
    rast.project(params, fr)
    rast.bin_sort(fr)
    T.cuda.synchronize()
    assert int(fr.d_overflow.item()) == 1
    m = int(fr.d_num_pairs.item())
    assert m > 100
    assert rast.fit_capacity(fr)
    assert int(fr.d_num_pairs.item()) == m and int(fr.d_overflow.item()) == 0


def test_invalid_arguments_raise():
    from paper_2409_13055_amd import _lib as L
    from paper_2409_13055_amd import rasterizer as R
    sc = small_scene(seed=5, n=10)
    params = R.GaussianParams.from_scene(sc, "cuda")
    with pytest.raises(L.GsError) as ei:
        R.Rasterizer(sc.cameras, params.n, params.sh_degree, tile_size=12, device="cuda")
    assert "UNSUPPORTED" in str(ei.value)
    rast = R.Rasterizer(sc.cameras, params.n, params.sh_degree, device="cuda")
    fr = rast.new_frame()
    bad = params.c_params()
    bad.sh_degree = 7
    with pytest.raises(L.GsError) as ei:
        L.gs_project(bad, rast.cams, rast.n_views, rast.opts, fr.c_proj(), None)
    assert "INVALID_VALUE" in str(ei.value) and "sh_degree" in str(ei.value)


def test_adam_matches_oracle():
    import torch as T
    from paper_2409_13055_amd import rasterizer as R
    rng = np.random.default_rng(0)
    n = 1001  # ragged: not a multiple of the vector width
    sc = small_scene(seed=6, n=n, D=3)
    params = R.GaussianParams.from_scene(sc, "cuda")
    grads = params.zeros_like()
    lrs = dict(S.DEFAULT_LRS)
    opt = R.FusedAdam(params, grads, lrs)
    ref = {k: (getattr(params, k).cpu().numpy().astype(np.float64), 0.0, 0.0) for k in R.PARAM_NAMES}
    mag = {k: 0.0 for k in R.PARAM_NAMES}  # |m| recurrence: scale of the first moment's rounding error
    for step in range(1, 4):
        gs = {}
        for k in R.PARAM_NAMES:
            g = rng.standard_normal(getattr(params, k).shape).astype(np.float32) * 10 ** rng.uniform(-5, -1)
            getattr(grads, k).copy_(T.as_tensor(g))
            gs[k] = g.astype(np.float64)
        opt.step(zero_grad=True)
        T.cuda.synchronize()
        for k in R.PARAM_NAMES:
            p0, m, v = ref[k]
            p, m, v = O.adam_step(p0, gs[k], m, v, step, lrs[k])
            ref[k] = (p, m, v)
            mag[k] = 0.9 * mag[k] + 0.1 * np.abs(gs[k])
            # relative 1e-6 of the parameter or of its update, whichever is larger (an update can
            # cancel most of the parameter), plus FP32 rounding of the stored value
            got = getattr(params, k).cpu().numpy().astype(np.float64)
            tol = 1e-6 * np.maximum(np.abs(p), np.abs(p - p0)) + np.spacing(np.float32(np.abs(p))).astype(np.float64)
            assert np.all(np.abs(got - p) <= tol), (k, np.max(np.abs(got - p) / tol))
            # first moment: relative to the magnitude of its terms (a new gradient can cancel it)
            gm = getattr(opt.exp_avg, k).cpu().numpy().astype(np.float64)
            assert np.all(np.abs(gm - m) <= 2e-6 * mag[k] + 1e-30), (k, np.max(np.abs(gm - m) / mag[k]))
            # second moment: a sum of non-negative terms
            np.testing.assert_allclose(getattr(opt.exp_avg_sq, k).cpu().numpy(), v, rtol=2e-6, atol=1e-30)
            assert np.all(getattr(grads, k).cpu().numpy() == 0.0)
    assert int(opt.d_step.item()) == 3


@pytest.mark.parametrize("workload,tile", [(2, 16), (3, 16), (3, 8), (4, 32)])
def test_bin_sort_bitexact_full_size(workload, tile):
    """Full-size workloads: tile assignment, key order and ranges equal the oracle's stable sort of
    the (tile, depth bits, id) keys computed from the GPU's own FP32 records."""
    sc = S.make_config(workload)
    g = U.run_gpu(sc, tile=tile, backward=False)
    assert g["m"] > 500_000
    check_bins(sc, g, tile)


def test_render_stats_counts_match_oracle():
    """gs_render_stats (work counts used for roofline accounting) against the oracle's per-pixel
    trace, on the GPU's own lists and records."""
    sc = small_scene(seed=13, n=3000)
    g = U.run_gpu(sc, backward=False)
    rast, fr = g["rast"], g["frame"]
    st = rast.render_stats(fr)
    opts = O.Options(tile=16)
    orec = U.gpu_rec_to_oracle(g["rec"])
    ev, bl = O.pixel_counts(sc.cameras, opts, orec, g["ids"], g["ranges"])
    ref = O.render(sc.cameras, opts, orec, g["ids"], g["ranges"])
    flagged = ref["pix_flags"] != 0
    assert st["contrib_prefix"] == int(g["n_contrib"].astype(np.int64).sum())
    # decisions can only differ at flagged pixels
    assert abs(st["evaluated"] - int(ev.sum())) <= int(ev[flagged].sum())
    assert abs(st["blended"] - int(bl.sum())) <= int(bl[flagged].sum())
    assert st["blended"] > 0 and st["evaluated"] >= st["blended"]
