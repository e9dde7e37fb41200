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
    orec = U.gpu_rec_to_oracle(g["rec"])
    ref = O.render(sc.cameras, opts, orec, g["ids"], g["ranges"])
    ok = ref["pix_flags"] == 0
    assert ok.mean() > 0.999
    U.check_image_one_flip(sc.cameras, opts, orec, g["ids"], g["ranges"], g["image"], ref, msg="pinned lists")
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
    g2_ref, mag = O.render_backward_mag(sc.cameras, opts, orec, g["ids"], g["ranges"], dl)
    U.compare_grad2d(g["grad2d"], g2_ref, msg=f"two views, tile {tile}", mag=mag)
    # projection backward alone: oracle chain rule fed with the GPU's image-space gradients
    P = O.Params.from_scene(sc)
    U.compare_grads(g["grads"], O.project_backward(P, sc.cameras, opts, g["grad2d"]), 1e-3, "chain")
    # end to end against the oracle's own image-space gradients
    U.compare_grads(g["grads"], O.project_backward(P, sc.cameras, opts, g2_ref), 1e-3, "end-to-end")


@pytest.mark.parametrize("tile", [8, 32])
def test_the_most_views_of_ragged_sizes(tile):
    """GS_MAX_VIEWS (32) views in one call, every one of another size that is not a multiple of the tile
    or of the 8-tile binning window (one pixel wide and tall among them), from scattered camera centres:
    projection, bins (bit-exact), image and image-space gradients against the oracle."""
    from paper_2409_13055_amd import _lib as L
    rng = np.random.default_rng(41)
    sizes = [(1, 1), (1, 37), (29, 1)] + [(int(rng.integers(3, 150)), int(rng.integers(3, 120)))
                                          for _ in range(L.GS_MAX_VIEWS - 3)]
    cams = []
    for w, h in sizes:
        eye = (rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), rng.uniform(-0.8, -0.2))
        cams.append(S.pinhole(w, h, max(0.9 * max(w, h), 1.0), *S.look_at(eye, (0.0, 0.0, 3.0))))
    sc = S.make_scene(43 + tile, 1500, 1, cams, "box", log_scale_mu=-3.0, log_scale_sigma=0.8, logit_sigma=1.5)
    opts = O.Options(tile=tile)
    g = U.run_gpu(sc, tile=tile)
    assert g["m"] > 0
    check_projection(sc, g, opts)
    check_bins(sc, g, tile)
    check_image_pinned(sc, g, opts)
    np.testing.assert_allclose(g["loss"], O.l1_loss_per_view(g["image"], sc.targets, sc.cameras), rtol=1e-5)
    orec = U.gpu_rec_to_oracle(g["rec"])
    _, dl = O.l1_loss(g["image"], sc.targets, sc.cameras)
    g2_ref, mag = O.render_backward_mag(sc.cameras, opts, orec, g["ids"], g["ranges"], dl)
    U.compare_grad2d(g["grad2d"], g2_ref, msg=f"{L.GS_MAX_VIEWS} views, tile {tile}", mag=mag)
    P = O.Params.from_scene(sc)
    U.compare_grads(g["grads"], O.project_backward(P, sc.cameras, opts, g["grad2d"]), 1e-3, "chain")


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
    U.check_image_one_flip(cams, opts, orec, g["ids"], g["ranges"], g["image"], ref, msg=f"needles, tile {tile}")
    assert np.abs(g["t_final"] - ref["t_final"])[ok].max() <= 1e-4
    assert np.array_equal(g["n_contrib"][ok], ref["n_contrib"][ok])
    _, dl = O.l1_loss(g["image"], sc.targets, cams)
    g2_ref, mag = O.render_backward_mag(cams, opts, orec, g["ids"], g["ranges"], dl)
    U.compare_grad2d(g["grad2d"], g2_ref, msg=f"needles, tile {tile}", mag=mag)


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


def _lists_of(ids, ranges, t):
    a, b = ranges[t]
    return ids[a:b]


def attribute_independent(sc, g, opts, tol=1e-4, margin=1e-2):
    """Whole FP64 pipeline (own projection, binning, sort) against the GPU.  Every pixel that differs by
    more than tol is attributed to one class of discrete decision:
      rect      its tile's list holds a different set of Gaussians, each of them one whose radius or
                rect lies at a floor/ceil boundary in the oracle's projection;
      depth     same set, another order, the reordered Gaussians' FP32 depths within 2 ulp;
      blend     the GPU differs from the oracle's render of the GPU's own lists and records by a
                one-flip alternative of a flagged decision (FP32 blending near a threshold);
      threshold same lists, and the two renders take a different alpha/transmittance decision whose
                relative distance from its threshold is below `margin` (the FP32 projection moves it);
    and `unattributed` otherwise.  Returns the counts."""
    cams = sc.cameras
    P = O.Params.from_scene(sc)
    ref = O.forward(P, cams, opts)
    idx = U.pixel_channel_index(cams)
    d = np.abs(g["image"][idx] - ref["image"][idx]).max(axis=1)
    exceed = np.nonzero(d > tol)[0]
    orec_g = U.gpu_rec_to_oracle(g["rec"])
    pinned = O.render(cams, opts, orec_g, g["ids"], g["ranges"])
    dec_g = O.pixel_decisions(cams, opts, orec_g, g["ids"], g["ranges"])
    dec_o = O.pixel_decisions(cams, opts, ref["proj"]["rec"], ref["ids"], ref["ranges"])
    boundary = (ref["proj"]["flags"] & (O.F_NEAR_RADIUS | O.F_NEAR_RECT | O.F_NEAR_PLANE)) != 0
    depth_f32 = ref["proj"]["rec"][:, 2].astype(np.float32).view(np.int32).astype(np.int64)
    # pixel -> global tile
    tile_of, B = [], opts.tile
    toff = 0
    for c in cams:
        TX, TY = (c.width + B - 1) // B, (c.height + B - 1) // B
        ys, xs = np.mgrid[0:c.height, 0:c.width]
        tile_of.append((toff + (ys // B) * TX + xs // B).reshape(-1))
        toff += TX * TY
    tile_of = np.concatenate(tile_of)
    blend_px = set()
    dp = np.abs(g["image"][idx] - pinned["image"][idx]).max(axis=1)
    pin_bad = np.nonzero(dp > tol)[0]
    if pin_bad.shape[0]:
        n_alt, alt, _ = O.render_flips(cams, opts, orec_g, g["ids"], g["ranges"], pin_bad)
        for q, p in enumerate(pin_bad):
            if n_alt[q] > 0 and np.any(np.abs(alt[q, :n_alt[q]] - g["image"][idx[p]][None]).max(axis=1) <= tol):
                blend_px.add(int(p))
    counts = dict(pixels=int(d.shape[0]), exceed=int(exceed.shape[0]), rect=0, depth=0, blend=0, threshold=0,
                  unattributed=0)
    for p in exceed:
        t = tile_of[p]
        lg, lo = _lists_of(g["ids"], g["ranges"], t), _lists_of(ref["ids"], ref["ranges"], t)
        if set(lg.tolist()) != set(lo.tolist()):
            diff = np.array(sorted(set(lg.tolist()) ^ set(lo.tolist())), np.int64)
            counts["rect" if np.all(boundary[diff]) else "unattributed"] += 1
        elif not np.array_equal(lg, lo):
            k = np.nonzero(lg != lo)[0]
            near = np.abs(depth_f32[lg[k]] - depth_f32[lo[k]]) <= 2
            counts["depth" if np.all(near) else "unattributed"] += 1
        elif int(p) in blend_px:
            counts["blend"] += 1
        elif (dec_g["blend_hash"][p] != dec_o["blend_hash"][p] or dec_g["stop_id"][p] != dec_o["stop_id"][p]) and \
                min(dec_g["margin_alpha"][p], dec_g["margin_t"][p], dec_o["margin_alpha"][p],
                    dec_o["margin_t"][p]) <= margin:
            counts["threshold"] += 1
        else:
            counts["unattributed"] += 1
    print(f"[independent] {sc.name if hasattr(sc, 'name') else ''}: {counts}, median diff {np.median(d):.2e}",
          flush=True)
    return counts, d


@pytest.mark.parametrize("case", ["render-1k", "fwdbwd-100k-small", "needles"])
def test_forward_independent_mode_attributed(case):
    """Whole FP64 pipeline (own projection, binning, sort) vs the GPU: every pixel beyond 1e-4 is
    attributed to a discrete decision class (rect boundary, depth near-tie, alpha/transmittance
    threshold), none left unattributed, and they stay rare."""
    if case == "render-1k":
        sc, tile = S.make_config(1), 16
    elif case == "fwdbwd-100k-small":
        sc, tile = S.make_config(2, n=20_000, res_div=4), 16
    else:
        cams = [S.pinhole(150, 113, 120.0), S.pinhole(97, 131, 80.0, *S.look_at((0.2, 0.3, -0.4), (0.0, 0.0, 3.0)))]
        sc, tile = S.make_scene(31, 1500, 1, cams, "box", log_scale_mu=-2.8, log_scale_sigma=1.3, logit_sigma=2.0,
                                transparent_frac=0.3), 32
    opts = O.Options(tile=tile)
    g = U.run_gpu(sc, tile=tile, backward=False)
    counts, d = attribute_independent(sc, g, opts)
    assert counts["unattributed"] == 0, counts
    assert counts["exceed"] <= 0.005 * counts["pixels"], counts
    assert np.median(d) < 1e-6


def _hand_lists(recs):
    """GPU frame of one 8x8 view (tile 8, one tile) whose list is the given records in order, records as
    (opacity, rgb, depth) with a zero conic (alpha = opacity at every pixel)."""
    import torch as T
    from paper_2409_13055_amd import rasterizer as R
    cam = S.pinhole(8, 8, 10.0)
    n = len(recs)
    rast = R.Rasterizer([cam], n, 0, tile_size=8, device="cuda", lists="tile")
    rast.reserve(n)
    fr = rast.new_frame()
    rec = np.zeros((n, 12), np.float32)
    for i, (op, rgb, depth) in enumerate(recs):
        rec[i, 0:2] = 3.5
        rec[i, 5] = op
        rec[i, 6:9] = rgb
        rec[i, 9] = depth
    fr.rec.copy_(T.as_tensor(rec.reshape(-1)))
    fr.ids[:n].copy_(T.arange(n, dtype=T.int32))
    fr.ranges.copy_(T.tensor([0, n], dtype=T.int32))
    fr.d_num_pairs.fill_(n)
    rast.render_fwd(fr)
    T.cuda.synchronize()
    orec = np.concatenate([rec[:, 0:2], rec[:, 9:10], rec[:, 2:9]], axis=1).astype(np.float64)
    return rast, fr, [cam], orec, np.arange(n, dtype=np.uint32), np.array([[0, n]], np.uint32)


@pytest.mark.parametrize("k_skip,k_after", [(0, 0), (5, 0), (7, 3)])
def test_contributor_count_is_list_position_on_gpu(k_skip, k_after):
    """The oracle's closed form for n_contrib (one blending entry behind k_skip transparent ones gives
    k_skip + 1 at every pixel) and its work counts, on the GPU through the C ABI."""
    recs = [(0.002, (1, 1, 1), 1.0 + 0.1 * i) for i in range(k_skip)] + [(0.5, (0.2, 0.4, 0.8), 3.0)] + \
           [(0.003, (1, 1, 1), 5.0 + 0.1 * i) for i in range(k_after)]
    rast, fr, cams, orec, ids, ranges = _hand_lists(recs)
    assert np.all(fr.n_contrib.cpu().numpy() == k_skip + 1)
    np.testing.assert_allclose(fr.t_final.cpu().numpy(), 0.5, rtol=1e-7)
    st = rast.render_stats(fr)
    assert st == {"evaluated": 64 * (k_skip + 1 + k_after), "blended": 64, "contrib_prefix": 64 * (k_skip + 1)}
    ref = O.render(cams, O.Options(tile=8), orec, ids, ranges)
    assert np.array_equal(fr.n_contrib.cpu().numpy(), ref["n_contrib"])


@pytest.mark.parametrize("k_skip", [0, 4])
def test_opaque_walls_stop_at_the_known_entry_on_gpu(k_skip):
    """Walls of alpha 0.95 behind k_skip transparent entries end every pixel at the fourth wall: n_contrib
    k_skip + 3, T_final 0.05^3, C = c (1 - 0.05^3), k_skip + 4 entries evaluated and 3 blended per pixel."""
    recs = [(0.001, (1, 1, 1), 0.5 + 0.1 * i) for i in range(k_skip)] + \
           [(0.95, (0.3, 0.6, 0.9), 2.0 + i) for i in range(6)]
    rast, fr, cams, orec, ids, ranges = _hand_lists(recs)
    assert np.all(fr.n_contrib.cpu().numpy() == k_skip + 3)
    np.testing.assert_allclose(fr.t_final.cpu().numpy(), 0.05 ** 3, rtol=1e-5)
    img = fr.rgb.cpu().numpy().reshape(3, -1)
    for ch, c in enumerate((0.3, 0.6, 0.9)):
        np.testing.assert_allclose(img[ch], c * (1 - 0.05 ** 3), rtol=1e-6)
    st = rast.render_stats(fr)
    assert st == {"evaluated": 64 * (k_skip + 4), "blended": 64 * 3, "contrib_prefix": 64 * (k_skip + 3)}


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


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_lds_batch_changes_no_output(tile):
    """Two splat records per lane per LDS batch (gs_options.lds_batch = 2) against one: images, final
    transmittance, contributor counts and losses bit-identical; image-space gradients, the homodirectional
    ones and the parameter gradients equal up to the order of the FP32 atomics."""
    sc = small_scene(seed=21, n=2500)
    a = U.run_gpu(sc, tile=tile, lds_batch=1, with_abs=True)
    b = U.run_gpu(sc, tile=tile, lds_batch=2, with_abs=True)
    assert a["m"] == b["m"] > 0
    for k in ("image", "t_final", "n_contrib", "loss", "ids", "ranges"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for k in ("grad2d", "abs2d"):
        assert U.rel_l2(b[k], a[k]) <= 1e-5, k
    for k in a["grads"]:
        assert U.rel_l2(b["grads"][k], a["grads"][k]) <= 1e-5, k


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


@pytest.mark.parametrize("lists", ["tile", "window"])
def test_capacity_overflow_is_reported_and_recovers(lists):
    """A capacity below the list entries (incidences, or window items) raises the overflow flag, leaves
    every tile empty (the forward renders the background) and is grown to fit by fit_capacity."""
    import torch as T
    from paper_2409_13055_amd import rasterizer as R
    sc = small_scene(seed=5, n=800)
    params = R.GaussianParams.from_scene(sc, "cuda")
    rast = R.Rasterizer(sc.cameras, params.n, params.sh_degree, device="cuda", lists=lists)
    rast.reserve(100)
    fr = rast.new_frame()
    rast.project(params, fr)
    rast.bin_sort(fr)
    rast.render_fwd(fr)
    T.cuda.synchronize()
    assert int(fr.d_overflow.item()) == 1
    assert bool((fr.rgb == 0.0).all())
    m, entries = int(fr.d_num_pairs.item()), fr.list_entries()
    assert entries > 100 and m >= entries
    assert rast.fit_capacity(fr)
    assert int(fr.d_num_pairs.item()) == m and fr.list_entries() == entries and int(fr.d_overflow.item()) == 0


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


def test_autotune_times_every_tile_and_parity_holds_at_its_choice():
    """gs_autotune (through the C ABI) times tiles 8, 16 and 32, LDS batches 1 and 2 and both forms of the
    bins on the actual problem, picks the fastest, leaves the parameters untouched and caches the choice;
    the chosen configuration passes the parity checks."""
    from paper_2409_13055_amd import autotune as A
    from paper_2409_13055_amd import rasterizer as R
    sc = small_scene(seed=17, n=3000)
    params = R.GaussianParams.from_scene(sc, "cuda")
    before = [t.clone() for t in params.tensors()]
    target = R.pack_images(sc.targets, "cuda")
    res = A.autotune_tile(params, sc.cameras, target, refresh=True)
    ms, pairs = res["ms_fwd_bwd"], res["pairs"]
    assert not res["from_cache"] and all(v > 0 for v in ms.values()), res
    assert set(ms) == {f"{t}/{b}/{f}" for t in (8, 16, 32) for b in (1, 2) for f in ("tile", "window")}, res
    assert f"{res['best']}/{res['lds_batch']}/{res['lists']}" == min(ms, key=ms.get)
    assert pairs[8] >= pairs[16] >= pairs[32] > 0  # a finer grid lists a splat in at least as many tiles
    for a, b in zip(before, params.tensors()):
        assert torch.equal(a, b)
    again = A.autotune_tile(params, sc.cameras, target)
    assert again["from_cache"] and (again["best"], again["lds_batch"], again["lists"]) == \
        (res["best"], res["lds_batch"], res["lists"])
    only = A.autotune_tile(params, sc.cameras, target, candidates=(16,), batches=(2,), refresh=True, lists="window")
    assert set(only["ms_fwd_bwd"]) == {"16/2/window"} and (only["best"], only["lds_batch"], only["lists"]) == \
        (16, 2, "window")
    tile = res["best"]
    opts = O.Options(tile=tile)
    g = U.run_gpu(sc, tile=tile, lds_batch=res["lds_batch"], lists=res["lists"])
    check_bins(sc, g, tile)
    check_image_pinned(sc, g, opts)
    orec = U.gpu_rec_to_oracle(g["rec"])
    _, dl = O.l1_loss(g["image"], sc.targets, sc.cameras)
    U.compare_grad2d(g["grad2d"], O.render_backward(sc.cameras, opts, orec, g["ids"], g["ranges"], dl),
                     msg=f"autotuned tile {tile}")


# --- window lists (GS_OPT_WINDOW_LISTS): the bins as each 8 x 8-tile window's list ----------------------

def _windows_scene(multi_pass):
    if multi_pass:
        # 2 views of 150 x 85 tiles at tile 8: 418 windows, so the window sort takes two 8-bit passes
        cams = [S.pinhole(1200, 680, 900.0), S.pinhole(1200, 680, 800.0, *S.look_at((0.3, -0.1, -0.5),
                                                                                  (0.0, 0.0, 3.0)))]
        return S.make_scene(61, 6000, 1, cams, "box", log_scale_mu=-2.6, log_scale_sigma=0.7, logit_sigma=1.5)
    return small_scene(seed=62, n=3000)


@pytest.mark.parametrize("tile,multi_pass", [(8, False), (16, False), (32, False), (8, True)])
def test_window_lists_stand_for_the_tile_lists(tile, multi_pass):
    """The window-list form against the tile-list form on the same scene: the tile lists the window lists
    stand for equal the tile lists bit for bit (and so the oracle's binning, which the tile form matches);
    images, final transmittance, contributor counts, losses and work counts equal; gradients equal up to
    the order of the FP32 atomics."""
    sc = _windows_scene(multi_pass)
    a = U.run_gpu(sc, tile=tile, lists="tile", with_abs=True)
    b = U.run_gpu(sc, tile=tile, lists="window", with_abs=True)
    assert a["m"] == b["m"] > 0
    n_win = b["win_ranges"].shape[1]
    assert (n_win > 256) == multi_pass
    assert b["items"].shape[0] == int(b["win_ranges"][1].max())
    for k in ("ids", "ranges", "image", "t_final", "n_contrib", "loss"):
        np.testing.assert_array_equal(b[k], a[k], err_msg=k)
    for k in ("grad2d", "abs2d"):
        assert U.rel_l2(b[k], a[k]) <= 1e-5, k
    # the image-space gradients differ only in the order of their FP32 atomics (above); the chain to the
    # parameters sums views and cancels (the rotation gradients most), which can amplify that tenfold
    for k in a["grads"]:
        assert U.rel_l2(b["grads"][k], a["grads"][k]) <= 1e-4, k
    assert a["rast"].render_stats(a["frame"]) == b["rast"].render_stats(b["frame"])
    check_bins(sc, b, tile)


def _hand_window_frames(recs0, recs1, lds_batch):
    """One 16 x 8 view at tile 8: two tiles in one binning window.  Tile 0's list is recs0 and tile 1's is
    recs1 (records as (opacity, rgb, depth) with a zero conic: alpha = opacity at every pixel), as tile
    lists and as one window list that interleaves them; returns {form: (rasteriser, frame)}."""
    import torch as T
    from paper_2409_13055_amd import rasterizer as R
    cam = S.pinhole(16, 8, 10.0)
    recs = list(recs0) + list(recs1)
    n, n0 = len(recs), len(recs0)
    rec = np.zeros((n, 12), np.float32)
    for i, (op, rgb, depth) in enumerate(recs):
        rec[i, 0:2] = (3.5 if i < n0 else 11.5, 3.5)
        rec[i, 5] = op
        rec[i, 6:9] = rgb
        rec[i, 9] = depth
    code0, code1 = 0 | 1 << 4 | 0 << 8 | 1 << 12, 1 | 2 << 4 | 0 << 8 | 1 << 12
    items = []
    for k in range(max(n0, n - n0)):
        if k < n0:
            items.append((k, code0))
        if k < n - n0:
            items.append((n0 + k, code1))
    out = {}
    for form in ("tile", "window"):
        rast = R.Rasterizer([cam], n, 0, tile_size=8, device="cuda", lists=form, lds_batch=lds_batch)
        rast.reserve(n)
        fr = rast.new_frame()
        fr.rec.copy_(T.as_tensor(rec.reshape(-1)))
        if form == "tile":
            fr.ids[:n].copy_(T.arange(n, dtype=T.int32))
            fr.ranges.copy_(T.tensor([0, n0, n0, n], dtype=T.int32))
        else:
            it = np.array(items, np.uint32).reshape(-1)
            fr.items[:n].copy_(T.as_tensor(it.view(np.int64)))
            fr.win_ranges.copy_(T.tensor([0, n], dtype=T.int32))
            fr.d_num_items.fill_(n)
        fr.d_num_pairs.fill_(n)
        rast.render_fwd(fr)
        out[form] = (rast, fr)
    T.cuda.synchronize()
    return out


@pytest.mark.parametrize("lds_batch", [1, 2])
@pytest.mark.parametrize("k_skip", [0, 5, 70, 150])
def test_window_list_positions_are_tile_list_positions(k_skip, lds_batch):
    """n_contrib counts positions in the tile's own list when the entries come from a window list that
    interleaves another tile's: one blending entry behind k_skip transparent ones gives k_skip + 1 at every
    pixel of tile 0, also when the entries span several LDS batches (64 or 128 entries at tile 8); the
    image, transmittance and work counts equal those of the tile lists."""
    recs0 = [(0.002, (1, 1, 1), 1.0 + 0.01 * i) for i in range(k_skip)] + [(0.5, (0.2, 0.4, 0.8), 3.0)] + \
            [(0.003, (1, 1, 1), 5.0 + 0.01 * i) for i in range(3)]
    recs1 = [(0.004, (0.5, 0.5, 0.5), 1.0 + 0.01 * i) for i in range(k_skip + 9)] + [(0.6, (0.9, 0.1, 0.1), 4.0)]
    fr = _hand_window_frames(recs0, recs1, lds_batch)
    (ra, fa), (rb, fb) = fr["tile"], fr["window"]
    nc = fb.n_contrib.cpu().numpy().reshape(8, 16)
    assert np.all(nc[:, :8] == k_skip + 1) and np.all(nc[:, 8:] == k_skip + 10)
    assert torch.equal(fa.n_contrib, fb.n_contrib) and torch.equal(fa.t_final, fb.t_final)
    assert torch.equal(fa.rgb, fb.rgb)
    assert ra.render_stats(fa) == rb.render_stats(fb)
