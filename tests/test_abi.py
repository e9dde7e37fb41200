"""The C ABI library on the CPU: it loads, exports every function include/gs.h
declares, and its host-only entry points (queries, option defaults, argument
validation) behave as documented.  No call here launches GPU work: validation
rejects the arguments before anything would be enqueued."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2409_13055_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2409_13055_amd import build
        build.build()
    _lib.load()
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(gs_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 16, names
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.EXPORTS) == set(names)


def test_defaults_and_queries(L):
    from paper_2409_13055_amd import synthetic as S
    o = L.default_options()
    assert o.tile_size == 16 and o.checkpoint == 0 and o.flags == 0 and o.lds_batch == 1
    assert L.load().gs_abi_version() == L.GS_ABI_VERSION == 4
    assert abs(o.alpha_min - 1 / 255) < 1e-9 and abs(o.alpha_max - 0.99) < 1e-7 and abs(o.t_min - 1e-4) < 1e-10
    assert abs(o.near_plane - 0.2) < 1e-7 and abs(o.eps2d - 0.3) < 1e-7 and o.radius_sigmas == 3.0
    cams = [S.pinhole(1200, 680, 600.0), S.pinhole(640, 480, 525.0), S.pinhole(100, 75, 90.0)]
    cc = L.make_cameras(cams)
    for B in (8, 16, 32):
        exp = sum(((c.width + B - 1) // B) * ((c.height + B - 1) // B) for c in cams)
        assert L.gs_total_tiles(cc, 3, B) == exp
    assert L.gs_total_pixels(cc, 3) == sum(c.width * c.height for c in cams)
    for B in (8, 16, 32):  # binning windows: 8 x 8 tiles of one view
        exp = sum(-(-((c.width + B - 1) // B) // 8) * -(-((c.height + B - 1) // B) // 8) for c in cams)
        assert L.gs_total_windows(cc, 3, B) == exp
    assert L.gs_total_windows(L.make_cameras([S.pinhole(1, 1, 1.0)]), 1, 32) == 1
    assert C.sizeof(L.gs_bins) == 9 * 8  # seven pointers and the int64 capacity, as gs.h lays them out
    assert L.gs_render_bwd_workspace_size(1000, 3) >= 1000 * 3 * 9 * 4
    assert L.gs_render_fwd_workspace_size(cc, 3, o) >= 4 * L.gs_total_tiles(cc, 3, 16)
    a = L.gs_bin_sort_workspace_size(1000, cc, 3, o, 10_000)
    b = L.gs_bin_sort_workspace_size(1000, cc, 3, o, 100_000)
    assert b > a > 0


def test_invalid_arguments_are_rejected_before_any_launch(L):
    from paper_2409_13055_amd import synthetic as S
    o = L.default_options()
    cc = L.make_cameras([S.pinhole(64, 48, 50.0)])
    with pytest.raises(L.GsError, match="UNSUPPORTED"):
        L.gs_total_tiles(cc, 1, 12)
    with pytest.raises(L.GsError, match="n_views"):
        L.gs_total_pixels(cc, 0)
    with pytest.raises(L.GsError, match="pair_capacity"):
        L.gs_bin_sort_workspace_size(10, cc, 1, o, 1 << 33)
    bad = L.default_options(alpha_min=0.5, alpha_max=0.4)
    with pytest.raises(L.GsError, match="alpha"):
        L.gs_render_fwd_workspace_size(cc, 1, bad)
    for batch in (0, 3):
        with pytest.raises(L.GsError, match="lds_batch"):
            L.gs_render_fwd_workspace_size(cc, 1, L.default_options(lds_batch=batch))
    # hot-path calls with NULL device pointers fail validation (nothing is enqueued)
    params = L.gs_params()
    params.n, params.sh_degree = 10, 0
    out = L.gs_projected()
    with pytest.raises(L.GsError, match="INVALID_VALUE"):
        L.gs_project(params, cc, 1, o, out, None)
    params.sh_degree = 5
    with pytest.raises(L.GsError, match="sh_degree"):
        L.gs_project(params, cc, 1, o, out, None)
    # the projection's visible-pair segments are required by the projection and the bin sort
    params.sh_degree = 0
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh_dc"):
        setattr(params, k, C.c_void_p(0x1000))
    out.rec, out.tiles_touched = C.c_void_p(0x1000), C.c_void_p(0x2000)
    with pytest.raises(L.GsError, match="vis"):
        L.gs_project(params, cc, 1, o, out, None)
    with pytest.raises(L.GsError, match="proj is incomplete"):
        L.gs_bin_sort(out, 10, cc, 1, o, L.gs_bins(), None, 0, None)
    out.vis, out.vis_count = C.c_void_p(0x3008), C.c_void_p(0x4000)
    with pytest.raises(L.GsError, match="vis must be 16-byte aligned"):
        L.gs_bin_sort(out, 10, cc, 1, o, L.gs_bins(), None, 0, None)
    # the two forms of the bins need their own buffers; unknown option bits are rejected
    out.vis = C.c_void_p(0x3000)
    bins = L.gs_bins()
    bins.d_num_pairs, bins.d_overflow = C.c_void_p(0x5000), C.c_void_p(0x5100)
    bins.items, bins.win_ranges = C.c_void_p(0x6000), C.c_void_p(0x7000)
    with pytest.raises(L.GsError, match="tile lists need"):
        L.gs_bin_sort(out, 10, cc, 1, o, bins, None, 0, None)
    ow = L.default_options()
    ow.flags = L.GS_OPT_WINDOW_LISTS
    bins.items = C.c_void_p(0x6004)
    with pytest.raises(L.GsError, match="8-byte aligned"):
        L.gs_bin_sort(out, 10, cc, 1, ow, bins, None, 0, None)
    bins.items, bins.win_ranges = C.c_void_p(0x6000), None
    with pytest.raises(L.GsError, match="window lists need"):
        L.gs_bin_sort(out, 10, cc, 1, ow, bins, None, 0, None)
    with pytest.raises(L.GsError, match="items/win_ranges"):
        L.gs_render_fwd(out, 10, bins, cc, 1, ow, None, L.gs_image(), None, 0, None)
    bins.win_ranges = C.c_void_p(0x7000)
    with pytest.raises(L.GsError, match="CAPACITY"):  # a workspace is still required
        L.gs_bin_sort(out, 10, cc, 1, ow, bins, None, 0, None)
    ow.flags = 2
    with pytest.raises(L.GsError, match="flags"):
        L.gs_bin_sort(out, 10, cc, 1, ow, bins, None, 0, None)
    groups = (L.gs_adam_group * 1)()
    groups[0].numel = 4
    with pytest.raises(L.GsError, match="NULL"):
        L.gs_adam_step(groups, 1, 0.9, 0.999, 1e-15, C.c_void_p(16), 0, None)
    with pytest.raises(L.GsError, match="beta"):
        L.gs_adam_step(groups, 1, 1.5, 0.999, 1e-15, C.c_void_p(16), 0, None)
    # the fused projection backward + Adam checks its groups against the parameter arrays
    fp = L.gs_params()
    fp.n, fp.sh_degree = 10, 0
    fp.means, fp.log_scales, fp.quats = C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000)
    fp.opacity_logits, fp.sh_dc = C.c_void_p(0x4000), C.c_void_p(0x5000)
    fproj = L.gs_projected()
    fproj.tiles_touched = C.c_void_p(0x6000)
    six = (L.gs_adam_group * 6)()
    for k, (addr, width) in enumerate([(0x1000, 3), (0x2000, 3), (0x3000, 4), (0x4000, 1), (0x5000, 3), (0, 0)]):
        six[k].param, six[k].numel, six[k].lr = C.c_void_p(addr or None), 10 * width, 1e-3
        if width:
            six[k].exp_avg, six[k].exp_avg_sq = C.c_void_p(0x8000), C.c_void_p(0x9000)
    six[2].numel = 39
    with pytest.raises(L.GsError, match="numel"):
        L.gs_project_bwd_adam(fp, fproj, cc, 1, o, C.c_void_p(0x7000), six, 0.9, 0.999, 1e-15, C.c_void_p(16), None)
    six[2].numel = 40
    six[1].param = C.c_void_p(0x2100)
    with pytest.raises(L.GsError, match="params array"):
        L.gs_project_bwd_adam(fp, fproj, cc, 1, o, C.c_void_p(0x7000), six, 0.9, 0.999, 1e-15, C.c_void_p(16), None)
    # the photometric loss validates its arguments before enqueuing anything
    c2 = L.make_cameras([S.pinhole(64, 48, 50.0), S.pinhole(30, 20, 20.0)])
    wsb = L.gs_photometric_loss_workspace_size(c2, 2)
    assert wsb >= 36 * (64 * 48 + 30 * 20)
    img, tgt, dl, lo = C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000), C.c_void_p(0x4000)
    with pytest.raises(L.GsError, match="image and target"):
        L.gs_photometric_loss(c2, 2, None, tgt, 0.2, lo, dl, C.c_void_p(0x5000), wsb, None)
    with pytest.raises(L.GsError, match="lambda"):
        L.gs_photometric_loss(c2, 2, img, tgt, 1.5, lo, dl, C.c_void_p(0x5000), wsb, None)
    with pytest.raises(L.GsError, match="nothing to compute"):
        L.gs_photometric_loss(c2, 2, img, tgt, 0.2, None, None, C.c_void_p(0x5000), wsb, None)
    with pytest.raises(L.GsError, match="CAPACITY"):
        L.gs_photometric_loss(c2, 2, img, tgt, 0.2, lo, dl, C.c_void_p(0x5000), wsb - 1, None)
    lib = L.load()
    assert lib.gs_status_string(3) == b"GS_ERR_CAPACITY"
    assert b"workspace too small" in lib.gs_last_error()


def test_pyramid_camera_host_arithmetic_and_reduce_validation(L, oracle_lib):
    """gs_pyramid_camera is host arithmetic (no device work): it equals the oracle's level camera.
    gs_pyramid_reduce rejects bad arguments before enqueuing anything."""
    from paper_2409_13055_amd import synthetic as S
    O = oracle_lib
    cam = S.pinhole(1201, 679, 600.0, *S.look_at((0.3, -0.2, -0.7), (0.0, 0.1, 2.0)))
    cam.cx, cam.cy = 601.75, 338.5
    cc = L.make_cameras([cam])
    for levels in range(5):
        got = L.gs_pyramid_camera(cc[0], levels)
        ref = O.pyramid_camera(cam, levels)
        assert (got.width, got.height) == (ref.width, ref.height)
        for k in ("fx", "fy", "cx", "cy"):
            assert abs(getattr(got, k) - getattr(ref, k)) <= 1e-7 * abs(getattr(ref, k)), (levels, k)
        assert list(got.R) == list(cc[0].R) and list(got.t) == list(cc[0].t)
    with pytest.raises(L.GsError, match="levels"):
        L.gs_pyramid_camera(cc[0], -1)
    with pytest.raises(L.GsError, match="levels"):
        L.gs_pyramid_camera(cc[0], 16)
    c2 = L.make_cameras([S.pinhole(64, 48, 50.0), S.pinhole(31, 21, 20.0)])
    n_src = 3 * (64 * 48 + 31 * 21)
    with pytest.raises(L.GsError, match="src and dst"):
        L.gs_pyramid_reduce(c2, 2, None, C.c_void_p(0x100000), None)
    with pytest.raises(L.GsError, match="overlap"):
        L.gs_pyramid_reduce(c2, 2, C.c_void_p(0x100000), C.c_void_p(0x100000 + 4 * n_src - 4), None)
    with pytest.raises(L.GsError, match="n_views"):
        L.gs_pyramid_reduce(c2, 0, C.c_void_p(0x100000), C.c_void_p(0x900000), None)


def test_density_control_host_entry_points(L, oracle_lib):
    """Defaults, the scene extent (host arithmetic, against the oracle) and argument validation of
    the density-control calls; nothing is launched."""
    from paper_2409_13055_amd import synthetic as S
    O = oracle_lib
    c = L.default_density_config()
    assert (c.grad_threshold, c.percent_dense, c.min_opacity, c.split_scale_div, c.extent) == pytest.approx(
        (0.0002, 0.01, 0.005, 1.6, 1.0), rel=1e-7)
    cams = S.make_config(5, n=10).cameras
    ext = L.gs_scene_extent(L.make_cameras(cams), len(cams))
    assert ext == pytest.approx(O.scene_extent(cams), rel=1e-6)
    assert L.gs_density_workspace_size(1000) >= 1000 + 2 * 3 * 4 * 4
    p = L.gs_params()
    p.n, p.sh_degree = 1000, 0
    p.means, p.log_scales, p.quats = C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000)
    p.opacity_logits, p.sh_dc = C.c_void_p(0x4000), C.c_void_p(0x5000)
    st = L.gs_density_stats(C.c_void_p(0x6000), C.c_void_p(0x7000), C.c_void_p(0x8000))
    wsb = L.gs_density_workspace_size(1000)
    ws, cnt = C.c_void_p(0x100000), C.c_void_p(0x9000)
    with pytest.raises(L.GsError, match="statistics"):
        L.gs_density_plan(p, L.gs_density_stats(), c, cnt, ws, wsb, None)
    with pytest.raises(L.GsError, match="min_opacity"):
        L.gs_density_plan(p, st, L.default_density_config(min_opacity=1.0), cnt, ws, wsb, None)
    with pytest.raises(L.GsError, match="extent"):
        L.gs_density_plan(p, st, L.default_density_config(extent=0.0), cnt, ws, wsb, None)
    with pytest.raises(L.GsError, match="CAPACITY"):
        L.gs_density_plan(p, st, c, cnt, ws, wsb - 1, None)
    m = L.gs_params()
    m.n, m.sh_degree = 999, 0
    m.means, m.log_scales, m.quats = C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000)
    m.opacity_logits, m.sh_dc = C.c_void_p(0x4000), C.c_void_p(0x5000)
    out = L.gs_grads()
    with pytest.raises(L.GsError, match="moments"):
        L.gs_density_apply(p, m, m, c, None, 0, 10, out, out, out, ws, wsb, None)
    with pytest.raises(L.GsError, match="n_out"):
        L.gs_density_apply(p, p, p, c, None, 0, 3001, out, out, out, ws, wsb, None)
    with pytest.raises(L.GsError, match="eps"):
        L.gs_density_apply(p, p, p, c, None, 6, 10, out, out, out, ws, wsb, None)
    with pytest.raises(L.GsError, match="out_params"):
        L.gs_density_apply(p, p, p, c, None, 0, 10, out, out, out, ws, wsb, None)
    cc = L.make_cameras([S.pinhole(64, 48, 50.0)])
    proj = L.gs_projected()
    with pytest.raises(L.GsError, match="tiles_touched"):
        L.gs_density_accumulate(proj, 1000, cc, 1, C.c_void_p(0x1000), C.c_void_p(0x2000), st, None)


def test_delaunay_host_triangulation_matches_qhull(L, oracle_lib):
    """gs_delaunay is host code: its triangles equal scipy's Qhull on points in general position,
    and on integer grids (cocircular quadruples) both are valid Delaunay triangulations."""
    import numpy as np
    O = oracle_lib
    rng = np.random.default_rng(17)
    for n, W, H in [(3, 10, 10), (12, 30, 20), (300, 1200, 680), (2000, 1200, 680)]:
        flat = rng.choice(W * H, n, replace=False)
        pts = np.stack([flat % W, flat // W], 1)
        got = L.gs_delaunay(pts)
        ref = O.delaunay_triangles(pts)
        same = np.array_equal(np.unique(np.sort(got, 1), axis=0), ref)
        if not same:  # a cocircular quadruple: check validity instead
            assert len(got) == len(ref)
            P = [tuple(int(v) for v in p) for p in pts]
            for i, j, k in got:
                assert O._orient(P[i], P[j], P[k]) > 0
                for m in rng.choice(n, min(n, 200), replace=False):
                    if m not in (i, j, k):
                        assert _incircle_exact(P[i], P[j], P[k], P[m]) <= 0
        # canonical form: smallest index first, positive orientation, sorted
        assert np.all(got[:, 0] < got[:, 1]) and np.all(got[:, 0] < got[:, 2])
        assert [tuple(t) for t in got] == sorted(tuple(t) for t in got)
    grid = np.array([(x, y) for y in range(0, 20, 4) for x in range(0, 24, 4)])
    got = L.gs_delaunay(grid)
    assert len(got) == 2 * (6 - 1) * (5 - 1)  # a grid of squares: two triangles each
    with pytest.raises(L.GsError, match="distinct"):
        L.gs_delaunay(np.array([[1, 1], [2, 5], [1, 1], [7, 3]]))
    with pytest.raises(L.GsError, match="collinear"):
        L.gs_delaunay(np.array([[0, 0], [1, 1], [2, 2], [5, 5]]))
    with pytest.raises(L.GsError, match="outside"):
        L.gs_delaunay(np.array([[0, 0], [40000, 1], [2, 9]]))


def _incircle_exact(a, b, c, d):
    rows = [(p[0] - d[0], p[1] - d[1]) for p in (a, b, c)]
    m = [(x, y, x * x + y * y) for x, y in rows]
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def gs_offset(struct, field):
    return getattr(type(struct), field).offset


def test_autotune_validates_before_any_launch(L):
    """gs_autotune (host-side, synchronising) rejects bad arguments before touching the device."""
    from paper_2409_13055_amd import synthetic as S
    o = L.default_options()
    cc = L.make_cameras([S.pinhole(64, 48, 50.0)])
    params = L.gs_params()
    params.n, params.sh_degree = 10, 0
    for k, a in zip(("means", "log_scales", "quats", "opacity_logits", "sh_dc"), (0x1000, 0x2000, 0x3000, 0x4000,
                                                                                 0x5000)):
        setattr(params, k, C.c_void_p(a))
    with pytest.raises(L.GsError, match="target is required"):
        L.gs_autotune(params, cc, 1, o, None, 3, 0, 0, None)
    with pytest.raises(L.GsError, match="iters"):
        L.gs_autotune(params, cc, 1, o, C.c_void_p(0x6000), 0, 0, 0, None)
    for mask in (128, -1):
        with pytest.raises(L.GsError, match="candidate_mask"):
            L.gs_autotune(params, cc, 1, o, C.c_void_p(0x6000), 3, mask, 0, None)
    params.sh_degree = 4
    with pytest.raises(L.GsError, match="sh_degree"):
        L.gs_autotune(params, cc, 1, o, C.c_void_p(0x6000), 3, 0, 0, None)
    r = L.gs_autotune_result()
    # int32 x (5 + 3 x 12), float x 12, then int64 x 12 at the next 8-byte boundary: the layout gs.h declares
    assert L.GS_AUTOTUNE_MAX_CANDIDATES == 12
    assert C.sizeof(r) == 216 + 8 * 12 and gs_offset(r, "pairs") == 216


def test_layout_calls_validate_before_any_launch(L):
    """gs_spatial_order and gs_gather_rows reject bad arguments before touching the device."""
    assert L.gs_spatial_order_workspace_size(1000) >= 4 * 4 * 1000
    with pytest.raises(L.GsError, match="n must be"):
        L.gs_spatial_order_workspace_size(0)
    ws = L.gs_spatial_order_workspace_size(10)
    with pytest.raises(L.GsError, match="required"):
        L.gs_spatial_order(None, 10, C.c_void_p(0x1000), C.c_void_p(0x2000), ws, None)
    with pytest.raises(L.GsError, match="workspace too small"):
        L.gs_spatial_order(C.c_void_p(0x1000), 10, C.c_void_p(0x2000), C.c_void_p(0x3000), ws - 1, None)
    with pytest.raises(L.GsError, match="must not be the same"):
        L.gs_gather_rows(C.c_void_p(0x1000), 10, 3, C.c_void_p(0x2000), C.c_void_p(0x1000), None)
    with pytest.raises(L.GsError, match="width"):
        L.gs_gather_rows(C.c_void_p(0x1000), 10, 0, C.c_void_p(0x2000), C.c_void_p(0x3000), None)


def test_noalloc_forward_validates_before_any_launch(L):
    """gs_render_fwd_noalloc rejects bad arguments before touching the device, as gs_render_fwd does."""
    from paper_2409_13055_amd import synthetic as S
    o = L.default_options()
    cc = L.make_cameras([S.pinhole(64, 48, 50.0)])
    proj = L.gs_projected()
    with pytest.raises(L.GsError, match="rec"):
        L.gs_render_fwd_noalloc(proj, 10, L.gs_bins(), cc, 1, o, None, L.gs_image(), None)
    assert L.GS_NOALLOC_MAX_TILES == 1 << 20
