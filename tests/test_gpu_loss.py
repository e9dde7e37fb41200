"""The photometric loss of eq. (2) with its SSIM term (gs_photometric_loss) against the FP64 oracle.

Tolerances: per-view losses relative 2e-5 (FP32 window sums of values in [0, 1]); dL/dimage relative
1e-4 in L2 and 1e-3 of its largest entry at every element (on smooth, low-variance images the FP32
variances E[x^2] - mu^2 lose digits against C2 = 9e-4, so those get 1e-3 in L2).
"""
import numpy as np
import pytest

from paper_2409_13055_amd import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle.oracle as O  # noqa: E402
from paper_2409_13055_amd import rasterizer as R  # noqa: E402
from tests import gpu_util as U  # noqa: E402

DEV = "cuda"


def run_loss(cams, img_flat, targets, lam):
    pl = R.PhotometricLoss(cams, device=DEV)
    img = torch.as_tensor(np.asarray(img_flat, np.float32), device=DEV)
    tgt = R.pack_images(targets, DEV)
    loss = torch.zeros(len(cams), device=DEV)
    dl = torch.zeros_like(img)
    pl(img, tgt, lam, loss, dl)
    torch.cuda.synchronize()
    return loss.cpu().numpy().astype(np.float64), dl.cpu().numpy().astype(np.float64)


def f32_images(cams, rng, smooth=False):
    out = []
    for c in cams:
        if smooth:
            yy, xx = np.mgrid[0:c.height, 0:c.width]
            base = 0.5 + 0.3 * np.sin(xx / 17.0) * np.cos(yy / 23.0)
            out.append(np.stack([base + 0.01 * k + 0.002 * rng.standard_normal(base.shape) for k in range(3)]))
        else:
            out.append(rng.random((3, c.height, c.width)))
    return [np.asarray(np.clip(a, 0, 1), np.float32) for a in out]


def compare(cams, img_views, tgt_views, lam, l2_tol=1e-4):
    img_flat = O.pack_views(img_views)
    loss_g, dl_g = run_loss(cams, img_flat, tgt_views, lam)
    loss_o, dl_o = O.photometric_loss(img_flat.astype(np.float64), tgt_views, cams, lam)
    np.testing.assert_allclose(loss_g, loss_o, rtol=2e-5)
    assert U.rel_l2(dl_g, dl_o) <= l2_tol, U.rel_l2(dl_g, dl_o)
    assert np.abs(dl_g - dl_o).max() <= 1e-3 * np.abs(dl_o).max()
    return loss_g, dl_g


@pytest.mark.parametrize("lam", [1.0, 0.2])
def test_photometric_loss_matches_oracle_ragged_tiles(lam):
    # view sizes that leave ragged 16 x 64 tiles and windows reaching past every border
    cams = [S.pinhole(130, 97, 110.0), S.pinhole(70, 45, 60.0), S.pinhole(11, 7, 9.0)]
    rng = np.random.default_rng(31)
    compare(cams, f32_images(cams, rng), f32_images(cams, rng), lam)


def test_photometric_loss_on_smooth_images():
    cams = [S.pinhole(200, 150, 150.0)]
    rng = np.random.default_rng(5)
    tgt = f32_images(cams, rng, smooth=True)
    img = [np.asarray(np.clip(t + 0.02 * rng.standard_normal(t.shape), 0, 1), np.float32) for t in tgt]
    compare(cams, img, tgt, 0.2, l2_tol=1e-3)


def test_photometric_loss_full_size_views():
    # two keyframes of the 16-view 1200 x 680 workload, rendered-like images against random targets
    cams = S.make_config(5).cameras[:2]
    rng = np.random.default_rng(9)
    compare(cams, f32_images(cams, rng), f32_images(cams, rng), 0.2)


def test_lambda_zero_is_the_fused_l1_term():
    sc = S.make_scene(4, 3000, 1, [S.pinhole(96, 80, 90.0), S.pinhole(64, 48, 60.0)], "box",
                      log_scale_mu=-3.0)
    g = U.run_gpu(sc, tile=16, backward=False)
    loss_g, dl_g = run_loss(sc.cameras, g["image"], sc.targets, 0.0)
    np.testing.assert_allclose(loss_g, g["loss"], rtol=1e-6)
    _, dl_ref = O.l1_loss(g["image"], sc.targets, sc.cameras)
    np.testing.assert_allclose(dl_g, dl_ref, rtol=1e-6, atol=0)


def test_ssim_gradient_through_the_raster_backward():
    """Image-space gradients driven by the SSIM loss's dL/dimage, against the oracle's backward fed
    with the oracle's gradient of the same loss (pinned lists and records)."""
    cams = [S.pinhole(130, 97, 110.0), S.pinhole(100, 76, 90.0, *S.look_at((0.35, -0.1, -0.5), (0.0, 0.0, 3.0)))]
    sc = S.make_scene(3, 2000, 3, cams, "box", log_scale_mu=-3.3, log_scale_sigma=0.6, logit_sigma=1.5)
    g = U.run_gpu(sc, tile=16, backward=False)
    rast, fr = g["rast"], g["frame"]
    lam = 0.2
    pl = R.PhotometricLoss(cams, device=DEV)
    dl = torch.zeros_like(fr.rgb)
    pl(fr.rgb, R.pack_images(sc.targets, DEV), lam, None, dl)
    g2 = torch.zeros(rast.n_views * rast.n, 9, device=DEV)
    rast.raster_bwd(fr, g2, dl_dimage=dl)
    torch.cuda.synchronize()
    _, dl_o = O.photometric_loss(g["image"], sc.targets, cams, lam)
    ref = O.render_backward(cams, O.Options(tile=16), U.gpu_rec_to_oracle(g["rec"]), g["ids"], g["ranges"], dl_o)
    got = g2.cpu().numpy().astype(np.float64)
    U.compare_grad2d(got, ref, msg="SSIM dL/dimage through the raster backward")


def test_mapping_step_with_ssim_graph_replays_match_eager():
    sc = S.make_config(3, n=20_000, res_div=4)
    pa = R.GaussianParams.from_scene(sc, DEV)
    pb = R.GaussianParams.from_scene(sc, DEV)
    a = R.MappingStep(pa, sc.cameras, sc.targets, lrs=dict(S.DEFAULT_LRS), tile_size=16, ssim_lambda=0.2)
    b = R.MappingStep(pb, sc.cameras, sc.targets, lrs=dict(S.DEFAULT_LRS), tile_size=16, ssim_lambda=0.2)
    a.size()
    b.size()
    b.capture()  # one eager step
    a.run()
    for _ in range(3):
        a.run()
        b.replay()
        x = torch.randn(1 << 20, device=DEV)  # eager work between replays
        _ = (x * x).sum().item()
        torch.cuda.synchronize()
        np.testing.assert_allclose(b.loss.cpu().numpy(), a.loss.cpu().numpy(), rtol=1e-4)
    # the loss is eq. (2) of the step's own image (checked against the oracle on the last frame)
    ref, _ = O.photometric_loss(b.frame.rgb.cpu().numpy().astype(np.float64), sc.targets, sc.cameras, 0.2)
    b.photometric(b.frame.rgb, b.target, 0.2, b.loss, None)
    torch.cuda.synchronize()
    np.testing.assert_allclose(b.loss.cpu().numpy(), ref, rtol=2e-5)
