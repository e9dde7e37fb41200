"""The training-system patterns around the rasteriser, on the GPU:

- the torch.autograd.Function (dL/dimage from a loss written in torch) against
  the oracle's analytic gradient and central finite differences;
- the 100k-Gaussian SH-3 workload: the fused L1 gradients of every parameter
  of a 200-Gaussian sample against central finite differences of the oracle;
- HIP-graph replays of the batched iteration against eager execution;
- the projection backward fused with Adam against the two separate calls.
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

PER_PARAM = [("means", 3), ("log_scales", 3), ("quats", 4), ("opacity_logits", 1)]


def gpu_grad_at(grads, g, p, K):
    """GPU gradient of raw parameter index p (oracle order) of Gaussian g."""
    if p < 11:
        for name, a, b in O.PARAM_SLICES:
            if a <= p < b:
                return grads[name].reshape(grads[name].shape[0], -1)[g, p - a]
    k, ch = divmod(p - 11, 3)
    if k == 0:
        return grads["sh_dc"][g, ch]
    return grads["sh_rest"][g, k - 1, ch]


def fd_compare(sc, gpu_grads, gidx, tol, msg=""):
    """Central FD of the oracle's L1 loss vs the GPU gradient, per parameter group (rel L2)."""
    P = O.Params.from_scene(sc)
    K = (sc.sh_degree + 1) ** 2
    npar = 11 + 3 * K
    gg = np.repeat(gidx, npar)
    pp = np.tile(np.arange(npar), len(gidx))
    fd, st = O.fd_local(P, sc.cameras, sc.targets, O.Options(tile=16), gg, pp)
    ok = st < 2
    assert ok.mean() > 0.9, np.bincount(st)
    got = np.array([gpu_grad_at(gpu_grads, g, p, K) for g, p in zip(gg, pp)])
    groups = {"means": (0, 3), "log_scales": (3, 6), "quats": (6, 10), "opacity": (10, 11), "sh": (11, npar)}
    out = {}
    for name, (a, b) in groups.items():
        m = ok & (pp >= a) & (pp < b)
        out[name] = U.rel_l2(got[m], fd[m])
    print(f"[fd] {msg}: kept {ok.mean():.3f} of {ok.shape[0]} samples; rel-L2 per group {out}", flush=True)
    bad = {k: v for k, v in out.items() if not v <= tol}
    assert not bad, out
    return out


def test_autograd_function_matches_oracle_and_fd():
    cams = [S.pinhole(96, 72, 80.0), S.pinhole(80, 64, 70.0, *S.look_at((0.3, 0.1, -0.4), (0.0, 0.0, 3.0)))]
    sc = S.make_scene(12, 500, 2, cams, "box", log_scale_mu=-3.0, log_scale_sigma=0.5, logit_sigma=1.5)
    params = R.GaussianParams.from_scene(sc, "cuda")
    rast = R.Rasterizer(cams, params.n, params.sh_degree, device="cuda")
    leaves = [t.clone().requires_grad_(True) for t in params.tensors()]
    img = R.render(rast, *leaves)
    target = R.pack_images(sc.targets, "cuda")
    # the L1 term of the photometric loss written in torch; the rasteriser only sees dL/dimage
    loss = 0
    off = 0
    for c in cams:
        k = 3 * c.width * c.height
        loss = loss + (img[off:off + k] - target[off:off + k]).abs().mean()
        off += k
    loss.backward()
    grads = {k: t.grad.detach().cpu().numpy().astype(np.float64) for k, t in zip(R.PARAM_NAMES, leaves)}
    P = O.Params.from_scene(sc)
    ref = O.forward_backward_l1(P, cams, sc.targets, O.Options(tile=16))
    assert abs(loss.item() - ref["loss"]) <= 1e-5 * ref["loss"]
    U.compare_grads(grads, ref["grads"], 1e-3, "autograd vs oracle")
    vis = np.nonzero(ref["proj"]["radius"].reshape(len(cams), -1).max(axis=0) > 0)[0]
    gidx = np.random.default_rng(0).choice(vis, 25, replace=False)
    fd_compare(sc, grads, gidx, 1e-3, "autograd")


@pytest.mark.slow
def test_fused_l1_gradients_match_fd_on_200_gaussians_100k():
    """Workload with 100k Gaussians, SH degree 3, 640x480: gradients of means, scales, quaternions,
    opacity and SH of a seeded 200-Gaussian visible subset against central finite differences."""
    sc = S.make_config(2)
    g = U.run_gpu(sc)
    vis = np.nonzero(U.gpu_extents(g["rec"])[:, 0] > 0)[0]
    gidx = np.random.default_rng(200).choice(vis, 200, replace=False)
    fd_compare(sc, g["grads"], gidx, 1e-3, "100k SH3, 200 Gaussians")


@pytest.mark.parametrize("lists", ["window", "tile"])
def test_graph_replays_match_eager(lists):
    sc = S.make_config(3, n=40_000, res_div=4)
    params = R.GaussianParams.from_scene(sc, "cuda")
    step = R.MappingStep(params, sc.cameras, sc.targets, tile_size=16, with_adam=False, lists=lists)
    step.size()
    step.run()
    torch.cuda.synchronize()
    fr = step.frame
    lists_of = (lambda: (fr.items[:int(fr.d_num_items.item())], fr.win_ranges)) if fr.windowed else \
        (lambda: (fr.ids[:int(fr.d_num_pairs.item())], fr.ranges))
    ref_img = step.frame.rgb.clone()
    ref_ids, ref_ranges = (t.clone() for t in lists_of())
    ref_loss = step.loss.clone()
    ref_grads = [t.clone() for t in step.grads.tensors()]
    for t in step.grads.tensors():
        t.zero_()
    step.capture()  # runs the step once eagerly on the capture stream, then records it
    torch.cuda.synchronize()
    for r in range(1, 5):
        step.frame.rgb.fill_(-1.0)
        step.replay()
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * x).sum().item()
        torch.cuda.synchronize()
        assert torch.equal(step.frame.rgb, ref_img), r
        ids, ranges = lists_of()
        assert torch.equal(ids, ref_ids), r
        assert torch.equal(ranges, ref_ranges), r
        assert torch.equal(step.loss, ref_loss), r
        # gradients accumulate: capture warm-up + r replays
        for a, b in zip(step.grads.tensors(), ref_grads):
            assert U.rel_l2(a.cpu().numpy(), (r + 1) * b.cpu().numpy()) <= 1e-5, r


def test_graph_replays_with_adam_advance_the_step():
    sc = S.make_config(3, n=20_000, res_div=4)
    p_eager = R.GaussianParams.from_scene(sc, "cuda")
    p_graph = R.GaussianParams.from_scene(sc, "cuda")
    a = R.MappingStep(p_eager, sc.cameras, sc.targets, lrs=dict(S.DEFAULT_LRS), tile_size=16)
    b = R.MappingStep(p_graph, sc.cameras, sc.targets, lrs=dict(S.DEFAULT_LRS), tile_size=16)
    a.size()
    b.size()
    b.capture()  # one eager step
    a.run()
    for _ in range(3):
        a.run()
        b.replay()
        torch.cuda.synchronize()
        la, lb = a.loss.cpu().numpy(), b.loss.cpu().numpy()
        np.testing.assert_allclose(lb, la, rtol=1e-4)
    assert int(a.adam.d_step.item()) == int(b.adam.d_step.item()) == 4
    for ta, tb in zip(p_eager.tensors(), p_graph.tensors()):
        # FP32 atomics make the summation order differ between runs, and Adam normalises the
        # step (a near-zero gradient can flip sign), so compare the bulk, not every element
        d = (ta - tb).abs()
        assert (d > 1e-4).float().mean().item() < 0.01
        assert d.median().item() < 1e-6


def test_gradient_buffer_cleared_on_side_stream_before_the_backward():
    """The fused step clears the image-space gradient buffer on a second stream while the forward
    runs.  After every graph replay (and an eager step) the buffer must hold exactly this
    iteration's raster backward: recomputed from the same frame into a freshly zeroed buffer."""
    sc = S.make_config(3, n=20_000, res_div=4)
    p = R.GaussianParams.from_scene(sc, "cuda")
    step = R.MappingStep(p, sc.cameras, sc.targets, lrs=dict(S.DEFAULT_LRS), tile_size=16)
    step.size()
    target = R.pack_images(sc.targets, "cuda")
    step.capture()
    for r in range(4):
        if r == 3:
            step.run()
        else:
            step.replay()
        x = torch.randn(1 << 20, device="cuda")  # eager work between iterations
        _ = (x * x).sum().item()
        torch.cuda.synchronize()
        got = step.rast.grad2d.clone()
        ref = torch.zeros_like(got)
        step.rast.raster_bwd(step.frame, ref, target=target)
        torch.cuda.synchronize()
        assert ref.abs().sum().item() > 0
        assert U.rel_l2(got.cpu().numpy(), ref.cpu().numpy()) <= 1e-5, r


def test_fused_projection_backward_adam_equals_separate_calls():
    """gs_project_bwd_adam is gs_project_bwd into zeroed gradients then gs_adam_step, bit for bit, fed
    the same image-space gradients (two steps, so the bias corrections of t = 1 and t = 2 both enter)."""
    sc = S.make_config(3, n=20_000, res_div=4)
    p_sep = R.GaussianParams.from_scene(sc, "cuda")
    p_fus = R.GaussianParams.from_scene(sc, "cuda")
    lrs = dict(S.DEFAULT_LRS)
    rast = R.Rasterizer(sc.cameras, p_sep.n, p_sep.sh_degree, tile_size=16, device="cuda")
    target = R.pack_images(sc.targets, "cuda")
    grads = p_sep.zeros_like()
    adam_sep = R.FusedAdam(p_sep, grads, lrs)
    adam_fus = R.FusedAdam(p_fus, p_fus.zeros_like(), lrs)
    fr = rast.new_frame()
    for it in range(2):
        # one frame of the separate path's parameters; both paths take its image-space gradients
        rast.project(p_sep, fr)
        rast.bin_sort(fr)
        rast.fit_capacity(fr)
        rast.render_fwd(fr)
        g2 = torch.zeros(rast.n_views * p_sep.n, 9, device="cuda")
        rast.raster_bwd(fr, g2, target=target)
        rast.project_bwd(p_sep, fr, g2, grads)
        adam_sep.step(zero_grad=True)
        rast.project_bwd_adam(p_fus, fr, g2, adam_fus)
        torch.cuda.synchronize()
        assert g2.abs().sum().item() > 0
        for name, a, b in zip(R.PARAM_NAMES, p_sep.tensors(), p_fus.tensors()):
            assert torch.equal(a, b), (it, name)
        for name, a, b in zip(R.PARAM_NAMES, adam_sep.exp_avg.tensors(), adam_fus.exp_avg.tensors()):
            assert torch.equal(a, b), (it, "m", name)
        for name, a, b in zip(R.PARAM_NAMES, adam_sep.exp_avg_sq.tensors(), adam_fus.exp_avg_sq.tensors()):
            assert torch.equal(a, b), (it, "v", name)
        assert all(t.abs().sum().item() == 0 for t in grads.tensors())
    assert int(adam_sep.d_step.item()) == int(adam_fus.d_step.item()) == 2
