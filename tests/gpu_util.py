"""Helpers shared by the GPU parity tests: run the HIP path on a scene and
convert its outputs for the oracle (test infrastructure)."""
import numpy as np
import torch

import oracle.oracle as O
from paper_2409_13055_amd import rasterizer as R

DEV = "cuda"


def gpu_extents(rec):
    """Tile rect half-extents (rx, ry) [VN,2] from GPU record word 10 (rx | ry << 16; 0 = culled)."""
    w = np.ascontiguousarray(np.asarray(rec, np.float32)[:, 10]).view(np.int32)
    return np.stack([w & 0xffff, w >> 16], axis=1).astype(np.int32)


def gpu_rec_to_oracle(rec):
    """GPU record [VN,12] (mx,my,ca,cb,cc,op,r,g,b,depth,extents,flags) -> oracle [VN,10] FP64."""
    rec = np.asarray(rec, np.float32)
    return np.concatenate([rec[:, 0:2], rec[:, 9:10], rec[:, 2:9]], axis=1).astype(np.float64)


def run_gpu(sc, tile=16, checkpoint=False, backward=True, want_keys=True, capacity=None, cams=None,
            external_dl=None):
    """Forward (+ L1 backward) of `sc` on the GPU; returns numpy outputs."""
    cams = sc.cameras if cams is None else cams
    params = R.GaussianParams.from_scene(sc, DEV)
    rast = R.Rasterizer(cams, params.n, params.sh_degree, tile_size=tile, checkpoint=checkpoint, device=DEV,
                        want_keys=want_keys)
    if capacity is not None:
        rast.reserve(capacity)
    target = R.pack_images(sc.targets, DEV) if sc.targets is not None else None
    loss = torch.zeros(len(cams), device=DEV)
    fr = rast.forward(params, target=target, loss_out=loss if target is not None else None)
    out = dict(params=params, rast=rast, frame=fr)
    if backward:
        grads = params.zeros_like()
        if external_dl is not None:
            rast.render_bwd(params, fr, grads, dl_dimage=torch.as_tensor(external_dl, dtype=torch.float32,
                                                                          device=DEV))
        else:
            rast.render_bwd(params, fr, grads, target=target)
        torch.cuda.synchronize()
        out["grad2d"] = rast.grad2d.cpu().numpy().astype(np.float64)
        out["grads"] = {k: getattr(grads, k).cpu().numpy().astype(np.float64) for k in R.PARAM_NAMES}
    torch.cuda.synchronize()
    m = int(fr.d_num_pairs.item())
    out["m"] = m
    out["rec"] = fr.rec.view(-1, 12).cpu().numpy()
    out["tiles"] = fr.tiles.cpu().numpy()
    out["ids"] = fr.ids[:m].cpu().numpy().view(np.uint32)
    out["keys"] = fr.keys[:m].cpu().numpy().view(np.uint64) if fr.keys is not None else None
    out["ranges"] = fr.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    out["image"] = fr.rgb.cpu().numpy().astype(np.float64)
    if fr.t_final is not None:
        out["t_final"] = fr.t_final.cpu().numpy().astype(np.float64)
        out["n_contrib"] = fr.n_contrib.cpu().numpy()
    out["loss"] = loss.cpu().numpy().astype(np.float64)
    return out


def oracle_grads_sh(g):
    """Split the oracle's [N,K,3] SH gradient into (dc, rest) like the GPU layout."""
    return g["sh"][:, 0, :], g["sh"][:, 1:, :]


def rel_l2(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def compare_grads(gpu_grads, ref, tol, msg=""):
    dc, rest = oracle_grads_sh(ref)
    pairs = [("means", ref["means"]), ("log_scales", ref["log_scales"]), ("quats", ref["quats"]),
             ("opacity_logits", ref["opacity_logits"]), ("sh_dc", dc)]
    if rest.shape[1] > 0:
        pairs.append(("sh_rest", rest))
    out = {}
    for k, r in pairs:
        out[k] = rel_l2(gpu_grads[k], r)
    bad = {k: v for k, v in out.items() if not v <= tol}
    assert not bad, f"{msg} gradient rel-L2 above {tol}: {bad} (all: {out})"
    return out
