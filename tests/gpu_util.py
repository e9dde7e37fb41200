"""Helpers shared by the GPU parity tests: run the HIP path on a scene and
convert its outputs for the oracle (test infrastructure)."""
import numpy as np
import torch

import oracle.oracle as O
from paper_2409_13055_amd import rasterizer as R

DEV = "cuda"


def _spread3(v):
    v = v.astype(np.uint64) & 0x3FF
    out = np.zeros_like(v)
    for b in range(10):
        out |= ((v >> b) & 1) << (3 * b)
    return out


def morton_codes(means):
    """The codes gs_spatial_order sorts by, written out in FP32 like the device: per axis the cell
    min(1023, floor((m - lo) * (1024 / (hi - lo)))) over the means' box (a flat axis and a NaN give
    0), bits interleaved x, y, z from bit 0."""
    m = np.asarray(means, np.float32)
    lo, hi = np.nanmin(m, axis=0), np.nanmax(m, axis=0)
    ext = (hi - lo).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(ext > 0, np.float32(1024) / ext, np.float32(0)).astype(np.float32)
        q = np.floor(((m - lo).astype(np.float32) * scale).astype(np.float32))
        cell = np.where(q >= 0, np.minimum(q, 1023), 0).astype(np.uint64)
    return _spread3(cell[:, 0]) | (_spread3(cell[:, 1]) << 1) | (_spread3(cell[:, 2]) << 2)


def morton_order_reference(means):
    """The permutation gs_spatial_order defines: a stable sort of morton_codes."""
    return np.argsort(morton_codes(means), kind="stable")


def gpu_extents(rec):
    """Tile rect half-extents (rx, ry) [VN,2] from GPU record word 10 (rx | ry << 16; 0 = culled)."""
    w = np.ascontiguousarray(np.asarray(rec, np.float32)[:, 10]).view(np.int32)
    return np.stack([w & 0xffff, w >> 16], axis=1).astype(np.int32)


def gpu_rec_to_oracle(rec):
    """GPU record [VN,12] (mx,my,ca,cb,cc,op,r,g,b,depth,extents,flags) -> oracle [VN,10] FP64."""
    rec = np.asarray(rec, np.float32)
    return np.concatenate([rec[:, 0:2], rec[:, 9:10], rec[:, 2:9]], axis=1).astype(np.float64)


def window_tile_lists(items, win_ranges, cams, tile):
    """The tile lists (ids, ranges) that window lists stand for, as gs_bins defines them: tile
    (tx, ty) takes, in window order, the items of its window whose clipped rect covers
    (tx mod 8, ty mod 8).  Also checks every item's clipped rect is a non-empty part of its window."""
    items = np.asarray(items, np.uint32).reshape(-1, 2)
    wr = np.asarray(win_ranges, np.uint32).reshape(2, -1)
    lists, t_off, w_off = [], 0, 0
    for c in cams:
        TX, TY = -(-c.width // tile), -(-c.height // tile)
        WX, WY = -(-TX // 8), -(-TY // 8)
        per_tile = [None] * (TX * TY)
        for wy in range(WY):
            for wx in range(WX):
                w = w_off + wy * WX + wx
                b, e = int(wr[0, w]), int(wr[1, w])
                assert b <= e
                code = items[b:e, 1]
                x0, x1, y0, y1 = code & 15, (code >> 4) & 15, (code >> 8) & 15, (code >> 12) & 15
                assert np.all((x0 < x1) & (x1 <= 8) & (y0 < y1) & (y1 <= 8) & (code >> 16 == 0))
                assert np.all(x1 <= TX - 8 * wx) and np.all(y1 <= TY - 8 * wy)
                for ly in range(min(8, TY - 8 * wy)):
                    for lx in range(min(8, TX - 8 * wx)):
                        sel = (x0 <= lx) & (lx < x1) & (y0 <= ly) & (ly < y1)
                        per_tile[(8 * wy + ly) * TX + 8 * wx + lx] = items[b:e, 0][sel]
        lists += per_tile
        t_off += TX * TY
        w_off += WX * WY
    assert w_off == wr.shape[1]
    lens = np.array([len(x) for x in lists], np.int64)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    ranges = np.stack([starts, starts + lens], 1)
    ranges[lens == 0] = 0
    ids = np.concatenate(lists) if lists else np.zeros(0, np.uint32)
    return ids.astype(np.uint32), ranges.astype(np.uint32)


def window_tile_list(items, win_ranges, cams, tile, t):
    """The tile list of global tile t that window lists stand for (see window_tile_lists)."""
    items = np.asarray(items, np.uint32).reshape(-1, 2)
    wr = np.asarray(win_ranges, np.uint32).reshape(2, -1)
    t_off = w_off = 0
    for c in cams:
        TX, TY = -(-c.width // tile), -(-c.height // tile)
        WX, WY = -(-TX // 8), -(-TY // 8)
        if t < t_off + TX * TY:
            ty, tx = divmod(t - t_off, TX)
            w = w_off + (ty // 8) * WX + tx // 8
            b, e = int(wr[0, w]), int(wr[1, w])
            code = items[b:e, 1]
            lx, ly = tx % 8, ty % 8
            sel = ((code & 15) <= lx) & (lx < ((code >> 4) & 15)) & (((code >> 8) & 15) <= ly) & \
                (ly < ((code >> 12) & 15))
            return items[b:e, 0][sel]
        t_off += TX * TY
        w_off += WX * WY
    raise IndexError(t)


def run_gpu(sc, tile=16, checkpoint=False, backward=True, want_keys=True, capacity=None, cams=None,
            external_dl=None, lds_batch=1, with_abs=False, lists="window"):
    """Forward (+ L1 backward) of `sc` on the GPU; returns numpy outputs.  with_abs: also the raster
    backward with the homodirectional gradient (gs_raster_bwd_abs) into out["abs2d"].  lists: the form
    of the bins; window lists are returned as they are ("items", "win_ranges") and as the tile lists
    they stand for ("ids", "ranges"); the sort keys (want_keys) come with tile lists only."""
    cams = sc.cameras if cams is None else cams
    params = R.GaussianParams.from_scene(sc, DEV)
    rast = R.Rasterizer(cams, params.n, params.sh_degree, tile_size=tile, checkpoint=checkpoint, device=DEV,
                        want_keys=want_keys and lists == "tile", lds_batch=lds_batch, lists=lists)
    if capacity is not None:
        rast.reserve(capacity)
    target = R.pack_images(sc.targets, DEV) if sc.targets is not None else None
    loss = torch.zeros(len(cams), device=DEV)
    # gs_project leaves the records of culled pairs unwritten and nothing may read them: NaN there
    # would reach every output that did
    fr = rast.new_frame()
    fr.rec.fill_(float("nan"))
    fr = rast.forward(params, fr, target=target, loss_out=loss if target is not None else None)
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
        if with_abs:
            g2 = torch.zeros(len(cams) * params.n, 9, dtype=torch.float32, device=DEV)
            a2 = torch.zeros(len(cams) * params.n, 2, dtype=torch.float32, device=DEV)
            rast.raster_bwd(fr, g2, target=target, abs2d=a2)
            torch.cuda.synchronize()
            out["abs2d"] = a2.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    m = int(fr.d_num_pairs.item())
    out["m"] = m
    out["tiles"] = fr.tiles.cpu().numpy()
    rec = fr.rec.view(-1, 12).cpu().numpy()
    rec[out["tiles"] == 0] = 0.0  # culled pairs' rows are unwritten: read them as zero (extents 0)
    out["rec"] = rec
    if fr.windowed:
        n_items = int(fr.d_num_items.item())
        out["items"] = fr.items[:n_items].cpu().numpy().view(np.uint32).reshape(-1, 2)
        out["win_ranges"] = fr.win_ranges.cpu().numpy().view(np.uint32).reshape(2, -1)
        out["ids"], out["ranges"] = window_tile_lists(out["items"], out["win_ranges"], cams, tile)
        assert out["ids"].shape[0] == m
        out["keys"] = None
    else:
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


# Element-wise gradient bound: |gpu - oracle| <= REL |oracle| + KAPPA mag + FLOOR max|oracle|, where mag
# is the sum over pixels of the magnitudes of the per-pixel terms the gradient adds up (the oracle gives
# it).  A sum of terms that cancel can only be as accurate as the terms: an FP32 term carries a relative
# error of order 1e-6 (1e-5 for elongated splats, whose exponent is a difference of large quantities),
# so KAPPA = 1e-4 leaves a factor of ten over the worst of them.
REL, KAPPA, FLOOR = 1e-3, 1e-4, 1e-6


def elementwise_frac(a, b, rel=REL, floor=FLOOR, mag=None, kappa=KAPPA):
    """Fraction of elements with |a - b| <= rel |b| + kappa mag + floor max|b| (b the oracle's value;
    mag as above, or none)."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    if b.size == 0:
        return 1.0
    bound = rel * np.abs(b) + floor * np.abs(b).max()
    if mag is not None:
        bound = bound + kappa * np.asarray(mag, np.float64).reshape(-1)
    return float(np.mean(np.abs(a - b) <= bound))


def compare_grads(gpu_grads, ref, tol, msg="", min_frac=0.999):
    """Per tensor: relative L2 error <= tol, and the element-wise bound (elementwise_frac) met by at
    least min_frac of the elements.  Returns {name: (rel_l2, frac)}."""
    dc, rest = oracle_grads_sh(ref)
    pairs = [("means", ref["means"]), ("log_scales", ref["log_scales"]), ("quats", ref["quats"]),
             ("opacity_logits", ref["opacity_logits"]), ("sh_dc", dc)]
    if rest.shape[1] > 0:
        pairs.append(("sh_rest", rest))
    out = {}
    for k, r in pairs:
        out[k] = (rel_l2(gpu_grads[k], r), elementwise_frac(gpu_grads[k], r))
    print(f"[grads] {msg}: " + ", ".join(f"{k} rel {v[0]:.2e} elem {v[1]:.5f}" for k, v in out.items()), flush=True)
    bad = {k: v for k, v in out.items() if not (v[0] <= tol and v[1] >= min_frac)}
    assert not bad, f"{msg} gradient above rel-L2 {tol} or element-wise fraction below {min_frac}: {bad} (all: {out})"
    return out


def compare_grad2d(got, ref, tol=1e-3, msg="", min_frac=0.999, mag=None):
    """Image-space gradients [rows, C] per component: relative L2 <= tol and the element-wise bound
    (elementwise_frac, with the oracle's per-term magnitudes when given) for at least min_frac of the
    rows."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    out = [(rel_l2(got[:, c], ref[:, c]),
            elementwise_frac(got[:, c], ref[:, c], mag=None if mag is None else mag[:, c]))
           for c in range(ref.shape[1])]
    print(f"[grad2d] {msg}: rel " + " ".join(f"{r:.1e}" for r, _ in out) + " | elem "
          + " ".join(f"{f:.5f}" for _, f in out) + ("" if mag is None else " (with term magnitudes)"), flush=True)
    bad = [(c, v) for c, v in enumerate(out) if not (v[0] <= tol and v[1] >= min_frac)]
    for c, _ in bad:  # the worst elements of a failing component
        b = np.abs(ref[:, c])
        bound = REL * b + FLOOR * b.max() + (0.0 if mag is None else KAPPA * mag[:, c])
        r = np.abs(got[:, c] - ref[:, c]) / np.maximum(bound, 1e-300)
        for k in np.argsort(-r)[:4]:
            print(f"  component {c} row {k}: gpu {got[k, c]:.6e} oracle {ref[k, c]:.6e} "
                  f"mag {(0.0 if mag is None else mag[k, c]):.3e} |d|/bound {r[k]:.2f}", flush=True)
    assert not bad, f"{msg} image-space gradient components above rel-L2 {tol} / below {min_frac}: {bad}"
    return out


def pixel_channel_index(cams):
    """[P, 3] index of each pixel's three channels in the packed planar image (views packed)."""
    parts, off = [], 0
    for c in cams:
        hw = c.width * c.height
        base = off + np.arange(hw)
        parts.append(np.stack([base, base + hw, base + 2 * hw], axis=1))
        off += 3 * hw
    return np.concatenate(parts)


def check_image_one_flip(cams, opts, orec, ids, ranges, img_gpu, ref, pixels=None, tol=1e-4, msg=""):
    """Every pixel (or every listed pixel) of the GPU image within tol of the oracle's render on the same
    lists and records, or, where a decision lies within the FP32 rounding bound of its threshold
    (flagged), within tol of that render with one such decision taken the other way.  Returns counts."""
    idx = pixel_channel_index(cams)
    P = idx.shape[0]
    sel = np.arange(P) if pixels is None else np.asarray(pixels, np.int64)
    d = np.abs(np.asarray(img_gpu, np.float64)[idx[sel]] - ref["image"][idx[sel]]).max(axis=1)
    flagged = ref["pix_flags"][sel] != 0
    bad = ~(d <= tol)
    unflagged_bad = bad & ~flagged
    assert not unflagged_bad.any(), (f"{msg}: {int(unflagged_bad.sum())} unflagged pixels differ by more than {tol} "
                                     f"(max {d[unflagged_bad].max():.3e})")
    fb = sel[bad]
    explained = 0
    if fb.shape[0]:
        n_alt, alt, _ = O.render_flips(cams, opts, orec, ids, ranges, fb)
        g = np.asarray(img_gpu, np.float64)[idx[fb]]
        da = np.abs(alt - g[:, None, :]).max(axis=2)  # [pixels, alternatives]
        ok = np.array([(n_alt[q] > 0) and bool(np.any(da[q, :n_alt[q]] <= tol)) for q in range(fb.shape[0])])
        explained = int(ok.sum())
        assert ok.all(), (f"{msg}: {int((~ok).sum())} flagged pixels differ by more than {tol} from the oracle and from "
                          f"every one-flip alternative")
    st = dict(pixels=int(sel.shape[0]), flagged=int(flagged.sum()), flagged_frac=float(flagged.mean()),
              differing=int(bad.sum()), explained_by_one_flip=explained, max_abs_unflagged=float(d[~flagged].max(initial=0)))
    print(f"[image] {msg}: {st}", flush=True)
    return st


def gpu_flips(cams, opts, orec, ids, ranges, img_gpu, ref, pixels, nc_gpu=None, tf_gpu=None):
    """The decisions the GPU took the other way, for the oracle's backward to take them the GPU's way:
    - where the GPU's contributor count or final transmittance (nc_gpu, tf_gpu, per pixel; optional)
      differs from the oracle's (the transmittance by more than 1e-3 relative: a blended entry changes
      it by at least 1/255), the single decision that gives the oracle both (or_find_flips), nearest
      the GPU's colour;
    - at other flagged pixels, the one-flip alternative closest to the GPU's colour, when the GPU's
      colour is off the oracle's own by more than FP32 noise (1e-6) and at most half as far from the
      alternative.
    Returns ((pixels, list positions, kinds), number of pixels whose count no single flip explains)."""
    idx = pixel_channel_index(cams)
    pixels = np.asarray(pixels, np.int64)
    img_gpu = np.asarray(img_gpu, np.float64)
    chosen = {}
    unexplained = 0
    if nc_gpu is not None:
        nc_gpu, tf_gpu = np.asarray(nc_gpu), np.asarray(tf_gpu, np.float64)
        differ = (nc_gpu[pixels] != ref["n_contrib"][pixels]) | \
                 (np.abs(tf_gpu[pixels] - ref["t_final"][pixels]) > 1e-3 * ref["t_final"][pixels])
        mism = pixels[differ]
        if mism.shape[0]:
            found, ks, kinds = O.find_flips(cams, opts, orec, ids, ranges, mism, nc_gpu[mism], tf_gpu[mism],
                                            img_gpu[idx[mism]])
            for q, p in enumerate(mism):
                if found[q] == 1:
                    chosen[int(p)] = (int(ks[q]), int(kinds[q]))
            unexplained = int((found < 0).sum())
    fl = np.array([p for p in pixels[ref["pix_flags"][pixels] != 0] if int(p) not in chosen], np.int64)
    if fl.shape[0]:
        n_alt, alt, kinds, ks = O.render_flips(cams, opts, orec, ids, ranges, fl, with_positions=True)
        g = img_gpu[idx[fl]]
        d0 = np.abs(g - ref["image"][idx[fl]]).max(axis=1)
        da = np.abs(alt - g[:, None, :]).max(axis=2)
        for q in range(fl.shape[0]):
            if n_alt[q] <= 0:
                continue
            a = int(np.argmin(da[q, :n_alt[q]]))
            if d0[q] > 1e-6 and da[q, a] < 0.5 * d0[q]:
                chosen[int(fl[q])] = (int(ks[q, a]), int(kinds[q, a]))
    px = np.array(sorted(chosen), np.int64)
    out = (px, np.array([chosen[int(p)][0] for p in px], np.int32), np.array([chosen[int(p)][1] for p in px], np.uint32))
    return out, unexplained
