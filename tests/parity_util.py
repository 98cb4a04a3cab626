"""Shared steps of the parity procedure between the HIP path and the oracle.

Discrete decisions that FP32 cannot reproduce exactly (a pair within 1e-5 r^2
of the footprint cutoff, a depth within 2^-40 of a float32 rounding midpoint)
flag rays.  The rays both sides score are the complement of the union of the
oracle's flags and the GPU's own (gs_params.ambiguous_rays).  For unmasked
runs (plans take no ray mask), Gaussians touched by a flagged ray are left
out of the element-wise comparison; every other Gaussian's sensitivity comes
from unflagged rays only and must meet the bar.
"""
import numpy as np

import synth


def mask_tensor(bits):
    import torch
    return torch.as_tensor(np.ascontiguousarray(bits, np.uint32).view(np.int32)).cuda()


def gpu_flags(gs, dsc, vw, **kw):
    """Rays the GPU flags (a pair within 1e-5 r^2 of the cutoff), as bools."""
    import torch
    words = (vw.n_rays + 31) // 32
    amb = torch.zeros(words, dtype=torch.int32, device="cuda")
    _, st = gs.sensitivity(dsc, vw, stats=True, count_pairs=True, ambiguous_rays=amb, **kw)
    torch.cuda.synchronize()
    flags = synth.unpack_bits(amb.cpu().numpy().view(np.uint32), vw.n_rays)
    return flags, st


def union_mask(gs, ora, sc, vw, dsc=None, ora_params=None, **kw):
    """(bits of the rays to score, oracle flags, GPU flags)."""
    if dsc is None:
        dsc = gs.DeviceScene.from_scene(sc)
    ref_all = ora.sensitivity(sc, vw, ora_params)
    g, _ = gpu_flags(gs, dsc, vw, **kw)
    flag = ref_all["flag"] | g
    return synth.pack_bits(~flag), ref_all["flag"], g


def touched_by_flagged(ora, sc, vw, flag, r=3.0, params=None):
    """Gaussians whose footprint (d^2 <= r^2 (1 + 1e-4)) holds the centre of
    some flagged ray: their unmasked sensitivity may come from such a ray."""
    pr = ora.project(sc, vw, params)
    touched = np.zeros(sc.n, bool)
    base = 0
    for v in range(vw.n_views):
        W, H = int(vw.size[v, 0]), int(vw.size[v, 1])
        rays = np.nonzero(flag[base:base + W * H])[0]
        base += W * H
        if rays.size == 0:
            continue
        pres = pr["present"][v]
        m2 = pr["mean2d"][v][pres]
        cn = pr["conic"][v][pres]
        ids = np.nonzero(pres)[0]
        for ray in rays:
            ux, uy = ray % W + 0.5, ray // W + 0.5
            dx, dy = ux - m2[:, 0], uy - m2[:, 1]
            d2 = cn[:, 0] * dx * dx + 2.0 * cn[:, 1] * dx * dy + cn[:, 2] * dy * dy
            touched[ids[d2 <= r * r * (1.0 + 1e-4)]] = True
    return touched


def compare_unmasked(s_gpu, ref, touched, rel=1e-5, abs_=1e-12):
    """Element-wise bar on the Gaussians no flagged ray touches; returns the
    worst excess and the count compared."""
    s = np.asarray(s_gpu, np.float64)
    keep = ~touched
    excess = np.abs(s[keep] - ref[keep]) - (rel * ref[keep] + abs_)
    return (float(excess.max()) if keep.any() else -1.0), int(keep.sum())
