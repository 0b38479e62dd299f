"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle on the same seeded scene.

Parity bar (FP32 kernel vs FP64 oracle):
  * primary hit ids bit-exact on every pixel whose decision margin is at
    least GRAZING (1e-6, relative);
  * colour within COLOUR_TOL (1e-4 absolute) on every non-grazing pixel that
    the oracle's jittered re-traces classify as well conditioned;
  * two ceilings per case, so that a classifier that excluded more pixels, or
    a kernel that drifted on the pixels it does not check, cannot pass
    silently: the share of pixels classified ill conditioned (max_ill), and
    the share of all non-grazing pixels off by more than COLOUR_TOL
    (max_mismatch, the mismatch fraction the colour bar reports).
"""

from __future__ import annotations

import os
import re
import sys

import numpy as np
import torch

GRAZING = 1e-6
COLOUR_TOL = 1e-4

# Default ceilings for small scenes; full-size workloads pass their own.
MAX_ILL = 0.10
MAX_MISMATCH = 0.005


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def record_stats(stats):
    """Appends one parity result as a JSON line to the file named by
    RT_PARITY_LOG (nothing when it is unset), so that a run of the GPU suite
    leaves every case's mismatch and exclusion fractions in one place."""
    path = os.environ.get("RT_PARITY_LOG")
    if path:
        import json
        with open(path, "a") as f:
            f.write(json.dumps(stats) + "\n")


def gpu_render(rt, scene, cam, W, H, D, records=False, sky=None):
    h = rt.SceneHandle(scene)
    try:
        if sky is not None:
            rt.rt_scene_set_sky(h.handle, sky)
        rgb, ids, rec = rt.render(h.handle, cam, W, H, D, ids=True, records=records)
        torch.cuda.synchronize()
        out = dict(rgb=rgb.cpu().numpy().reshape(-1, 3).astype(np.float64),
                   ids=ids.cpu().numpy().reshape(-1))
        if records:
            out["seg_id"] = rec.ids.cpu().numpy().reshape(D + 1, -1).T
            out["lit"] = rec.lit.cpu().numpy().reshape(D + 1, -1).T.astype(np.uint32)
        return out
    finally:
        h.close()


def compare(oracle, scene, cam, W, H, D, gpu, pixels=None, label="", samples=1,
            light_radius=0.0, sky=None, max_ill=MAX_ILL, max_mismatch=MAX_MISMATCH):
    """Returns a stats dict; raises AssertionError when the parity bar fails.
    samples > 1 compares soft shadows of lights of radius light_radius; `sky`
    is the skybox [h, w, 3] both sides render with."""
    base = oracle.render(scene, cam, W, H, D, pixels, samples=samples, light_radius=light_radius,
                         sky=sky)
    ok_cond = oracle.condition(scene, cam, W, H, D, pixels, base=base, samples=samples,
                               light_radius=light_radius, sky=sky)
    sel = base.pixels
    g_rgb = gpu["rgb"][sel]
    g_ids = gpu["ids"][sel]
    nongrazing = base.margin >= GRAZING
    id_bad = (g_ids != base.prim_id) & nongrazing
    err = np.abs(g_rgb - base.rgb).max(1)
    col_bad_all = (err > COLOUR_TOL) & nongrazing
    checked = nongrazing & ok_cond
    col_bad = (err > COLOUR_TOL) & checked
    stats = dict(label=label, pixels=int(sel.size), grazing=float((~nongrazing).mean()),
                 ill_conditioned=float((~ok_cond).mean()),
                 id_mismatch_nongrazing=int(id_bad.sum()),
                 id_mismatch_all=int((g_ids != base.prim_id).sum()),
                 colour_mismatch_frac_nongrazing=float(col_bad_all.sum() / max(nongrazing.sum(), 1)),
                 colour_mismatch_checked=int(col_bad.sum()),
                 max_err_checked=float(err[checked].max()) if checked.any() else 0.0,
                 max_err_all=float(err.max()) if err.size else 0.0)
    log("parity", stats)
    record_stats(dict(stats, max_ill=max_ill, max_mismatch=max_mismatch))
    if id_bad.any() or col_bad.any():
        _dump(label, sel, base, gpu, err, nongrazing, ok_cond)
    assert not id_bad.any(), f"{label}: {int(id_bad.sum())} non-grazing primary id mismatches"
    assert not col_bad.any(), (f"{label}: {int(col_bad.sum())} well-conditioned pixels off by "
                               f"> {COLOUR_TOL}; max {err[checked].max():.3g}")
    assert stats["ill_conditioned"] <= max_ill, (
        f"{label}: {stats['ill_conditioned']:.4f} of pixels ill conditioned, ceiling {max_ill}")
    assert stats["colour_mismatch_frac_nongrazing"] <= max_mismatch, (
        f"{label}: {stats['colour_mismatch_frac_nongrazing']:.5f} of non-grazing pixels off by "
        f"> {COLOUR_TOL}, ceiling {max_mismatch}")
    if "seg_id" in gpu:
        robust = checked
        assert np.array_equal(gpu["seg_id"][sel][robust], base.seg_id[robust]), "segment ids"
        assert np.array_equal(gpu["lit"][sel][robust], base.lit[robust]), "lit masks"
    return stats, base


def _dump(label, sel, base, gpu, err, nongrazing, ok_cond):
    """Save the mismatching pixels (both sides) for offline analysis."""
    out = os.path.join(os.environ.get("GRAFT_REPO_ROOT", "."), "gpurun_out")
    os.makedirs(out, exist_ok=True)
    bad = np.where(((err > COLOUR_TOL) | (gpu["ids"][sel] != base.prim_id)))[0]
    worst = bad[np.argsort(-err[bad])][:200]
    extra = {}
    if "seg_id" in gpu:
        extra = dict(gpu_seg=gpu["seg_id"][sel][worst], gpu_lit=gpu["lit"][sel][worst])
    name = re.sub(r"[^A-Za-z0-9_.=-]", "_", label)
    np.savez(os.path.join(out, f"mismatch_{name}.npz"), pixels=sel[worst],
             gpu_rgb=gpu["rgb"][sel][worst], gpu_ids=gpu["ids"][sel][worst],
             ora_rgb=base.rgb[worst], ora_ids=base.prim_id[worst], ora_seg=base.seg_id[worst],
             ora_lit=base.lit[worst], margin=base.margin[worst], err=err[worst],
             nongrazing=nongrazing[worst], ok_cond=ok_cond[worst], **extra)
    log("dumped", len(worst), "mismatching pixels of", label)
