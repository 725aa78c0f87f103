"""Element-wise comparison of GPU render outputs with the CPU oracle, outside the FP32 band.

The band (computed by the oracle) holds the samples whose answer is not fixed by FP32
arithmetic: there either answer is accepted and the sample is counted.  Outside it:
  - hit triangle id and shadow-mask bits must be equal (bit-exact),
  - t, u, v must lie within the oracle's FP32 error bound of the FP64 values,
  - radiance must agree to 1e-4 relative (floor 1e-6 of the image maximum).
"""
import numpy as np

NO_HIT = 0xFFFFFFFF
RTOL = 1e-4


def to_np(t):
    return t.detach().cpu().numpy()


def compare_point(hit, mask, srgba, orc, n_lights, rtol=RTOL):
    """hit (n,4) uint32, mask (n,) uint32 or None, srgba (n,4) float32 for the sampled rows;
    orc = oracle render_point output for the same samples."""
    hit = hit.view(np.uint32)
    gid = hit[:, 0]
    gt, gu, gv = hit[:, 1].view(np.float32), hit[:, 2].view(np.float32), hit[:, 3].view(np.float32)
    bp = orc["band_primary"].astype(bool)
    oid = orc["hit_id"]
    out = {"n": len(gid), "band_primary": int(bp.sum())}
    ok = ~bp
    out["id_mismatch"] = int((gid[ok] != oid[ok]).sum())
    hitm = ok & (oid != NO_HIT)
    slack = 1e-12
    for k, g in enumerate((gt, gu, gv)):
        err = np.abs(g[hitm].astype(np.float64) - orc["tuv"][hitm, k])
        out[f"tuv{k}_viol"] = int((err > orc["tuv_err"][hitm, k] + slack).sum())
    out["miss_t_not_inf"] = int((~np.isinf(gt[ok & (oid == NO_HIT)])).sum())
    full = (1 << n_lights) - 1
    if n_lights:
        bs = orc["band_shadow"]
        cmp_bits = (~bs) & full
        mask = mask.view(np.uint32)
        diff = (mask ^ orc["mask"]) & cmp_bits
        out["mask_mismatch"] = int((diff[ok] != 0).sum())
        out["band_shadow"] = int(((bs != 0) & ok).sum())
        clean = ok & (bs == 0)
    else:
        out["mask_mismatch"] = 0
        out["band_shadow"] = 0
        clean = ok
    if srgba is not None:
        L = orc["rgb"]
        lmax = max(float(L.max()), 1e-30)
        tol = rtol * np.maximum(np.abs(L), 1e-6 * lmax)
        err = np.abs(srgba[:, :3].astype(np.float64) - L)
        bad = (err > tol) & clean[:, None]
        out["rgb_viol"] = int(bad.any(axis=1).sum())
        rel = err / np.maximum(np.abs(L), 1e-6 * lmax)
        out["rgb_max_rel"] = float(rel[clean].max()) if clean.any() else 0.0
        alpha_want = (oid != NO_HIT).astype(np.float32)
        out["alpha_mismatch"] = int((srgba[ok, 3] != alpha_want[ok]).sum())
    out["clean"] = int(clean.sum())
    return out


def assert_clean(stats, max_band_frac=0.05):
    for k in ("id_mismatch", "tuv0_viol", "tuv1_viol", "tuv2_viol", "miss_t_not_inf", "mask_mismatch",
              "rgb_viol", "alpha_mismatch"):
        assert stats.get(k, 0) == 0, (k, stats)
    assert stats["band_primary"] <= max_band_frac * stats["n"], stats
