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


def bvh_bound_errors(nodes, order, pos, idx):
    """Vectorised check that every child box of an exported 4-wide BVH equals the exact FP32 min/max
    of what it contains (the leaf's triangles, or the child node's boxes).  Returns the number of
    child boxes that differ, and a histogram of leaf sizes."""
    nodes = np.asarray(nodes, np.uint32)
    f = nodes.view(np.float32)
    lo = np.stack([f[:, 0:4], f[:, 8:12], f[:, 16:20]], axis=1)     # (n, 3, 4)
    hi = np.stack([f[:, 4:8], f[:, 12:16], f[:, 20:24]], axis=1)
    child = nodes[:, 24:28]
    empty = child == 0xFFFFFFFF
    leaf = ((child & 0x80000000) != 0) & ~empty
    inner = ~leaf & ~empty
    bad = 0
    # leaves
    ni, ci = np.nonzero(leaf)
    w = child[ni, ci]
    first = (w & 0x0FFFFFFF).astype(np.int64)
    cnt = (((w >> 28) & 7) + 1).astype(np.int64)
    elo = np.full((len(w), 3), np.inf, np.float32)
    ehi = np.full((len(w), 3), -np.inf, np.float32)
    for k in range(4):
        m = k < cnt
        tri = order[first[m] + k]
        for v in range(3):
            p = pos[idx[tri, v]]
            elo[m] = np.minimum(elo[m], p)
            ehi[m] = np.maximum(ehi[m], p)
    bad += int((~((lo[ni, :, ci] == elo).all(1) & (hi[ni, :, ci] == ehi).all(1))).sum())
    # internal children
    ni, ci = np.nonzero(inner)
    w = child[ni, ci].astype(np.int64)
    clo = np.where(empty[w][:, None, :], np.inf, lo[w]).min(axis=2)
    chi = np.where(empty[w][:, None, :], -np.inf, hi[w]).max(axis=2)
    bad += int((~((lo[ni, :, ci] == clo).all(1) & (hi[ni, :, ci] == chi).all(1))).sum())
    return bad, np.bincount(cnt, minlength=5)
