"""FP64 oracle of the temporal gradient (A-SVGF), the answer to temporal lag
that the paper's related work names (Section 2): surface samples of the
previous frame are carried forward into the current one, shaded again, and
the difference between the two shadings drives the temporal blend.

TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path; it shares no
code with the HIP library.

The paper describes the method in one paragraph without formulas; the
steps below are the readings used (each is stated where it is made):

1. One sample per 3x3 stratum of the previous frame: pixel q = (3 sx + k %
   3, 3 sy + k // 3) with k the stratum's pick (0..8, drawn by the
   renderer, an input); a pick outside the image, or above 8, gives no
   sample.
2. Forward projection: q lands on pixel p = floor(q + fmv(q) + 1/2) of the
   current frame (fmv: forward motion in pixels; the two additions are
   binary32 roundings, the device's precision, since they decide an
   integer).  The sample is kept if p is inside the image, the current
   pixel has a surface, and the depth of the moved point fz(q) agrees with
   the current depth z(p) as in the reprojection test,
   |z(p) - fz(q)| <= tau_z z(p) (binary32, as there).
3. The sample goes to the current 3x3 cell of p; when several samples land
   in one cell, the one of the lowest stratum index (row-major) is kept.
4. Gradient sample: delta = L(reshade(q)) - L(prev(q)) and
   norm = max(L(reshade(q)), L(prev(q))), L the Rec. 709 luminance, reshade
   the sample traced again in the current frame with its old random
   numbers.
5. Dense gradient: a normalized convolution over the cells, cascading
   `levels` 5x5 a-trous B3 kernels at cell steps 1, 2, 4, ... with a depth
   edge weight exp(-|z_c - z_d| / (sigma_z |dz . o| + eps)) between the
   cells' centre pixels (o the offset in pixels); delta, norm and the
   sample indicator are filtered alike and divided at the end.  The sums
   are carried as the ratios (weighted means of delta and norm) and the
   logarithm of the filtered indicator, each level's terms combined with
   their largest exponent factored out: the same quotients, with no
   underflow where every weight reaching a cell is tiny (a cell far across
   depth edges from every sample), where plain binary64 sums would fall
   into subnormal numbers and lose the ratio's digits.
6. lambda = min(1, |delta_hat| / norm_hat) (0 where norm_hat is 0 or no
   sample reached the cell), and the blend factor of every pixel of the
   cell is alpha' = (1 - lambda) alpha + lambda: the history is dropped
   where the shading changed.
"""

from __future__ import annotations

import numpy as np

__all__ = ["cells_of", "gradient_samples", "reconstruct", "temporal_gradient"]

_W = (0.2126, 0.7152, 0.0722)
_H1 = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


def _luma(rgb):
    rgb = np.asarray(rgb, np.float64)
    return _W[0] * rgb[0] + _W[1] * rgb[1] + _W[2] * rgb[2]


def cells_of(H, W):
    """Cell (and stratum) grid size: ceil(H / 3) x ceil(W / 3)."""
    return (H + 2) // 3, (W + 2) // 3


def _empty(z):
    return not (z > 0.0) or not np.isfinite(z)


def gradient_samples(prev_rgb, reshade_rgb, fmv, fz, pick, z, tau_z=0.1):
    """Steps 1-4.  Returns (delta, norm, present, src): per current cell the
    gradient sample, whether one landed, and the stratum index it came from
    (-1 for none)."""
    H, W = z.shape
    CH, CW = cells_of(H, W)
    Lp, Lr = _luma(prev_rgb), _luma(reshade_rgb)
    f32 = np.float32
    src = -np.ones((CH, CW), np.int64)
    for sy in range(CH):
        for sx in range(CW):
            k = int(pick[sy, sx])
            qx, qy = 3 * sx + k % 3, 3 * sy + k // 3
            if k > 8 or qx >= W or qy >= H:
                continue
            tx = f32(f32(qx) + f32(fmv[0][qy, qx])) + f32(0.5)
            ty = f32(f32(qy) + f32(fmv[1][qy, qx])) + f32(0.5)
            if not (0.0 <= tx < W and 0.0 <= ty < H):  # NaN fails too
                continue
            px, py = int(np.floor(tx)), int(np.floor(ty))
            zc = f32(z[py, px])
            if _empty(zc):
                continue
            # the reprojection's depth test, in binary32 with its order
            if not (abs(f32(f32(fz[qy, qx]) - zc)) <= f32(f32(tau_z) * zc)):
                continue
            cy, cx = py // 3, px // 3
            s = sy * CW + sx
            if src[cy, cx] < 0 or s < src[cy, cx]:
                src[cy, cx] = s
    delta = np.zeros((CH, CW))
    norm = np.zeros((CH, CW))
    for cy in range(CH):
        for cx in range(CW):
            s = src[cy, cx]
            if s < 0:
                continue
            sy, sx = divmod(int(s), CW)
            k = int(pick[sy, sx])
            qx, qy = 3 * sx + k % 3, 3 * sy + k // 3
            delta[cy, cx] = Lr[qy, qx] - Lp[qy, qx]
            norm[cy, cx] = max(Lr[qy, qx], Lp[qy, qx])
    return delta, norm, (src >= 0).astype(np.float64), src


def reconstruct(delta, norm, present, z, dzdx, dzdy, levels=3, sigma_z=1.0, eps_z=1e-10):
    """Step 5 and the ratio of step 6: lambda per cell.

    The normalized convolution sum_j w_j x_j / sum_j w_j p_j, cascaded over
    the levels, is carried per cell as (mean of delta, mean of norm, natural
    logarithm of the filtered indicator): a level's sum over taps j of
    w_ij * (indicator sum of j) * (means of j) is formed as
    exp(t_ij - t_max) terms with t_ij = log w_ij + log(indicator sum of j),
    which is the plain sum divided by exp(t_max)."""
    H, W = z.shape
    CH, CW = delta.shape
    cyy = np.minimum(3 * np.arange(CH) + 1, H - 1)
    cxx = np.minimum(3 * np.arange(CW) + 1, W - 1)
    zc = np.asarray(z, np.float64)[np.ix_(cyy, cxx)]
    gx = np.asarray(dzdx, np.float64)[np.ix_(cyy, cxx)]
    gy = np.asarray(dzdy, np.float64)[np.ix_(cyy, cxx)]
    have = present > 0
    d = np.where(have, delta, 0.0)          # weighted mean of delta
    m = np.where(have, norm, 0.0)           # weighted mean of norm
    lg = np.where(have, 0.0, -np.inf)       # log of the indicator's sum
    for lvl in range(levels):
        s = 1 << lvl
        nd, nm, nlg = np.zeros_like(d), np.zeros_like(m), np.full_like(lg, -np.inf)
        for cy in range(CH):
            for cx in range(CW):
                ts, ds, ms = [], [], []
                for b in range(-2, 3):
                    for c in range(-2, 3):
                        ny, nx = cy + b * s, cx + c * s
                        if not (0 <= ny < CH and 0 <= nx < CW) or lg[ny, nx] == -np.inf:
                            continue
                        # offset between the centre pixels, in pixels
                        ox, oy = 3.0 * c * s, 3.0 * b * s
                        den = sigma_z * abs(gx[cy, cx] * ox + gy[cy, cx] * oy) + eps_z
                        ts.append(np.log(_H1[b + 2] * _H1[c + 2])
                                  - abs(zc[cy, cx] - zc[ny, nx]) / den + lg[ny, nx])
                        ds.append(d[ny, nx])
                        ms.append(m[ny, nx])
                if not ts:
                    continue
                t = np.array(ts)
                top = t.max()
                w = np.exp(t - top)
                nd[cy, cx] = np.dot(w, ds) / w.sum()
                nm[cy, cx] = np.dot(w, ms) / w.sum()
                nlg[cy, cx] = top + np.log(w.sum())
        d, m, lg = nd, nm, nlg
    reached = lg > -np.inf
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = np.where(reached & (m > 0), np.minimum(1.0, np.abs(d) / m), 0.0)
    return lam


def temporal_gradient(prev_rgb, reshade_rgb, fmv, fz, pick, z, dzdx, dzdy, alpha=0.2,
                      tau_z=0.1, sigma_z=1.0, levels=3):
    """The whole gradient: returns (alpha_map (H, W), lambda (cells))."""
    delta, norm, present, _ = gradient_samples(prev_rgb, reshade_rgb, fmv, fz, pick, z, tau_z)
    lam = reconstruct(delta, norm, present, z, dzdx, dzdy, levels, sigma_z)
    H, W = z.shape
    per_px = lam[np.arange(H)[:, None] // 3, np.arange(W)[None, :] // 3]
    return (1.0 - per_px) * alpha + per_px, lam
