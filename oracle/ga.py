"""Plain float64 definition of camera global alignment (GA).

Paper anchors (arXiv 2509.25191):
  * Sec. 3.3, Eq. (epi): the loss is the weighted mean of the epipolar
    residuals e_{m,k} of the correspondences k of the image pairs m, with the
    fundamental matrix F_m built from the two cameras of the pair.
  * Sec. 3.3: candidate pairs are those whose views differ by less than an
    angle threshold (30 degrees in Sec. 4.1).
  * Sec. 3.3, Eq. (weight): w_k = (f(e_k) / Avg f(e))^alpha, f the density of
    the residuals estimated by a histogram, alpha = 0.5; the residuals are
    those of the initial (predicted) cameras.
  * Sec. 3.3, Eq. (lr) and Sec. 4.1: the learning rate is lr0 / lr1 / lr2 =
    5e-4 / 1e-3 / 1e-2 when the median residual is below b1 = 2.5, between b1
    and b2 = 7.5, or above b2; at most 4096 correspondences per pair and 300
    iterations.

Readings where the paper is silent:
  * Camera: x_cam = R X + t, pixel = (f x/z + cx, f y/z + cy); the
    principal point is fixed, the focal length f is refined.
  * Residual: the distance in pixels of x'_k from the epipolar line F x_k in
    the second image, |x'^T F x| / ||(F x)_{0:2}|| (the paper's x'^T F x with
    F scaled so that the line has a unit normal; the histogram range of 20
    pixels in the paper's figure is a pixel distance).
  * Relative pose of pair (i, j): R_ij = R_j R_i^T, t_ij = t_j - R_ij t_i;
    F = K_j^-T [t_ij]_x R_ij K_i^-1.
  * Parameters per camera: an unnormalised quaternion q (R = R(q / |q|)), the
    translation t, and phi with f = f0 exp(phi); all start at the predicted
    camera.  Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias
    corrected) on the loss of Eq. (epi) with the weights held fixed.
  * Histogram: bins of 0.1 pixel over [0, 20) (bin b = floor(10 e)), one
    overflow bin for e >= 20 whose density is taken as zero;
    f(e) = count(bin) / (K * 0.1), Avg f = sum_k f(e_k) / K.  When no
    residual falls below 20 pixels every weight is 1.
  * Median: the bin holding the ceil(K/2)-th smallest residual decides the
    learning rate (bin < 25: lr0; 25 <= bin < 75: lr1; bin >= 75: lr2).  The
    bounds are bin edges, so this is the decision of the exact median.
  * View angle of a pair: the angle between the two optical axes (third rows
    of R_i and R_j); the learning rate and the weights are chosen once, from
    the initial cameras.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np

HIST_BINS = 200       # bins of 0.1 px over [0, 20)
HIST_SCALE = 10.0     # bins per pixel
ADAM = (0.9, 0.999, 1e-8)


# ---------------------------------------------------------------- rotations

def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of the unit quaternion q / |q|, q = (w, x, y, z); works on [..., 4]."""
    q = np.asarray(q, np.float64)
    n2 = (q * q).sum(-1)[..., None, None]
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    m = np.stack([
        np.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], -1),
    ], -2)
    return m / n2


def rot_to_quat(R: np.ndarray) -> np.ndarray:
    """A unit quaternion (w >= 0) of each rotation matrix in [..., 3, 3]."""
    R = np.asarray(R, np.float64)
    out = np.empty(R.shape[:-2] + (4,))
    for idx in np.ndindex(R.shape[:-2]):
        m = R[idx]
        tr = m[0, 0] + m[1, 1] + m[2, 2]
        # largest of the four candidates keeps the square root well conditioned
        c = np.array([tr, m[0, 0] - m[1, 1] - m[2, 2], m[1, 1] - m[0, 0] - m[2, 2], m[2, 2] - m[0, 0] - m[1, 1]])
        k = int(np.argmax(c))
        s = math.sqrt(max(c[k] + 1.0, 0.0)) * 2.0
        if k == 0:
            q = [s / 4, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif k == 1:
            q = [(m[2, 1] - m[1, 2]) / s, s / 4, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif k == 2:
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, s / 4, (m[1, 2] + m[2, 1]) / s]
        else:
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, s / 4]
        q = np.array(q)
        out[idx] = q if q[0] >= 0 else -q
    return out


def skew(t: np.ndarray) -> np.ndarray:
    return np.array([[0.0, -t[2], t[1]], [t[2], 0.0, -t[0]], [-t[1], t[0], 0.0]])


def k_inv(f: float, c: Sequence[float]) -> np.ndarray:
    return np.array([[1.0 / f, 0.0, -c[0] / f], [0.0, 1.0 / f, -c[1] / f], [0.0, 0.0, 1.0]])


# ---------------------------------------------------------------- pairs

def select_pairs(R: np.ndarray, max_angle_deg: float) -> np.ndarray:
    """Pairs (i, j), i < j, whose optical axes (third rows of R) differ by
    less than max_angle_deg, in row-major order of (i, j)."""
    z = np.asarray(R, np.float64)[:, 2, :]
    z = z / np.linalg.norm(z, axis=1, keepdims=True)
    cos_lim = math.cos(math.radians(max_angle_deg))
    out = []
    n = len(z)
    for i in range(n):
        for j in range(i + 1, n):
            if float(np.dot(z[i], z[j])) > cos_lim:
                out.append((i, j))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


# ---------------------------------------------------------------- residuals

def fundamental(Ri, ti, fi, ci, Rj, tj, fj, cj) -> np.ndarray:
    """F of the pair (i, j): x_j^T F x_i = 0 for a scene point seen at pixel
    x_i in camera i and x_j in camera j."""
    Rij = Rj @ Ri.T
    tij = tj - Rij @ ti
    return k_inv(fj, cj).T @ skew(tij) @ Rij @ k_inv(fi, ci)


def residuals(F: np.ndarray, corr: np.ndarray) -> np.ndarray:
    """e_k = |x'^T F x| / ||(F x)_{0:2}|| for corr [n, 4] = (u, v, u', v')."""
    c = np.asarray(corr, np.float64)
    x = np.stack([c[:, 0], c[:, 1], np.ones(len(c))], 1)
    xp = np.stack([c[:, 2], c[:, 3], np.ones(len(c))], 1)
    l = x @ F.T
    s = (xp * l).sum(1)
    return np.abs(s) / np.sqrt(l[:, 0] ** 2 + l[:, 1] ** 2)


def all_residuals(cams: Dict[str, np.ndarray], pairs: np.ndarray, offsets: np.ndarray, corr: np.ndarray) -> np.ndarray:
    R, t, f, c = cams["R"], cams["t"], cams["f"], cams["c"]
    e = np.empty(offsets[-1])
    for m, (i, j) in enumerate(pairs):
        F = fundamental(R[i], t[i], f[i], c[i], R[j], t[j], f[j], c[j])
        e[offsets[m]:offsets[m + 1]] = residuals(F, corr[offsets[m]:offsets[m + 1]])
    return e


# ---------------------------------------------------------------- weights, learning rate

def hist_bins(e: np.ndarray) -> np.ndarray:
    """Bin b = floor(10 e) for e < 20, HIST_BINS (overflow) otherwise."""
    e = np.asarray(e, np.float64)
    b = np.floor(e * HIST_SCALE)
    return np.where(e < HIST_BINS / HIST_SCALE, b, HIST_BINS).astype(np.int64)


def weight_table(bins: np.ndarray, alpha: float = 0.5) -> Tuple[np.ndarray, np.ndarray]:
    """(counts [HIST_BINS + 1], table [HIST_BINS + 1]) with w_k = table[bin_k]:
    f(b) = count_b / (K h) (0 for the overflow bin), Avg f = sum_k f(bin_k) / K,
    table[b] = (f(b) / Avg f)^alpha."""
    K = len(bins)
    counts = np.bincount(bins, minlength=HIST_BINS + 1).astype(np.float64)
    h = 1.0 / HIST_SCALE
    dens = counts / (K * h)
    dens[HIST_BINS] = 0.0
    avg = (counts * dens).sum() / K
    if avg <= 0.0:
        return counts, np.ones(HIST_BINS + 1)
    return counts, (dens / avg) ** alpha


def median_bin(counts: np.ndarray) -> int:
    """Bin of the ceil(K/2)-th smallest residual."""
    K = int(counts.sum())
    rank = (K + 1) // 2
    return int(np.searchsorted(np.cumsum(counts), rank))


def choose_lr(counts: np.ndarray, lrs=(5e-4, 1e-3, 1e-2), bounds=(2.5, 7.5)) -> float:
    b = median_bin(counts)
    if b < int(round(bounds[0] * HIST_SCALE)):
        return lrs[0]
    if b < int(round(bounds[1] * HIST_SCALE)):
        return lrs[1]
    return lrs[2]


# ---------------------------------------------------------------- loss and gradient

def params_to_cams(p: Dict[str, np.ndarray], f0: np.ndarray, c: np.ndarray) -> Dict[str, np.ndarray]:
    return {"R": quat_to_rot(p["q"]), "t": p["t"], "f": f0 * np.exp(p["phi"]), "c": c}


def loss(p, f0, c, pairs, offsets, corr, table, bins) -> float:
    cams = params_to_cams(p, f0, c)
    e = all_residuals(cams, pairs, offsets, corr)
    w = table[bins]
    return float((w * e).sum() / w.sum())


def _drot_dq(q: np.ndarray) -> np.ndarray:
    """d R(q/|q|) / d q_a for a = 0..3: [4, 3, 3]."""
    w, x, y, z = q
    n2 = float(q @ q)
    N = quat_to_rot(q) * n2  # numerator polynomial matrix
    dN = np.array([
        [[2 * w, -2 * z, 2 * y], [2 * z, 2 * w, -2 * x], [-2 * y, 2 * x, 2 * w]],
        [[2 * x, 2 * y, 2 * z], [2 * y, -2 * x, -2 * w], [2 * z, 2 * w, -2 * x]],
        [[-2 * y, 2 * x, 2 * w], [2 * x, 2 * y, 2 * z], [-2 * w, 2 * z, -2 * y]],
        [[-2 * z, -2 * w, 2 * x], [2 * w, -2 * z, 2 * y], [2 * x, 2 * y, 2 * z]],
    ])
    return (dN * n2 - N[None] * (2 * q)[:, None, None]) / (n2 * n2)


def gradient(p, f0, c, pairs, offsets, corr, table, bins) -> Dict[str, np.ndarray]:
    """Analytic gradient of ``loss`` with respect to q [N, 4], t [N, 3], phi [N]."""
    q, t, phi = p["q"], p["t"], p["phi"]
    R = quat_to_rot(q)
    f = f0 * np.exp(phi)
    w_all = table[bins]
    W = w_all.sum()
    gR = np.zeros_like(R); gt = np.zeros_like(t); gf = np.zeros_like(f)
    for m, (i, j) in enumerate(pairs):
        a, b = offsets[m], offsets[m + 1]
        if b == a:
            continue
        cc = np.asarray(corr[a:b], np.float64)
        w = w_all[a:b] / W
        Ki, Kj = k_inv(f[i], c[i]), k_inv(f[j], c[j])
        Rij = R[j] @ R[i].T
        tij = t[j] - Rij @ t[i]
        E = skew(tij) @ Rij
        F = Kj.T @ E @ Ki
        x = np.stack([cc[:, 0], cc[:, 1], np.ones(b - a)], 1)
        xp = np.stack([cc[:, 2], cc[:, 3], np.ones(b - a)], 1)
        l = x @ F.T
        s = (xp * l).sum(1)
        n = np.sqrt(l[:, 0] ** 2 + l[:, 1] ** 2)
        e = np.abs(s) / n
        # de/dF = g x^T with g_r = sign(s) x'_r / n - [r < 2] e l_r / n
        g = np.sign(s)[:, None] * xp / n[:, None]
        g[:, :2] -= (e / n)[:, None] * l[:, :2] / n[:, None]
        GF = (w[:, None] * g).T @ x                     # dL/dF (3x3)
        GE = Kj @ GF @ Ki.T                             # F = Kj^-T E Ki^-1
        GKi = (Kj.T @ E).T @ GF                         # dL/d(Ki^-1)
        GKjT = GF @ (E @ Ki).T                          # dL/d(Kj^-T)
        dKi = np.array([[-1 / f[i] ** 2, 0, c[i][0] / f[i] ** 2], [0, -1 / f[i] ** 2, c[i][1] / f[i] ** 2], [0, 0, 0]])
        dKjT = np.array([[-1 / f[j] ** 2, 0, 0], [0, -1 / f[j] ** 2, 0], [c[j][0] / f[j] ** 2, c[j][1] / f[j] ** 2, 0]])
        gf[i] += (GKi * dKi).sum()
        gf[j] += (GKjT * dKjT).sum()
        M = GE @ Rij.T                                  # dL/d[t]_x
        gtij = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
        GRij = skew(tij).T @ GE - np.outer(gtij, t[i])  # E = [t]_x Rij, t_ij = t_j - Rij t_i
        gt[j] += gtij
        gt[i] += -Rij.T @ gtij
        gR[j] += GRij @ R[i]                            # Rij = Rj Ri^T
        gR[i] += GRij.T @ R[j]
    gq = np.stack([np.einsum("aij,ij->a", _drot_dq(q[n]), gR[n]) for n in range(len(q))])
    return {"q": gq, "t": gt, "phi": gf * f}


# ---------------------------------------------------------------- the whole procedure

def align(R0, t0, f0, c, pairs, offsets, corr, iterations: int = 300, lrs=(5e-4, 1e-3, 1e-2),
          bounds=(2.5, 7.5), alpha: float = 0.5, adam=ADAM):
    """GA from the predicted cameras: weights and learning rate from the
    initial residuals, then ``iterations`` Adam steps on the weighted loss.
    Returns (R, t, f, weights per correspondence, losses) where losses[i] is
    the loss before step i and losses[iterations] the final one."""
    R0 = np.asarray(R0, np.float64); t0 = np.asarray(t0, np.float64)
    f0 = np.asarray(f0, np.float64); c = np.asarray(c, np.float64)
    pairs = np.asarray(pairs, np.int64); offsets = np.asarray(offsets, np.int64)
    cams0 = {"R": R0, "t": t0, "f": f0, "c": c}
    e0 = all_residuals(cams0, pairs, offsets, corr)
    bins = hist_bins(e0)
    counts, table = weight_table(bins, alpha)
    lr = choose_lr(counts, lrs, bounds)
    p = {"q": rot_to_quat(R0), "t": t0.copy(), "phi": np.zeros(len(f0))}
    mom = {k: np.zeros_like(v) for k, v in p.items()}
    vel = {k: np.zeros_like(v) for k, v in p.items()}
    b1, b2, eps = adam
    losses = []
    for it in range(1, iterations + 1):
        losses.append(loss(p, f0, c, pairs, offsets, corr, table, bins))
        g = gradient(p, f0, c, pairs, offsets, corr, table, bins)
        for k in p:
            mom[k] = b1 * mom[k] + (1 - b1) * g[k]
            vel[k] = b2 * vel[k] + (1 - b2) * g[k] ** 2
            mh = mom[k] / (1 - b1 ** it)
            vh = vel[k] / (1 - b2 ** it)
            p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    losses.append(loss(p, f0, c, pairs, offsets, corr, table, bins))
    cams = params_to_cams(p, f0, c)
    return cams["R"], cams["t"], cams["f"], table[bins], np.array(losses), lr
