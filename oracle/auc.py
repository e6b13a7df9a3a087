"""Plain float64 definition of the pose-accuracy metric AUC@30 and its
permutation-equivariant form (arXiv 2509.25191, appendix "Permutation-
Equivariant AUC@30").

Paper anchors: for an image pair (i, j) the relative pose is
E_i^-1 E_j = [R_i^T R_j | R_i^T (t_j - t_i)] with E = [R | t]; the relative
rotation error (RRE) and relative translation error (RTE) compare the
predicted and ground-truth relative poses; the conventional metric uses the
pairs i < j only, which makes the translation error depend on the image
order; the paper's modification uses both (i, j) and (j, i).

Readings where the paper is silent:
  * RRE = the rotation angle of dR_pred^T dR_gt, in degrees;
    RTE = the angle between dt_pred and dt_gt, in degrees (0 when either is
    the zero vector).
  * AUC@30 = (1/30) sum over tau = 1..30 degrees of the fraction of relative
    poses with max(RRE, RTE) < tau.
"""
from __future__ import annotations

import math

import numpy as np


def relative_pose(Ri, ti, Rj, tj):
    """E_i^-1 E_j = (R_i^T R_j, R_i^T (t_j - t_i))."""
    return Ri.T @ Rj, Ri.T @ (tj - ti)


def rotation_angle_deg(R: np.ndarray) -> float:
    c = (np.trace(R) - 1.0) / 2.0
    return math.degrees(math.acos(min(1.0, max(-1.0, c))))


def vector_angle_deg(a: np.ndarray, b: np.ndarray) -> float:
    na, nb = float(np.linalg.norm(a)), float(np.linalg.norm(b))
    if na == 0.0 or nb == 0.0:
        return 0.0
    c = float(np.dot(a, b)) / (na * nb)
    return math.degrees(math.acos(min(1.0, max(-1.0, c))))


def pair_errors(R_pred, t_pred, R_gt, t_gt, both_orders: bool = True):
    """max(RRE, RTE) of every ordered pair (i, j), i != j (both_orders) or i < j."""
    n = len(R_pred)
    out = []
    for i in range(n):
        for j in range(n):
            if i == j or (not both_orders and j < i):
                continue
            Rp, tp = relative_pose(R_pred[i], t_pred[i], R_pred[j], t_pred[j])
            Rg, tg = relative_pose(R_gt[i], t_gt[i], R_gt[j], t_gt[j])
            out.append(max(rotation_angle_deg(Rp.T @ Rg), vector_angle_deg(tp, tg)))
    return np.array(out)


def auc30(R_pred, t_pred, R_gt, t_gt, both_orders: bool = True):
    """(AUC@30, counts) with counts[b] = number of relative poses whose error
    lies in [b, b+1) degrees for b < 30 and counts[30] those at 30 or more."""
    err = pair_errors(np.asarray(R_pred, np.float64), np.asarray(t_pred, np.float64),
                      np.asarray(R_gt, np.float64), np.asarray(t_gt, np.float64), both_orders)
    bins = np.minimum(np.floor(err), 30).astype(np.int64)
    counts = np.bincount(bins, minlength=31)
    if len(err) == 0:
        return 0.0, counts
    frac = np.array([(err < tau).mean() for tau in range(1, 31)])
    return float(frac.mean()), counts
