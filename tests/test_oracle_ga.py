"""Pins of the global-alignment oracle (Sec. 3.3): the residual against
closed forms and an independent geometric construction, the analytic
gradient against torch autograd, Adam against torch.optim.Adam, the
histogram weights and the median rule against hand-worked examples and
numpy, the pair rule against a constructed camera ring."""
import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import ga
import synth


def _rng(s):
    return np.random.default_rng(s)


def test_quaternion_matches_scipy():
    rng = _rng(1)
    q = rng.normal(0, 1, (6, 4)) * 3.0  # unnormalised
    R = ga.quat_to_rot(q)
    ref = Rotation.from_quat(np.roll(q, -1, axis=1)).as_matrix()  # scipy order (x, y, z, w)
    np.testing.assert_allclose(R, ref, atol=1e-12)
    back = ga.quat_to_rot(ga.rot_to_quat(ref))
    np.testing.assert_allclose(back, ref, atol=1e-12)


def test_residual_rectified_stereo_is_row_difference():
    """R = I for both cameras, baseline along x, same K: epipolar lines are
    image rows, so e = |v' - v|."""
    c = np.array([260.0, 250.0])
    F = ga.fundamental(np.eye(3), np.zeros(3), 500.0, c, np.eye(3), np.array([-0.3, 0.0, 0.0]), 500.0, c)
    rng = _rng(2)
    corr = rng.uniform(0, 518, (50, 4))
    np.testing.assert_allclose(ga.residuals(F, corr), np.abs(corr[:, 3] - corr[:, 1]), atol=1e-9)


def test_residual_is_distance_to_projected_ray():
    """Independent construction: project two points of the ray of x into
    camera j; e is the distance of x' to the line through them."""
    rng = _rng(3)
    true, _ = synth.gen_ga_cameras(rng, 6, arc_deg=60.0)
    R, t, f, c = true["R"], true["t"], true["f"], true["c"]
    i, j = 1, 3
    F = ga.fundamental(R[i], t[i], f[i], c[i], R[j], t[j], f[j], c[j])
    corr = rng.uniform(150, 350, (20, 4))
    e = ga.residuals(F, corr)
    C_i = -R[i].T @ t[i]
    for k in range(20):
        ray = R[i].T @ np.array([(corr[k, 0] - c[i, 0]) / f[i], (corr[k, 1] - c[i, 1]) / f[i], 1.0])
        pts = []
        for depth in (2.0, 6.0):
            X = C_i + depth * ray
            Xc = R[j] @ X + t[j]
            pts.append(np.array([f[j] * Xc[0] / Xc[2] + c[j, 0], f[j] * Xc[1] / Xc[2] + c[j, 1]]))
        d = pts[1] - pts[0]
        r = corr[k, 2:] - pts[0]
        dist = abs(d[0] * r[1] - d[1] * r[0]) / np.linalg.norm(d)
        assert abs(dist - e[k]) < 1e-8 * max(1.0, dist)


def test_residual_zero_for_exact_correspondences():
    rng = _rng(4)
    true, _ = synth.gen_ga_cameras(rng, 5, arc_deg=40.0)
    pairs = ga.select_pairs(true["R"], 30.0)
    corr, off = synth.gen_ga_corr(rng, true, pairs, 64, noise_px=0.0, outlier_frac=0.0)
    e = ga.all_residuals(true, pairs, off, corr.astype(np.float64))
    assert e.max() < 2e-3  # float32 storage of the pixel coordinates only


def _torch_loss(q, t, phi, f0, c, pairs, off, corr, w):
    """The loss of Eq. (epi) written with torch ops, differentiated by autograd."""
    n2 = (q * q).sum(1)
    a, b, cc, d = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = torch.stack([
        torch.stack([a * a + b * b - cc * cc - d * d, 2 * (b * cc - a * d), 2 * (b * d + a * cc)], -1),
        torch.stack([2 * (b * cc + a * d), a * a - b * b + cc * cc - d * d, 2 * (cc * d - a * b)], -1),
        torch.stack([2 * (b * d - a * cc), 2 * (cc * d + a * b), a * a - b * b - cc * cc + d * d], -1),
    ], -2) / n2[:, None, None]
    f = f0 * torch.exp(phi)
    num = 0.0
    for m, (i, j) in enumerate(pairs):
        Ki = torch.zeros(3, 3, dtype=torch.float64); Kj = torch.zeros(3, 3, dtype=torch.float64)
        Ki[0, 0] = 1 / f[i]; Ki[1, 1] = 1 / f[i]; Ki[0, 2] = -c[i, 0] / f[i]; Ki[1, 2] = -c[i, 1] / f[i]; Ki[2, 2] = 1
        Kj[0, 0] = 1 / f[j]; Kj[1, 1] = 1 / f[j]; Kj[0, 2] = -c[j, 0] / f[j]; Kj[1, 2] = -c[j, 1] / f[j]; Kj[2, 2] = 1
        Rij = R[j] @ R[i].T
        tij = t[j] - Rij @ t[i]
        S = torch.zeros(3, 3, dtype=torch.float64)
        S[0, 1] = -tij[2]; S[0, 2] = tij[1]; S[1, 0] = tij[2]; S[1, 2] = -tij[0]; S[2, 0] = -tij[1]; S[2, 1] = tij[0]
        F = Kj.T @ S @ Rij @ Ki
        cm = torch.from_numpy(corr[off[m]:off[m + 1]].astype(np.float64))
        x = torch.stack([cm[:, 0], cm[:, 1], torch.ones(len(cm), dtype=torch.float64)], 1)
        xp = torch.stack([cm[:, 2], cm[:, 3], torch.ones(len(cm), dtype=torch.float64)], 1)
        l = x @ F.T
        e = (xp * l).sum(1).abs() / torch.sqrt(l[:, 0] ** 2 + l[:, 1] ** 2)
        num = num + (torch.from_numpy(w[off[m]:off[m + 1]]) * e).sum()
    return num / float(w.sum())


def test_gradient_matches_torch_autograd():
    rng = _rng(5)
    true, init = synth.gen_ga_cameras(rng, 5, arc_deg=50.0, rot_noise_deg=2.0)
    pairs = ga.select_pairs(init["R"], 30.0)
    corr, off = synth.gen_ga_corr(rng, true, pairs, 40, outlier_frac=0.2)
    bins = ga.hist_bins(ga.all_residuals(init, pairs, off, corr))
    _, table = ga.weight_table(bins)
    p = {"q": ga.rot_to_quat(init["R"]) * rng.uniform(0.5, 2.0, (5, 1)), "t": init["t"] + rng.normal(0, 0.01, (5, 3)),
         "phi": rng.normal(0, 0.02, 5)}
    g = ga.gradient(p, init["f"], init["c"], pairs, off, corr, table, bins)
    q = torch.tensor(p["q"], requires_grad=True); t = torch.tensor(p["t"], requires_grad=True)
    phi = torch.tensor(p["phi"], requires_grad=True)
    L = _torch_loss(q, t, phi, torch.from_numpy(init["f"]), torch.from_numpy(init["c"]), pairs, off, corr, table[bins])
    L.backward()
    assert abs(L.item() - ga.loss(p, init["f"], init["c"], pairs, off, corr, table, bins)) < 1e-10
    for k, tt in (("q", q), ("t", t), ("phi", phi)):
        np.testing.assert_allclose(g[k], tt.grad.numpy(), rtol=1e-9, atol=1e-9 * np.abs(tt.grad.numpy()).max())


def test_weight_table_hand_example():
    e = np.array([0.05, 0.05, 0.05, 0.15, 25.0])
    bins = ga.hist_bins(e)
    assert bins.tolist() == [0, 0, 0, 1, ga.HIST_BINS]
    counts, table = ga.weight_table(bins, 0.5)
    # densities 3/(5*0.1) = 6 and 1/(5*0.1) = 2; overflow 0; Avg f = (3*6 + 2 + 0)/5 = 4
    assert table[0] == math.sqrt(6 / 4) and table[1] == math.sqrt(2 / 4) and table[ga.HIST_BINS] == 0.0
    assert ga.weight_table(np.full(3, ga.HIST_BINS))[1].tolist() == [1.0] * (ga.HIST_BINS + 1)


def test_median_rule_matches_numpy_median():
    rng = _rng(6)
    for scale in (0.5, 1.5, 4.0, 9.0, 30.0):
        e = np.abs(rng.standard_cauchy(1001)) * scale
        med = float(np.median(e))
        want = 5e-4 if med < 2.5 else (1e-3 if med < 7.5 else 1e-2)
        counts, _ = ga.weight_table(ga.hist_bins(e))
        assert ga.choose_lr(counts) == want, (scale, med)


def test_select_pairs_on_a_ring():
    """Level cameras every 10 degrees on a full ring, threshold 25 degrees:
    the pairs are the neighbours at 10 and 20 degrees, wrap-around included."""
    yaw = np.radians(10.0 * np.arange(36))
    R = np.stack([synth._look_at_origin(np.array([math.sin(a), 0.0, -math.cos(a)])) for a in yaw])
    got = {tuple(p) for p in ga.select_pairs(R, 25.0).tolist()}
    want = {(min(i, (i + d) % 36), max(i, (i + d) % 36)) for i in range(36) for d in (1, 2)}
    assert got == want


def test_adam_matches_torch_optim():
    rng = _rng(8)
    true, init = synth.gen_ga_cameras(rng, 4, arc_deg=40.0, rot_noise_deg=2.0)
    pairs = ga.select_pairs(init["R"], 30.0)
    corr, off = synth.gen_ga_corr(rng, true, pairs, 30)
    R, t, f, w, losses, lr = ga.align(init["R"], init["t"], init["f"], init["c"], pairs, off, corr, iterations=6)
    bins = ga.hist_bins(ga.all_residuals(init, pairs, off, corr))
    _, table = ga.weight_table(bins)
    params = {"q": torch.tensor(ga.rot_to_quat(init["R"])), "t": torch.tensor(init["t"]),
              "phi": torch.zeros(4, dtype=torch.float64)}
    opt = torch.optim.Adam(list(params.values()), lr=lr, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(6):
        g = ga.gradient({k: v.numpy() for k, v in params.items()}, init["f"], init["c"], pairs, off, corr, table, bins)
        for k, v in params.items():
            v.grad = torch.from_numpy(g[k])
        opt.step()
    np.testing.assert_allclose(ga.quat_to_rot(params["q"].numpy()), R, atol=1e-12)
    np.testing.assert_allclose(params["t"].numpy(), t, atol=1e-12)
    np.testing.assert_allclose(init["f"] * np.exp(params["phi"].numpy()), f, rtol=1e-12)


def test_alignment_reduces_loss_and_downweights_outliers():
    rng = _rng(9)
    true, init = synth.gen_ga_cameras(rng, 8, arc_deg=80.0, rot_noise_deg=0.5, trans_noise=0.02, focal_noise=0.01)
    pairs = ga.select_pairs(init["R"], 30.0)
    rng2 = _rng(10)
    corr, off = synth.gen_ga_corr(rng2, true, pairs, 200, outlier_frac=0.3)
    R, t, f, w, losses, lr = ga.align(init["R"], init["t"], init["f"], init["c"], pairs, off, corr, iterations=100)
    assert losses[-1] < 0.5 * losses[0]
    # outliers were drawn with the same generator stream: recover them by their residual at the true cameras
    e_true = ga.all_residuals(true, pairs, off, corr)
    out = e_true > 5.0
    assert w[out].mean() < 0.5 * w[~out].mean()
