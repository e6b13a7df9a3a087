"""Pins of the AUC@30 oracle (paper appendix): relative pose algebra, the
order sensitivity of the conventional metric that the paper points out, the
invariance of the both-orders form, and hand-built error distributions."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import auc
import synth


def _poses(seed, n, noise_deg=0.0, tnoise=0.0):
    rng = np.random.default_rng(seed)
    R = Rotation.random(n, random_state=seed).as_matrix()
    t = rng.normal(0, 1, (n, 3))
    Rp = np.stack([Rotation.from_rotvec(rng.normal(0, math.radians(noise_deg), 3)).as_matrix() @ r for r in R])
    tp = t + rng.normal(0, tnoise, (n, 3))
    return R, t, Rp, tp


def test_relative_pose_is_inverse_times_other():
    R, t, _, _ = _poses(1, 2)
    E = [np.block([[R[k], t[k][:, None]], [np.zeros((1, 3)), np.ones((1, 1))]]) for k in range(2)]
    D = np.linalg.inv(E[0]) @ E[1]
    dR, dt = auc.relative_pose(R[0], t[0], R[1], t[1])
    np.testing.assert_allclose(D[:3, :3], dR, atol=1e-12)
    np.testing.assert_allclose(D[:3, 3], dt, atol=1e-12)


def test_angles_against_scipy_and_closed_forms():
    rng = np.random.default_rng(2)
    for _ in range(5):
        v = rng.normal(0, 1, 3)
        R = Rotation.from_rotvec(v).as_matrix()
        assert abs(auc.rotation_angle_deg(R) - math.degrees(np.linalg.norm(v) % (2 * math.pi))) < 1e-8 or \
            abs(auc.rotation_angle_deg(R) - (360 - math.degrees(np.linalg.norm(v) % (2 * math.pi)))) < 1e-8
    assert abs(auc.vector_angle_deg(np.array([1.0, 0, 0]), np.array([1.0, 1.0, 0])) - 45.0) < 1e-12
    assert auc.vector_angle_deg(np.zeros(3), np.ones(3)) == 0.0


def test_perfect_prediction_gives_one_and_order_sensitivity():
    R, t, Rp, tp = _poses(3, 12, noise_deg=3.0, tnoise=0.3)
    a, c = auc.auc30(R, t, R, t)
    assert a == 1.0 and c[0] == 12 * 11
    # conventional (i < j only) depends on the image order; both orders does not
    perm = np.random.default_rng(4).permutation(12)
    conv = [auc.auc30(Rp[p], tp[p], R[p], t[p], both_orders=False)[0] for p in (np.arange(12), perm)]
    both = [auc.auc30(Rp[p], tp[p], R[p], t[p], both_orders=True)[0] for p in (np.arange(12), perm)]
    assert conv[0] != conv[1]
    assert abs(both[0] - both[1]) < 1e-12


def test_auc_of_constructed_errors():
    """Identity cameras at x = 0, 1, 2; the prediction turns camera 2 by 10.5
    degrees about z.  Every ordered pair with camera 2 has RRE 10.5 degrees
    (its relative translation turns by 10.5 degrees when camera 2 comes
    first, and not at all otherwise), the pairs of cameras 0 and 1 are exact:
    errors {0, 0, 10.5 x 4}, so AUC@30 = (10 * 2/6 + 20 * 6/6) / 30 = 7/9."""
    R = np.stack([np.eye(3)] * 3)
    t = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    Rp = R.copy()
    Rp[2] = Rotation.from_rotvec([0, 0, math.radians(10.5)]).as_matrix()
    a, c = auc.auc30(Rp, t, R, t)
    assert abs(a - 7.0 / 9.0) < 1e-12
    assert c[0] == 2 and c[10] == 4 and c.sum() == 6
    # the conventional metric sees only (0,1), (0,2), (1,2): the same multiset here
    a1, c1 = auc.auc30(Rp, t, R, t, both_orders=False)
    assert c1[0] == 1 and c1[10] == 2 and abs(a1 - 7.0 / 9.0) < 1e-12


def test_head_input_packing_by_index():
    from oracle import heads
    rng = np.random.default_rng(9)
    gh, gw, C2 = 3, 4, 6
    f = rng.normal(0, 1, (2, 3, 5 + gh * gw, C2))
    out = heads.pack_head_inputs(f, gh, gw)
    assert out.shape == (2, 3, C2, gh, gw)
    for l in range(2):
        for s in range(3):
            for c in range(C2):
                for y in range(gh):
                    for x in range(gw):
                        assert out[l, s, c, y, x] == f[l, s, 5 + y * gw + x, c]
