"""Pins of the densification / pruning oracle against hand-worked cases."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import densify as D


def _params(n, rng, deg=1):
    k = (deg + 1) ** 2
    return {"means": rng.normal(size=(n, 3)).astype(np.float32),
            "log_scales": rng.normal(-3, 0.5, (n, 3)).astype(np.float32),
            "quats": rng.normal(size=(n, 4)).astype(np.float32),
            "opacity_logits": rng.normal(size=n).astype(np.float32),
            "sh": rng.normal(size=(n, k, 3)).astype(np.float32)}


def test_stats_use_ndc_scaled_norm():
    acc, den = D.accumulate_stats(np.zeros(2), np.zeros(2), np.array([[0.3, 0.4], [1.0, 1.0]]),
                                  [True, False], 200, 100)
    assert abs(acc[0] - math.hypot(0.3 * 100, 0.4 * 50)) < 1e-12 and acc[1] == 0
    np.testing.assert_array_equal(den, [1, 0])


def test_prune_clone_split_hand_worked():
    rng = np.random.default_rng(0)
    P = _params(4, rng)
    P["opacity_logits"][:] = [math.log(0.01 / 0.99), 0.0, 0.0, 0.0]   # first is pruned
    P["log_scales"][2] = math.log(0.005)                                # small -> clone
    P["log_scales"][3] = [math.log(0.5), math.log(0.1), math.log(0.2)]   # large -> split
    M = {f: np.ones_like(x) for f, x in P.items()}
    V = {f: 2 * np.ones_like(x) for f, x in P.items()}
    accum = np.array([1.0, 0.0005, 0.01, 0.01])
    denom = np.array([1.0, 1.0, 1.0, 1.0])
    normals = rng.standard_normal((4, 2, 3))
    out, om, ov = D.densify_prune(P, M, V, accum, denom, normals, 0.001, 0.02, 0.01, 1.0)
    # 0 pruned; 1 kept (below tau_p); 2 cloned; 3 split into two
    assert out["means"].shape[0] == 1 + 2 + 2
    np.testing.assert_array_equal(out["means"][0], P["means"][1])
    np.testing.assert_array_equal(out["means"][1], P["means"][2])
    np.testing.assert_array_equal(out["means"][2], P["means"][2])
    np.testing.assert_array_equal(om["means"][:2], 1.0)
    np.testing.assert_array_equal(om["means"][2:], 0.0)
    np.testing.assert_array_equal(ov["sh"][3:], 0.0)
    q = P["quats"][3].astype(np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    s = np.exp(P["log_scales"][3].astype(np.float64))
    for k in range(2):
        ref = P["means"][3].astype(np.float64) + R @ (s * normals[3, k])
        np.testing.assert_allclose(out["means"][3 + k], ref, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(np.exp(out["log_scales"][3 + k].astype(np.float64)), s / 1.6, rtol=1e-6)
        np.testing.assert_array_equal(out["sh"][3 + k], P["sh"][3])
