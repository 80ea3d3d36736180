"""Pins of the SSIM oracle (the SSIM term of Eq. (9)): the window sums
against a brute-force per-pixel definition, SSIM(x, x) = 1, and the
hand-derived gradient against torch autograd of a conv2d implementation
in float64 on the CPU."""
import math

import numpy as np
import pytest

from oracle import ssim as S


def _brute_ssim_map(x, y):
    g = S.window()
    w2 = np.outer(g, g)
    H, W = x.shape
    r = S.WIN // 2
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            acc = np.zeros(5)
            for a in range(-r, r + 1):
                for b in range(-r, r + 1):
                    ii, jj = i + a, j + b
                    if 0 <= ii < H and 0 <= jj < W:
                        wgt = w2[a + r, b + r]
                        acc += wgt * np.array([x[ii, jj], y[ii, jj], x[ii, jj] ** 2,
                                               y[ii, jj] ** 2, x[ii, jj] * y[ii, jj]])
            mx, my, exx, eyy, exy = acc
            sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
            out[i, j] = ((2 * mx * my + S.C1) * (2 * sxy + S.C2)) / \
                        ((mx * mx + my * my + S.C1) * (sxx + syy + S.C2))
    return out


def test_window_is_normalised_gaussian():
    g = S.window()
    assert abs(g.sum() - 1) < 1e-15
    assert abs(g[6] / g[5] - math.exp(-1 / (2 * 1.5 ** 2))) < 1e-14


def test_ssim_map_matches_brute_force():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(size=(13, 17)), rng.uniform(size=(13, 17))
    got, _ = S.ssim_terms(x, y)
    np.testing.assert_allclose(got, _brute_ssim_map(x, y), rtol=1e-12, atol=1e-14)


def test_ssim_of_identical_images_is_one():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 20, 24))
    assert abs(S.ssim(x, x) - 1.0) < 1e-12
    np.testing.assert_allclose(S.ssim_grad(x, x), 0.0, atol=1e-12)


def test_ssim_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    rng = np.random.default_rng(2)
    x, y = rng.uniform(size=(3, 19, 23)), rng.uniform(size=(3, 19, 23))
    g = torch.tensor(S.window())
    w = (g[:, None] * g[None, :]).expand(3, 1, 11, 11).contiguous()
    tx = torch.tensor(x[None], requires_grad=True)
    ty = torch.tensor(y[None])
    conv = lambda a: F.conv2d(a, w, padding=5, groups=3)
    mx, my = conv(tx), conv(ty)
    sxx, syy, sxy = conv(tx * tx) - mx * mx, conv(ty * ty) - my * my, conv(tx * ty) - mx * my
    smap = ((2 * mx * my + S.C1) * (2 * sxy + S.C2)) / ((mx * mx + my * my + S.C1) * (sxx + syy + S.C2))
    smap.mean().backward()
    assert abs(S.ssim(x, y) - smap.mean().item()) < 1e-13
    np.testing.assert_allclose(S.ssim_grad(x, y), tx.grad.numpy()[0], rtol=1e-9, atol=1e-15)


def test_rendered_loss_combines_terms():
    rng = np.random.default_rng(3)
    C, T = rng.uniform(size=(3, 8, 9)), rng.uniform(size=(3, 8, 9))
    D, Dt = rng.uniform(1, 2, (8, 9)), rng.uniform(1, 2, (8, 9))
    L, gC, gD = S.rendered_loss_and_grads(C, D, T, Dt, 0.2, 0.1)
    ref = 0.8 * np.abs(C - T).mean() + 0.2 * (1 - S.ssim(C, T)) + 0.1 * np.abs(D - Dt).mean()
    assert abs(L - ref) < 1e-14
    # directional finite difference of the total loss
    u = rng.standard_normal(C.shape)
    h = 1e-7
    Lp = S.rendered_loss_and_grads(C + h * u, D, T, Dt, 0.2, 0.1)[0]
    Lm = S.rendered_loss_and_grads(C - h * u, D, T, Dt, 0.2, 0.1)[0]
    assert abs((Lp - Lm) / (2 * h) - float((gC * u).sum())) < 1e-6
