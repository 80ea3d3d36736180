"""SSIM term of the rendered loss, Eq. (9) -- TEST INFRASTRUCTURE (FP64).

L_rendered = (1 - lambda_ssim) L1 + lambda_ssim (1 - SSIM), with the SSIM
of the 3DGS pipeline the paper retains (Sec. IV-A): per channel, an 11x11
Gaussian window of sigma 1.5 (normalised), zero padding outside the image,
constants C1 = 0.01^2 and C2 = 0.03^2, averaged over pixels and channels.

With m1 = G*x, m2 = G*(x^2), m3 = G*(x y) (y the target), mu_y = G*y,
s_yy = G*(y^2) - mu_y^2:
  A1 = 2 m1 mu_y + C1,  A2 = 2 (m3 - m1 mu_y) + C2,
  B1 = m1^2 + mu_y^2 + C1,  B2 = (m2 - m1^2) + s_yy + C2,  S = A1 A2 / (B1 B2)
and by the chain rule
  dS/dm1 = S (2 mu_y / A1 - 2 mu_y / A2 - 2 m1 / B1 + 2 m1 / B2),
  dS/dm2 = -S / B2,  dS/dm3 = 2 S / A2,
  d mean(S) / dx = (G^T * dS/dm1 + 2 x G^T * dS/dm2 + y G^T * dS/dm3) / N,
where G^T* is the adjoint of the zero-padded window correlation (the window
is symmetric, so it is the same correlation).
"""
from __future__ import annotations

import numpy as np

WIN = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window():
    x = np.arange(WIN, dtype=np.float64) - WIN // 2
    g = np.exp(-(x * x) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def filt(img):
    """Zero-padded 'same' correlation of a [H,W] image with the separable
    11x11 window (rows then columns)."""
    g = window()
    r = WIN // 2
    H, W = img.shape
    p = np.zeros((H + 2 * r, W + 2 * r))
    p[r:r + H, r:r + W] = img
    tmp = np.zeros((H + 2 * r, W))
    for k in range(WIN):
        tmp += g[k] * p[:, k:k + W]
    out = np.zeros((H, W))
    for k in range(WIN):
        out += g[k] * tmp[k:k + H, :]
    return out


def ssim_terms(x, y):
    mu_y = filt(y)
    syy = filt(y * y) - mu_y * mu_y
    m1, m2, m3 = filt(x), filt(x * x), filt(x * y)
    A1 = 2 * m1 * mu_y + C1
    A2 = 2 * (m3 - m1 * mu_y) + C2
    B1 = m1 * m1 + mu_y * mu_y + C1
    B2 = (m2 - m1 * m1) + syy + C2
    S = A1 * A2 / (B1 * B2)
    return S, (A1, A2, B1, B2, m1, mu_y)


def ssim(color, target):
    """Mean SSIM over channels and pixels of [C,H,W] images."""
    return float(np.mean([ssim_terms(np.asarray(color[c], np.float64),
                                     np.asarray(target[c], np.float64))[0].mean()
                          for c in range(color.shape[0])]))


def ssim_grad(color, target):
    """d mean(SSIM) / d color for [C,H,W] images."""
    C, H, W = color.shape
    N = C * H * W
    out = np.zeros((C, H, W))
    for c in range(C):
        x = np.asarray(color[c], np.float64)
        y = np.asarray(target[c], np.float64)
        S, (A1, A2, B1, B2, m1, mu_y) = ssim_terms(x, y)
        d1 = S * (2 * mu_y / A1 - 2 * mu_y / A2 - 2 * m1 / B1 + 2 * m1 / B2)
        d2 = -S / B2
        d3 = 2 * S / A2
        out[c] = (filt(d1) + 2 * x * filt(d2) + y * filt(d3)) / N
    return out


def rendered_loss_and_grads(color, depth, target_rgb, target_depth, lambda_ssim, lambda_depth):
    """Eq. (9) with the depth term of the RGB-D workloads:
    L = (1 - ls) mean|C - C*| + ls (1 - SSIM(C, C*)) + ld mean|D - D*|;
    returns (L, dL/dC, dL/dD), sign(0) = 0."""
    color = np.asarray(color, np.float64)
    tr = np.asarray(target_rgb, np.float64)
    npx = color.shape[1] * color.shape[2]
    d = color - tr
    loss = (1 - lambda_ssim) * np.abs(d).sum() / (3.0 * npx)
    gC = (1 - lambda_ssim) * np.sign(d) / (3.0 * npx)
    if lambda_ssim != 0.0:
        loss += lambda_ssim * (1.0 - ssim(color, tr))
        gC = gC - lambda_ssim * ssim_grad(color, tr)
    gD = np.zeros(color.shape[1:])
    if target_depth is not None and lambda_depth != 0.0:
        dd = np.asarray(depth, np.float64) - np.asarray(target_depth, np.float64)
        loss += lambda_depth * np.abs(dd).sum() / npx
        gD = lambda_depth * np.sign(dd) / npx
    return float(loss), gC, gD
