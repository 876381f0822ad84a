"""FP64 training loss of the point representation (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module. The distillation loss of Sec. 3.2 weighs a squared-error term against a structural
similarity term with lambda = 0.2:

    L = (1 - lambda) mean((x - y)^2) + lambda (1 - SSIM(x, y))

x is the rendered image, y the target; both are stacks of planes [P][H][W] (the three
colour planes of one or more views). Every sum is divided by n, the number of elements
the mean runs over (x.size by default): a batch of views of different sizes is the sum
of per-view calls that all pass the batch's total element count. Readings of the paper's loss (it writes the second
term as lambda SSIM, which would reward dissimilarity, so it is read as the usual D-SSIM
term 1 - SSIM): the squared error is the mean over all planes and pixels; SSIM is the
mean over all planes and pixels of the SSIM map of Wang et al. with an 11 x 11 Gaussian
window of standard deviation 1.5, C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1), local
statistics taken with zero padding outside the image.

The SSIM map is written from its definition: local means, variances and covariance are
window-weighted sums (scipy's 2D correlation, a library primitive), and the gradient is
the exact chain rule through those sums.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import correlate2d

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """Normalised 2D Gaussian window (outer product of the normalised 1D profile)."""
    k = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _filt(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Window-weighted local sum at every pixel, zero outside the image."""
    return correlate2d(img, w, mode="same", boundary="fill", fillvalue=0.0)


def _moments(x: np.ndarray, y: np.ndarray, w: np.ndarray):
    mx, my = _filt(x, w), _filt(y, w)
    exx, eyy, exy = _filt(x * x, w), _filt(y * y, w), _filt(x * y, w)
    return mx, my, exx - mx * mx, eyy - my * my, exy - mx * my, exx, exy


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM at every pixel of every plane, [P][H][W]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w = window()
    out = np.empty_like(x)
    for p in range(x.shape[0]):
        mx, my, vx, vy, cxy, _, _ = _moments(x[p], y[p], w)
        out[p] = ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    return out


def ssim(x: np.ndarray, y: np.ndarray) -> float:
    return float(ssim_map(x, y).mean())


def loss(x: np.ndarray, y: np.ndarray, lam: float = 0.2, n=None) -> float:
    """(1 - lam) sum (x - y)^2 / n + lam sum (1 - SSIM map) / n."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.size if n is None else n
    return ((1.0 - lam) * float(np.sum((x - y) ** 2)) + lam * float(np.sum(1.0 - ssim_map(x, y)))) / n


def loss_grad(x: np.ndarray, y: np.ndarray, lam: float = 0.2, n=None) -> np.ndarray:
    """dL/dx, [P][H][W]. With A1 = 2 mx my + C1, A2 = 2 cxy + C2, B1 = mx^2 + my^2 + C1,
    B2 = vx + vy + C2 and S = A1 A2 / (B1 B2), S depends on x through mx, exx = <x^2> and
    exy = <x y>: dS/dmx = (2 my A2 - 2 my A1 - S (2 mx B2 - 2 mx B1)) / (B1 B2),
    dS/dexx = -S / B2, dS/dexy = 2 A1 / (B1 B2); each local sum is a window correlation, so
    its adjoint is a correlation with the flipped (here identical) window."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w = window()
    m = x.size if n is None else n
    g = np.empty_like(x)
    for p in range(x.shape[0]):
        mx, my, vx, vy, cxy, _, _ = _moments(x[p], y[p], w)
        a1, a2 = 2 * mx * my + C1, 2 * cxy + C2
        b1, b2 = mx * mx + my * my + C1, vx + vy + C2
        s = a1 * a2 / (b1 * b2)
        d_mx = (2 * my * a2 - 2 * my * a1 - s * (2 * mx * b2 - 2 * mx * b1)) / (b1 * b2)
        d_exx = -s / b2
        d_exy = 2 * a1 / (b1 * b2)
        w_flip = w[::-1, ::-1]
        dssim = (_filt(d_mx, w_flip) + 2 * x[p] * _filt(d_exx, w_flip) + y[p] * _filt(d_exy, w_flip)) / m
        g[p] = (1.0 - lam) * 2.0 * (x[p] - y[p]) / m - lam * dssim
    return g
