"""FP64 oracle of the Adam step used to optimise the point representation (TEST
INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this module.
Sec. 3.2 optimises phi = {(p, k, s, o, q)} by gradient descent on its loss; the optimiser is
the one of 3D Gaussian splatting, Adam (Kingma and Ba), which the paper does not restate.
The step follows Adam's definition with bias-corrected moments; a group is optimised in a
parametrisation u of the stored value x: u = x (linear), u = log x (positive scales) or
u = logit x (opacities, x clamped to [1e-6, 1 - 1e-6] first), with du = dx (linear),
dx * x (log) or dx * x * (1 - x) (logit), and x mapped back from the updated u.
"""
from __future__ import annotations

import numpy as np

LINEAR, LOG, LOGIT = 0, 1, 2


def adam_step(x, g, m, v, lr, mode, step, b1=0.9, b2=0.999, eps=1e-15):
    """Returns (x', m', v') in FP64 for one Adam step (step counts from 1)."""
    x = np.asarray(x, np.float64).copy()
    g = np.asarray(g, np.float64)
    if mode == LOG:
        u, du = np.log(x), g * x
    elif mode == LOGIT:
        x = np.clip(x, 1e-6, 1.0 - 1e-6)
        u, du = np.log(x / (1.0 - x)), g * x * (1.0 - x)
    else:
        u, du = x, g
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * du
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * du * du
    m_hat = m / (1.0 - b1 ** step)
    v_hat = v / (1.0 - b2 ** step)
    u = u - lr * m_hat / (np.sqrt(v_hat) + eps)
    if mode == LOG:
        x = np.exp(u)
    elif mode == LOGIT:
        x = 1.0 / (1.0 + np.exp(-u))
    else:
        x = u
    return x, m, v
