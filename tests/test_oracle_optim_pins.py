"""Pins of the FP64 Adam oracle: torch.optim.Adam (a library routine) for the linear case over
several steps, the closed form of a constant gradient (each bias-corrected step moves by
lr * g / (|g| + eps)), and the log and logit parametrisations against those closed forms in u."""
import numpy as np
import torch

from oracle import optim as OO


def test_linear_matches_torch_adam():
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal(200)
    grads = [rng.standard_normal(200) for _ in range(5)]
    p = torch.nn.Parameter(torch.tensor(x0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    x, m, v = x0.copy(), np.zeros(200), np.zeros(200)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        x, m, v = OO.adam_step(x, g, m, v, 0.01, OO.LINEAR, t, eps=1e-8)
        np.testing.assert_allclose(x, p.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_constant_gradient_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    x, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        x, m, v = OO.adam_step(x, g, m, v, 0.1, OO.LINEAR, t, eps=1e-15)
        np.testing.assert_allclose(x, -0.1 * t * g / (np.abs(g) + 1e-15), rtol=1e-13)


def test_log_and_logit_parametrisations():
    # a constant gradient in u moves u by lr per step, i.e. x by a factor exp(-lr) (log) or
    # along the logistic curve (logit)
    s0 = np.array([0.01, 2.0])
    x, m, v = s0.copy(), np.zeros(2), np.zeros(2)
    for t in range(1, 4):
        g = 1.0 / x  # du = g * x = 1
        x, m, v = OO.adam_step(x, g, m, v, 0.05, OO.LOG, t)
        np.testing.assert_allclose(x, s0 * np.exp(-0.05 * t), rtol=1e-12)
    o0 = np.array([0.1, 0.7])
    x, m, v = o0.copy(), np.zeros(2), np.zeros(2)
    u0 = np.log(o0 / (1 - o0))
    for t in range(1, 4):
        g = -1.0 / (x * (1 - x))  # du = -1
        x, m, v = OO.adam_step(x, g, m, v, 0.2, OO.LOGIT, t)
        np.testing.assert_allclose(x, 1 / (1 + np.exp(-(u0 + 0.2 * t))), rtol=1e-12)
    # logit clamps its input away from 0 and 1
    x, _, _ = OO.adam_step(np.array([0.0, 1.0]), np.zeros(2), np.zeros(2), np.zeros(2), 0.1, OO.LOGIT, 1)
    np.testing.assert_allclose(x, [1e-6, 1 - 1e-6], rtol=1e-9)
