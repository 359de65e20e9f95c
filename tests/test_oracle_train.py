"""Pins of the oracle's training-step pieces (the 3DGS loss and optimiser the paper trains with,
Appendix, experimental details): the SSIM map against explicit window sums, the closed forms of
SSIM, finite differences of the loss, and Adam's first step."""
import numpy as np

from oracle import oracle as O


def test_ssim_map_matches_explicit_window_sums():
    rng = np.random.default_rng(120)
    x = rng.uniform(size=(3, 13, 17))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    import torch
    import torch.nn.functional as F
    g = torch.from_numpy(O.gaussian_window())
    win = torch.outer(g, g)[None, None]
    conv = lambda t: F.conv2d(torch.from_numpy(t)[:, None], win, padding=5)[:, 0].numpy()
    mx, my = conv(x), conv(y)
    s = ((2 * mx * my + O.SSIM_C1) * (2 * (conv(x * y) - mx * my) + O.SSIM_C2)) / \
        ((mx * mx + my * my + O.SSIM_C1) * (conv(x * x) - mx * mx + conv(y * y) - my * my + O.SSIM_C2))
    for c in range(3):
        np.testing.assert_allclose(s[c], O.ssim_map_direct(x[c], y[c]), rtol=1e-12, atol=1e-14)
    # and the loss built on it
    L, _ = O.photometric_loss([x], [y], lam=1.0)
    direct = 1 - np.mean([O.ssim_map_direct(x[c], y[c]) for c in range(3)])
    np.testing.assert_allclose(L, direct, rtol=1e-12)


def test_window_and_closed_forms():
    g = O.gaussian_window()
    assert len(g) == 11 and abs(g.sum() - 1) < 1e-15 and np.argmax(g) == 5
    np.testing.assert_allclose(g[4] / g[5], np.exp(-1 / (2 * 1.5 ** 2)), rtol=1e-14)
    rng = np.random.default_rng(121)
    x = rng.uniform(size=(3, 12, 12))
    L, gr = O.photometric_loss([x], [x])
    assert abs(L) < 1e-15 and np.abs(gr[0]).max() < 1e-12      # SSIM(x, x) = 1, its maximum
    # constant images a and b: away from the border SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    s = O.ssim_map_direct(np.full((30, 30), a), np.full((30, 30), b))
    np.testing.assert_allclose(s[10:20, 10:20], (2 * a * b + O.SSIM_C1) / (a * a + b * b + O.SSIM_C1), rtol=1e-12)
    # L1 part alone
    y = x + 0.05
    L, gr = O.photometric_loss([x], [y], lam=0.0)
    np.testing.assert_allclose(L, 0.05, rtol=1e-12)
    np.testing.assert_allclose(gr[0], -1.0 / x.size, rtol=1e-12)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(122)
    xs = [rng.uniform(size=(3, 9, 14)), rng.uniform(size=(3, 12, 8))]
    ys = [np.clip(x + rng.normal(0, 0.2, size=x.shape), 0, 1) for x in xs]
    L, grads = O.photometric_loss(xs, ys)
    h = 1e-6
    for v in range(2):
        for _ in range(12):
            idx = tuple(int(rng.integers(0, s)) for s in xs[v].shape)
            xp = [x.copy() for x in xs]; xp[v][idx] += h
            xm = [x.copy() for x in xs]; xm[v][idx] -= h
            fd = (O.photometric_loss(xp, ys)[0] - O.photometric_loss(xm, ys)[0]) / (2 * h)
            np.testing.assert_allclose(grads[v][idx], fd, rtol=1e-5, atol=1e-10)


def test_adam_first_steps():
    """Step 1 moves every parameter by lr sign(g) (up to eps); a constant gradient keeps moving
    it by lr per step, because the bias corrections cancel the moment decay exactly."""
    rng = np.random.default_rng(123)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    p1, m, v = O.adam_step(p, g, np.zeros(100), np.zeros(100), 1e-3, 0.9, 0.999, 1e-15, 1)
    np.testing.assert_allclose(p1, p - 1e-3 * np.sign(g), rtol=1e-12)
    p2, _, _ = O.adam_step(p1, g, m, v, 1e-3, 0.9, 0.999, 1e-15, 2)
    np.testing.assert_allclose(p2, p - 2e-3 * np.sign(g), rtol=1e-12)
