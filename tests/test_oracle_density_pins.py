"""Pins of the oracle's folding objective (Experiments, Filament Folding: mean
squared error between the Gaussian-splatted node density at the final step
and a target image).

The reading: the image covers the periodic world, pixel (a, b) centred at
(-1/2 + (a + 1/2) nx/W, -1/2 + (b + 1/2) ny/H); each node adds
amp exp(-r^2 / 2 sigma^2) to the pixels within 5 sigma (minimum image).
Pinned by what the mathematics fixes, independently of the code's formula:
  * a node on a pixel centre: the peak is amp, a neighbour one pixel away
    (spacing h) holds amp e^{-h^2 / 2 sigma^2}, and exactly the pixel centres
    within 5 sigma (counted by integer enumeration) are non-zero;
  * the Riemann sum of a Gaussian sampled at spacing <= sigma is its integral
    2 pi sigma^2 amp / (hx hy) to 1e-5 (truncation e^{-12.5});
  * moving a node by one pixel spacing rolls the image by one pixel; moving
    it by the world period leaves the image unchanged;
  * the loss is 0 at the target, mean(T^2) without nodes;
  * the autograd gradient of the loss equals central differences.
Each pin is run against planted mistakes in the oracle (a pixel centre off by
half a pixel, the Gaussian's 2 sigma^2 written sigma^2, distances not taken
modulo the period), which it must reject.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

DT = torch.float64


def _img(x, nx=64, ny=48, W=32, H=24, sigma=2.0, amp=1.0):
    return O.density_image(torch.tensor(x, dtype=DT).reshape(2, -1), nx, ny, W, H, sigma, amp)


def pin_peak_and_support(image_fn):
    """Node on the centre of pixel (5, 7): peak, neighbour, support count."""
    nx, ny, W, H, sigma, amp = 64, 48, 32, 24, 2.0, 1.7
    hx, hy = nx / W, ny / H
    x = [-0.5 + 5.5 * hx, -0.5 + 7.5 * hy]
    im = image_fn(x, nx, ny, W, H, sigma, amp).numpy()
    assert abs(im[7, 5] - amp) < 1e-12
    assert abs(im[7, 6] - amp * math.exp(-hx * hx / (2 * sigma * sigma))) < 1e-12
    assert abs(im[8, 5] - amp * math.exp(-hy * hy / (2 * sigma * sigma))) < 1e-12
    # the pixel centres within 5 sigma: (i hx)^2 + (j hy)^2 <= 25 sigma^2
    count = sum(1 for i in range(-W, W) for j in range(-H, H)
                if (i * hx) ** 2 + (j * hy) ** 2 <= (5 * sigma) ** 2)
    assert int((im > 0).sum()) == count


def pin_mass(image_fn):
    nx, ny, W, H = 96, 80, 48, 40
    hx, hy = nx / W, ny / H
    for sigma, amp in ((2.0, 1.0), (3.5, 0.4)):
        x = [[10.3, 50.1], [33.7, 5.2]]
        im = image_fn(np.array(x).T.ravel(), nx, ny, W, H, sigma, amp)
        want = 2 * amp * 2 * math.pi * sigma * sigma / (hx * hy)
        assert abs(float(im.sum()) / want - 1) < 1e-5, (sigma, float(im.sum()) / want)


def pin_shift_and_period(image_fn):
    nx, ny, W, H, sigma = 64, 48, 32, 24, 1.5
    hx, hy = nx / W, ny / H
    x = np.array([[3.3, 60.9], [1.2, 46.4]])                  # near the seams
    base = image_fn(x.ravel(), nx, ny, W, H, sigma, 1.0).numpy()
    moved = image_fn((x + np.array([[hx, hx], [0.0, 0.0]])).ravel(), nx, ny, W, H, sigma, 1.0).numpy()
    assert np.max(np.abs(moved - np.roll(base, 1, axis=1))) < 1e-12
    moved = image_fn((x + np.array([[0.0, 0.0], [hy, hy]])).ravel(), nx, ny, W, H, sigma, 1.0).numpy()
    assert np.max(np.abs(moved - np.roll(base, 1, axis=0))) < 1e-12
    wrapped = image_fn((x + np.array([[nx, -nx], [ny, 0]])).ravel(), nx, ny, W, H, sigma, 1.0).numpy()
    assert np.max(np.abs(wrapped - base)) < 1e-9


def _oracle(x, nx, ny, W, H, sigma, amp):
    return O.density_image(torch.tensor(np.asarray(x), dtype=DT).reshape(2, -1), nx, ny, W, H, sigma, amp)


@pytest.mark.parametrize("pin", [pin_peak_and_support, pin_mass, pin_shift_and_period])
def test_density_image_pins(pin):
    pin(_oracle)


def _mistake(kind):
    """The oracle with one planted mistake."""
    def fn(x, nx, ny, W, H, sigma, amp):
        x = torch.tensor(np.asarray(x), dtype=DT).reshape(2, -1)
        cx, cy = O.pixel_centres(nx, ny, W, H)
        if kind == "pixel centre":
            cx, cy = cx - 0.5 * nx / W, cy - 0.5 * ny / H
        dx = x[0][:, None, None] - cx[None, None, :]
        dy = x[1][:, None, None] - cy[None, :, None]
        if kind != "no minimum image":
            dx, dy = O.min_image(dx, nx), O.min_image(dy, ny)
        r2 = dx * dx + dy * dy
        s2 = sigma * sigma if kind == "sigma^2" else 2 * sigma * sigma
        g = amp * torch.exp(-r2 / s2)
        return torch.where(r2 <= (O.SPLAT_CUTOFF * sigma) ** 2, g, torch.zeros_like(g)).sum(0)
    return fn


@pytest.mark.parametrize("kind,pin", [("pixel centre", pin_peak_and_support),
                                      ("sigma^2", pin_mass),
                                      ("no minimum image", pin_shift_and_period)])
def test_planted_mistakes_are_caught(kind, pin):
    with pytest.raises(AssertionError):
        pin(_mistake(kind))


def test_loss_values_and_gradient():
    nx, ny, W, H, sigma = 40, 36, 20, 18, 2.0
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.uniform(0, 36, size=(2, 7)), dtype=DT)
    T = torch.tensor(rng.uniform(0, 1, size=(H, W)), dtype=DT)
    im = O.density_image(x, nx, ny, W, H, sigma)
    assert float(O.density_loss(im, im)) == 0.0
    empty = O.density_image(torch.zeros(2, 0, dtype=DT), nx, ny, W, H, sigma)
    assert abs(float(O.density_loss(empty, T)) - float((T ** 2).mean())) < 1e-15
    xr = x.clone().requires_grad_(True)
    L = O.density_loss(O.density_image(xr, nx, ny, W, H, sigma), T)
    (g,) = torch.autograd.grad(L, xr)
    h = 1e-6
    fd = torch.zeros_like(x)
    for k in range(2):
        for i in range(x.shape[1]):
            xp, xm = x.clone(), x.clone()
            xp[k, i] += h
            xm[k, i] -= h
            fd[k, i] = (O.density_loss(O.density_image(xp, nx, ny, W, H, sigma), T) -
                        O.density_loss(O.density_image(xm, nx, ny, W, H, sigma), T)) / (2 * h)
    assert float((g - fd).abs().max() / fd.abs().max()) < 1e-6
