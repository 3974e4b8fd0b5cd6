"""FP64 oracle of the alpha-shearlet transform (TEST INFRASTRUCTURE ONLY: imported by
the tests, the smoke check and the benchmark's CPU leg; the product library never
imports it and it imports nothing from the library).

The paper (TorchRadon, arXiv 2009.14788) lists an alpha-shearlet transform among its
GPU routines (Sec. 2.1) and compares it with the AlphaTransforms library (Sec. 3.2):
real-valued alpha-shearlets with alpha = 0.5 and 5 scales, normalised on the Fourier
side to a Parseval frame (the adjoint of the transform inverts it), 59 coefficient
channels for a 512 x 512 image, Fourier coefficients computed once and every later
step a product in the frequency domain.  It prints no construction; AlphaTransforms
(absent here) holds one.  This oracle builds a Parseval alpha-shearlet system from the
published ingredients of the cone-adapted alpha-shearlet construction, so parity with
AlphaTransforms' own coefficients stays unpinned; the frame properties are pinned.

Frequencies: the discrete Fourier grid of an H x W image, xi_1 = column frequency,
xi_2 = row frequency, in cycles per sample, in [-1/2, 1/2) (numpy.fft.fftfreq).

  nu(t)       smooth step, 0 for t <= 0, 1 for t >= 1, nu(t) + nu(1 - t) = 1
              (the polynomial t^4 (35 - 84 t + 70 t^2 - 20 t^3));
  phi(r)      low-pass profile: 1 for r <= c, cos(pi/2 nu(r/c - 1)) on [c, 2c], 0 beyond,
              with c = 2^-(J+1) for J scales (the finest band reaches the Nyquist edge);
  r           = max(|xi_1|, |xi_2|)  (the cone-adapted radial variable);
  W_j(r)^2    = phi(r / 2^(j+1))^2 - phi(r / 2^j)^2  for scales j = 0 .. J-2, and
  W_{J-1}^2   = 1 - phi(r / 2^(J-1))^2  (the finest band keeps everything beyond);
  cones       horizontal |xi_2| <= |xi_1| with slope t = xi_2 / xi_1, vertical
              |xi_1| < |xi_2| with slope t = xi_1 / xi_2, t in [-1, 1];
  shears      K_j = ceil(2^(j (1 - alpha_j))) per scale (the alpha-scaling: the angular
              width at radius 2^j is 2^(alpha j)), shear k = -K_j .. K_j in each cone;
  V(u)        angular window cos(pi/2 nu(|u|)) for |u| <= 1, 0 beyond, so that
              sum_k V(u - k)^2 = 1;
  psi_{j,cone,k}(xi) = W_j(r) V(K_j t - k) [xi in cone];   psi_low(xi) = phi(r).

Then phi^2 + sum over scales, cones and shears of psi^2 = 1 at every frequency (the
Parseval identity); every psi is real, even in xi and >= 0, so each channel's
coefficients c_m = IFFT2(FFT2(x) psi_m) are real.  On the grid of an even size the
Nyquist row and column have no mirror frequency, so each filter is symmetrised there,
psi_m[k] <- sqrt((psi_m[k]^2 + psi_m[-k]^2) / 2), which keeps the identity exactly.
Channel order: the low-pass, then per scale the horizontal cone's shears k = -K..K and
the vertical cone's shears k = -K..K.  `scales` gives each channel's scale: 0 for the
low-pass and j + 1 for scale j.

  forward   c[..., m, :, :] = Re IFFT2(FFT2(x) psi_m)
  adjoint   x = Re IFFT2(sum_m FFT2(c_m) psi_m)       (adjoint(forward(x)) = x)
"""
import math

import numpy as np


def smooth_step(t):
    """nu(t): 0 for t <= 0, 1 for t >= 1, and nu(t) + nu(1 - t) = 1."""
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, 1.0)
    return t ** 4 * (35.0 - 84.0 * t + 70.0 * t ** 2 - 20.0 * t ** 3)


def low_pass(r, c):
    """phi(r) with plateau [0, c] and zero beyond 2c."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r <= c, 1.0, np.where(r >= 2 * c, 0.0, np.cos(0.5 * np.pi * smooth_step(r / c - 1.0))))


def angular_window(u):
    """V(u) = cos(pi/2 nu(|u|)) on [-1, 1], 0 beyond."""
    a = np.abs(np.asarray(u, dtype=np.float64))
    return np.where(a >= 1.0, 0.0, np.cos(0.5 * np.pi * smooth_step(a)))


def shears_per_scale(alphas):
    """K_j = ceil(2^(j (1 - alpha_j))) for each scale j."""
    return [int(math.ceil(2.0 ** (j * (1.0 - float(a))) - 1e-12)) for j, a in enumerate(alphas)]


def channel_count(alphas):
    return 1 + sum(2 * (2 * k + 1) for k in shears_per_scale(alphas))


def scales(alphas):
    """Scale of every channel: 0 for the low-pass, j + 1 for the channels of scale j."""
    out = [0]
    for j, k in enumerate(shears_per_scale(alphas)):
        out += [j + 1] * (2 * (2 * k + 1))
    return np.asarray(out, dtype=np.int64)


def filters(width, height, alphas):
    """psi_m on the FFT grid: array [M][height][width] (FP64), M = channel_count."""
    J = len(alphas)
    if J < 1:
        raise ValueError("at least one scale")
    x1 = np.fft.fftfreq(width)[None, :]
    x2 = np.fft.fftfreq(height)[:, None]
    a1, a2 = np.abs(x1) + 0 * x2, np.abs(x2) + 0 * x1
    r = np.maximum(a1, a2)
    c = 2.0 ** -(J + 1)
    horiz = a2 <= a1
    with np.errstate(divide="ignore", invalid="ignore"):
        t_h = np.where(a1 > 0, (x2 + 0 * x1) / (x1 + 0 * x2), 0.0)
        t_v = np.where(a2 > 0, (x1 + 0 * x2) / (x2 + 0 * x1), 0.0)
    out = [low_pass(r, c)]
    for j, K in enumerate(shears_per_scale(alphas)):
        if j < J - 1:
            w2 = low_pass(r / 2.0 ** (j + 1), c) ** 2 - low_pass(r / 2.0 ** j, c) ** 2
        else:
            w2 = 1.0 - low_pass(r / 2.0 ** j, c) ** 2
        W = np.sqrt(np.maximum(w2, 0.0))
        for cone, t in ((horiz, t_h), (~horiz, t_v)):
            for k in range(-K, K + 1):
                out.append(W * angular_window(K * t - k) * cone)
    psi = np.stack(out)
    # symmetrise under xi -> -xi (only the Nyquist row / column change)
    mirror = psi[:, (-np.arange(height)) % height][:, :, (-np.arange(width)) % width]
    return np.sqrt(0.5 * (psi ** 2 + mirror ** 2))


def forward(x, psi):
    """Coefficients c[..., M, H, W] of real images x[..., H, W]."""
    X = np.fft.fft2(np.asarray(x, dtype=np.float64))
    return np.real(np.fft.ifft2(X[..., None, :, :] * psi))


def adjoint(c, psi):
    """Adjoint of forward: x[..., H, W] from c[..., M, H, W]."""
    C = np.fft.fft2(np.asarray(c, dtype=np.float64))
    return np.real(np.fft.ifft2(np.sum(C * psi, axis=-3)))
