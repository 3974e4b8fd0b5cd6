"""Pins of the alpha-shearlet oracle (oracle/shearlets.py) against what the paper and
the mathematics fix (TorchRadon Sec. 3.2: real-valued alpha-shearlets, alpha = 0.5,
5 scales, a Parseval frame on the Fourier side, 59 channels at 512 x 512):

* the channel count and the shears per scale of the alpha-scaling;
* the Parseval identity sum_m psi_m^2 = 1 at every frequency (1e-12), and with it
  ||forward(x)|| = ||x|| and adjoint(forward(x)) = x;
* Hermitian symmetry of every filter, so the coefficients of a real image are real;
* adjointness <forward(x), c> = <x, adjoint(c)>;
* the FFT route against a brute-force circular convolution with each channel's
  spatial filter, built from an explicit DFT matrix (no FFT);
* the construction's own partitions of unity (angular windows, radial bands) and its
  90-degree symmetry (vertical-cone filters are the horizontal ones transposed).
Parity with AlphaTransforms' own coefficients is unpinned (the library is absent)."""
import numpy as np
import pytest

from oracle import shearlets as sh


def test_channel_count_matches_paper():
    alphas = [0.5] * 5
    assert sh.shears_per_scale(alphas) == [1, 2, 2, 3, 4]
    assert sh.channel_count(alphas) == 59
    s = sh.scales(alphas)
    assert s.shape == (59,) and s[0] == 0
    assert [int((s == j + 1).sum()) for j in range(5)] == [6, 10, 10, 14, 18]
    # alpha = 1 is wavelet-like (one shear pair per cone), alpha = 0 doubles the
    # shears at every scale (the ridgelet end of the alpha-scale)
    assert sh.shears_per_scale([1.0] * 4) == [1, 1, 1, 1]
    assert sh.shears_per_scale([0.0] * 4) == [1, 2, 4, 8]


@pytest.mark.parametrize("w,h,alphas", [(512, 512, [0.5] * 5), (64, 64, [0.5] * 3),
                                        (96, 40, [0.5, 0.5, 0.25]), (33, 17, [0.5, 0.5])])
def test_parseval_identity(w, h, alphas):
    psi = sh.filters(w, h, alphas)
    assert psi.shape == (sh.channel_count(alphas), h, w)
    assert np.all(psi >= 0.0)
    assert np.max(np.abs(np.sum(psi ** 2, axis=0) - 1.0)) < 1e-12


@pytest.mark.parametrize("w,h", [(64, 64), (48, 80), (31, 20)])
def test_hermitian_symmetry_real_coefficients(w, h):
    psi = sh.filters(w, h, [0.5] * 3)
    mirror = psi[:, (-np.arange(h)) % h][:, :, (-np.arange(w)) % w]
    assert np.array_equal(psi, mirror)
    x = np.random.default_rng(1).standard_normal((h, w))
    full = np.fft.ifft2(np.fft.fft2(x)[None] * psi)
    assert np.max(np.abs(full.imag)) < 1e-13 * np.max(np.abs(full.real))


def test_frame_is_tight_and_inverted_by_its_adjoint():
    rng = np.random.default_rng(2)
    psi = sh.filters(128, 128, [0.5] * 4)
    x = rng.standard_normal((3, 128, 128))
    c = sh.forward(x, psi)
    assert c.shape == (3, psi.shape[0], 128, 128)
    assert abs(np.sum(c ** 2) - np.sum(x ** 2)) < 1e-12 * np.sum(x ** 2)
    rec = sh.adjoint(c, psi)
    assert np.linalg.norm(rec - x) < 1e-13 * np.linalg.norm(x)
    # adjointness with independent coefficients
    d = rng.standard_normal(c.shape)
    lhs = np.sum(c * d)
    rhs = np.sum(x * sh.adjoint(d, psi))
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)
    # a planted mistake (a channel dropped) breaks the identity
    assert np.linalg.norm(sh.adjoint(c[:, 1:], psi[1:]) - x) > 1e-3 * np.linalg.norm(x)


def test_fft_route_equals_direct_convolution():
    """Brute force on 12 x 16: the spatial filter of each channel from an explicit
    inverse DFT matrix, then a plain circular convolution sum per pixel."""
    h, w = 12, 16
    psi = sh.filters(w, h, [0.5, 0.5])
    x = np.random.default_rng(3).standard_normal((h, w))
    Fh = np.exp(2j * np.pi * np.outer(np.arange(h), np.arange(h)) / h) / h     # inverse DFT
    Fw = np.exp(2j * np.pi * np.outer(np.arange(w), np.arange(w)) / w) / w
    got = sh.forward(x, psi)
    for m in (0, 1, 4, psi.shape[0] - 1):
        g = (Fh @ psi[m] @ Fw.T)          # spatial filter g[r, c]
        assert np.max(np.abs(g.imag)) < 1e-14
        g = g.real
        ref = np.zeros((h, w))
        for r in range(h):
            for cc in range(w):
                s = 0.0
                for a in range(h):
                    for b in range(w):
                        s += x[a, b] * g[(r - a) % h, (cc - b) % w]
                ref[r, cc] = s
        assert np.max(np.abs(got[m] - ref)) < 1e-12 * np.max(np.abs(ref)), m
    # a planted mistake (the row and column frequencies swapped in the grid) fails
    bad = np.transpose(sh.filters(h, w, [0.5, 0.5]), (0, 2, 1))
    assert np.max(np.abs(sh.forward(x, bad)[1] - got[1])) > 1e-3 * np.max(np.abs(got[1]))


def test_construction_partitions_and_rotation():
    # angular windows: sum_k V(u - k)^2 = 1 on [-K, K]
    for K in (1, 2, 3, 4):
        u = np.linspace(-K, K, 4001)
        s = sum(sh.angular_window(u - k) ** 2 for k in range(-K, K + 1))
        assert np.max(np.abs(s - 1.0)) < 1e-14
    t = np.linspace(0, 1, 101)
    assert np.max(np.abs(sh.smooth_step(t) + sh.smooth_step(1 - t) - 1.0)) < 1e-14
    # radial bands telescope: phi^2 + sum_j W_j^2 = 1, each band >= 0, band j zero
    # below c 2^j and (except the finest) beyond c 2^(j+2)
    J, c = 5, 2.0 ** -6
    r = np.linspace(0, 0.5, 5001)
    bands = [sh.low_pass(r / 2 ** (j + 1), c) ** 2 - sh.low_pass(r / 2 ** j, c) ** 2 for j in range(J - 1)]
    bands.append(1 - sh.low_pass(r / 2 ** (J - 1), c) ** 2)
    assert min(b.min() for b in bands) > -1e-15
    assert np.max(np.abs(sh.low_pass(r, c) ** 2 + sum(bands) - 1)) < 1e-14
    for j, b in enumerate(bands):
        assert np.all(b[r < c * 2 ** j] == 0.0)
        if j < J - 1:
            assert np.all(b[r > c * 2 ** (j + 2)] == 0.0)
    # on a square grid the vertical cone's filters are the horizontal ones transposed
    # (off the diagonals |xi_1| = |xi_2|, which belong to the horizontal cone, and
    # inside the symmetrised Nyquist lines)
    alphas = [0.5] * 3
    psi = sh.filters(64, 64, alphas)
    f = np.abs(np.fft.fftfreq(64))
    off = (f[:, None] != f[None, :])[1:, 1:]
    m = 1
    for K in sh.shears_per_scale(alphas):
        n = 2 * K + 1
        for k in range(n):
            h_ = psi[m + k]
            v_ = psi[m + n + k]
            assert np.max(np.abs(v_[1:, 1:] - h_.T[1:, 1:])[off]) < 1e-15
        m += 2 * n
    assert m == psi.shape[0]


def test_low_pass_and_bands_live_where_the_scaling_puts_them():
    """At 512^2 with 5 scales the low-pass is flat to 8 and zero from 16 (integer
    frequencies); scale j's filters vanish below 8 * 2^j; the angular support of a
    shear at scale j spans 2 / K_j in slope."""
    psi = sh.filters(512, 512, [0.5] * 5)
    f = np.abs(np.fft.fftfreq(512) * 512)
    r = np.maximum(f[None, :], f[:, None])
    assert np.all(psi[0][r <= 8] == 1.0) and np.all(psi[0][r >= 16] == 0.0)
    s = sh.scales([0.5] * 5)
    for j in range(5):
        assert np.all(psi[s == j + 1][:, r < 8 * 2 ** j] == 0.0)
    # centre shear (k = 0) of the horizontal cone at scale 4 vanishes for |slope| >= 1/4
    K = 4
    m0 = 1 + sum(2 * (2 * k + 1) for k in sh.shears_per_scale([0.5] * 4)) + K
    fx = np.fft.fftfreq(512)
    with np.errstate(divide="ignore", invalid="ignore"):
        slope = np.abs(fx[:, None] / fx[None, :])
    assert np.all(psi[m0][(slope >= 1.0 / K) & np.isfinite(slope)] == 0.0)
