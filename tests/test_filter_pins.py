"""Pins of the FBP sinogram-filter oracle (oracle/filtering.py) against what the
mathematics fixes: the frequency response of Kak & Slaney's band-limited ramp
(ch. 3 eq. 61) is |f| on [-1/2, 1/2] with a small positive DC term, the windows'
values at Nyquist, the FFT route equals a plain truncated circular convolution, and
filtered backprojection of a projected disc gives back the disc (TorchRadon Sec. 3.1.3
uses FBP the same way)."""
import math

import numpy as np
import pytest

import oracle
from oracle import filtering
from paper_2009_14788_amd import inputs


@pytest.mark.parametrize("D", [23, 91, 363, 725])
def test_ramp_response_is_abs_frequency(D):
    L = filtering.padded_length(D)
    assert L >= 2 * D and L & (L - 1) == 0
    H = filtering.frequency_response("ram-lak", D)
    f = np.abs(np.fft.fftfreq(L))
    mid = (f >= 0.05) & (f <= 0.45)
    # the infinite kernel's transform is exactly |f|; truncation to L costs O(1/L)
    assert np.max(np.abs(H[mid] - f[mid])) < 2.0 / L
    # DC: positive and O(1/L) (sampling |f| directly would give exactly 0)
    assert 0.0 < H[0] < 1.0 / L
    # real and even
    assert np.allclose(H[1:], H[1:][::-1], atol=1e-15)


def test_windows_at_nyquist_and_dc():
    D = 100
    L = filtering.padded_length(D)
    ramp = filtering.frequency_response("ram-lak", D)
    ny = L // 2                                 # fftfreq gives -1/2 here
    for name, at_ny in [("ram-lak", 1.0), ("shepp-logan", 2.0 / math.pi), ("cosine", 0.0),
                        ("hamming", 0.08), ("hann", 0.0)]:
        H = filtering.frequency_response(name, D)
        assert abs(H[ny] - at_ny * ramp[ny]) < 1e-12, name
        assert abs(H[0] - ramp[0]) < 1e-15, name      # every window is 1 at DC
    with pytest.raises(ValueError):
        filtering.frequency_response("ramp", D)


@pytest.mark.parametrize("name", filtering.FILTERS)
def test_fft_route_equals_direct_convolution(name):
    rng = np.random.default_rng(3)
    y = rng.standard_normal((2, 7, 41))
    a = filtering.filter_sinogram(y, name)
    b = filtering.filter_sinogram_direct(y, name)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("sp", [1.0, 0.5, 0.7])
def test_fbp_reconstructs_disc(sp):
    """Project a disc (area-sampled), filter, backproject: the interior comes back at
    the disc's intensity and the outside at zero (parallel beam over [0, pi)), at bin
    spacing 1, 0.5 and 0.7 (the detector covers the image in every case)."""
    n, A = 96, 180
    D = int(math.ceil(n * math.sqrt(2) / sp))
    R, rho = 30.0, 1.0
    yy, xx = np.mgrid[0:n, 0:n] - 0.5 * (n - 1)
    m = 8
    off = (np.arange(m) + 0.5) / m - 0.5
    img = np.zeros((n, n))
    for dy in off:
        for dx in off:
            img += ((xx + dx) ** 2 + (yy + dy) ** 2 < R * R)
    img *= rho / (m * m)
    ang = inputs.uniform_angles(A)
    g = oracle.Geometry(n, ang, D, sp)
    y = oracle.forward(g, img[None])
    rec = oracle.backproject(g, filtering.filter_sinogram(y, "ram-lak"))[0]
    r = np.hypot(xx, yy)
    inner, outer = r < R - 4, (r > R + 4) & (r < 0.5 * n - 4)
    assert abs(rec[inner].mean() - rho) < 0.02
    assert np.abs(rec[inner] - rho).max() < 0.08
    assert np.abs(rec[outer]).mean() < 0.01
    # a wrong angular weight is caught, and so is a filter that divides by the bin
    # spacing once more (the transpose already gathers 1/spacing bins per unit length)
    rec2 = oracle.backproject(g, 0.5 * filtering.filter_sinogram(y, "ram-lak"))[0]
    assert abs(rec2[inner].mean() - rho) > 0.4
    if sp != 1.0:
        rec3 = oracle.backproject(g, filtering.filter_sinogram(y, "ram-lak") / sp)[0]
        assert abs(rec3[inner].mean() - rho) > 0.3
    # smoother windows trade resolution for noise but keep the level
    for name in ("shepp-logan", "hann"):
        recw = oracle.backproject(g, filtering.filter_sinogram(y, name))[0]
        assert abs(recw[inner].mean() - rho) < 0.03, name
