"""FP64 oracle of the sinogram filter of filtered backprojection (TEST INFRASTRUCTURE
ONLY: imported by the tests, the smoke check and the benchmark's CPU leg; the product
library never imports it and it imports nothing from the library).

The paper (TorchRadon, arXiv 2009.14788, Sec. 3.1.3 "Filtered Backprojection") filters
each projection in the frequency domain with one of five filters (Ram-Lak, Shepp-Logan,
cosine, Hamming, Hann) and builds the Fourier filter as Kak & Slaney, Principles of
Computerized Tomographic Imaging, ch. 3, eq. 61 prescribe: the ramp is not sampled in
frequency but obtained as the transform of the band-limited ramp's sampled impulse
response

    h(0) = 1/(4 tau^2),   h(n tau) = 0 (n even),   h(n tau) = -1/(n^2 pi^2 tau^2) (n odd),

with each projection zero-padded so the circular convolution equals the linear one.
The filtered projection is Q(n tau) = tau * sum_k h(n tau - k tau) p(k tau), and the
reconstruction f = (pi / K) * sum over the K angles of Q interpolated at x cos t +
y sin t (ch. 3, the discrete form of the parallel-beam FBP).

Readings (the paper names the filters but gives no formulas):
  * padded length L = the smallest power of two >= max(64, 2 D);
  * the windows multiply the ramp's transform at the normalised frequency f in
    [-1/2, 1/2) (numpy's fftfreq): Shepp-Logan sin(pi f)/(pi f), cosine cos(pi f),
    Hamming 0.54 + 0.46 cos(2 pi f), Hann 0.5 + 0.5 cos(2 pi f), Ram-Lak 1;
  * filter_sinogram returns (pi / A) * tau * Q for A angles and bin spacing tau, so that
    the exact transpose of the projector applied to it reconstructs the image when the
    angles cover [0, pi) uniformly (the paper's example backprojects the filtered
    sinogram directly).  The transpose gathers the rays through a pixel at a density
    of 1/tau bins per unit of detector length (its weights of one angle sum to 1/tau
    over the detector for a smooth projection), which is the 1/tau that Q's kernel
    carries, so the result no longer depends on tau:
    (pi / A) * tau * Q = (pi / A) * sum_k h_1(n - k) p(k tau), h_1 = h at tau = 1.
"""
import numpy as np

FILTERS = ("ram-lak", "shepp-logan", "cosine", "hamming", "hann")


def padded_length(det_count):
    """Smallest power of two >= max(64, 2 D)."""
    n = 64
    while n < 2 * det_count:
        n *= 2
    return n


def ramp_impulse(L):
    """Kak & Slaney ch. 3 eq. 61 impulse response (tau = 1), wrapped onto [0, L):
    entry n holds h at the signed offset n (n <= L/2) or n - L."""
    n = np.arange(L)
    off = np.where(n <= L // 2, n, n - L).astype(np.float64)
    h = np.zeros(L)
    h[0] = 0.25
    odd = (np.abs(off) % 2) == 1
    h[odd] = -1.0 / (np.pi ** 2 * off[odd] ** 2)
    return h


def window(name, L):
    """Window of filter `name` at the FFT frequencies of length L."""
    f = np.fft.fftfreq(L)
    if name == "ram-lak":
        return np.ones(L)
    if name == "shepp-logan":
        w = np.ones(L)
        nz = f != 0
        w[nz] = np.sin(np.pi * f[nz]) / (np.pi * f[nz])
        return w
    if name == "cosine":
        return np.cos(np.pi * f)
    if name == "hamming":
        return 0.54 + 0.46 * np.cos(2 * np.pi * f)
    if name == "hann":
        return 0.5 + 0.5 * np.cos(2 * np.pi * f)
    raise ValueError(f"unknown filter {name!r}; one of {FILTERS}")


def frequency_response(name, det_count):
    """Real filter H[k] of length L = padded_length(D): transform of the wrapped ramp
    impulse response times the window."""
    L = padded_length(det_count)
    return np.real(np.fft.fft(ramp_impulse(L))) * window(name, L)


def filter_sinogram(y, name="ram-lak"):
    """(pi / A) * tau * Q for every projection of y[..., A, D] (FP64): zero-pad each row
    to L, multiply its transform by H (the kernel at tau = 1), transform back, keep the
    first D samples, times pi / A.  Independent of the bin spacing tau."""
    y = np.asarray(y, dtype=np.float64)
    A, D = y.shape[-2], y.shape[-1]
    L = padded_length(D)
    H = frequency_response(name, D)
    P = np.fft.fft(y, n=L, axis=-1)
    Q = np.real(np.fft.ifft(P * H, axis=-1))[..., :D]
    return Q * (np.pi / A)


def filter_sinogram_direct(y, name="ram-lak"):
    """The same filter as a plain truncated circular convolution with the spatial
    kernel g = inverse transform of H (only for small cases: O(D^2) per row)."""
    y = np.asarray(y, dtype=np.float64)
    A, D = y.shape[-2], y.shape[-1]
    L = padded_length(D)
    g = np.real(np.fft.ifft(frequency_response(name, D)))
    n = np.arange(D)
    T = g[(n[:, None] - n[None, :]) % L]          # Q[n] = sum_k g[(n - k) mod L] p[k]
    return (y @ T.T) * (np.pi / A)
