"""radon_dot_f64_batched_noalloc (for callers that cannot allocate) against
radon_dot_f64_batched, both called through the C ABI on the same device buffers: two
calls in a row, the second on a smaller input, must give bitwise equal FP64 results
(the same kernels and reduction tree; only where the partial sums live differs), and
both must match an FP64 host sum to rounding.  A request beyond the fixed scratch is
rejected with RADON_ERR_SCRATCH.  Runs alone in a fresh process and after the other
GPU tests."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TDT = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _both(lib, a, b, n, batch, code):
    """(noalloc, reference) results of `batch` systems of n elements."""
    out = torch.full((2, max(batch, 1)), float("nan"), dtype=torch.float64, device="cuda")
    rc0 = lib.radon_dot_f64_batched_noalloc(a.data_ptr(), b.data_ptr(), n, batch, code,
                                             out[0].data_ptr(), _stream())
    rc1 = lib.radon_dot_f64_batched(a.data_ptr(), b.data_ptr(), n, batch, code,
                                    out[1].data_ptr(), _stream())
    assert rc0 == 0 and rc1 == 0, (rc0, rc1)
    torch.cuda.synchronize()
    return out[0, :batch].cpu().numpy(), out[1, :batch].cpu().numpy()


@pytest.mark.parametrize("code", [0, 1, 2])
def test_noalloc_dot_matches_allocating_dot(code):
    from paper_2009_14788_amd import _lib
    lib = _lib.lib
    g = torch.Generator(device="cpu").manual_seed(11 + code)
    # first call: 96 systems of 300001 elements (64 partials each: 6144 of 65536);
    # second call: 5 systems of 12345 elements (4 partials each)
    for n, batch in ((300001, 96), (12345, 5)):
        print(f"[gpu-step] noalloc dot dtype {code} n {n} batch {batch}", flush=True)
        a = torch.randn(batch * n, generator=g).to(TDT[code]).cuda()
        b = torch.randn(batch * n, generator=g).to(TDT[code]).cuda()
        got, ref = _both(lib, a, b, n, batch, code)
        assert np.array_equal(got, ref), (got[:4], ref[:4])
        ah = a.cpu().double().numpy().reshape(batch, n)
        bh = b.cpu().double().numpy().reshape(batch, n)
        exact = np.einsum("ij,ij->i", ah, bh)
        scale = np.sqrt(np.einsum("ij,ij->i", ah * ah, bh * bh))
        assert np.all(np.abs(got - exact) <= 1e-12 * n * scale), np.max(np.abs(got - exact) / scale)


def test_noalloc_dot_edges():
    from paper_2009_14788_amd import _lib
    lib = _lib.lib
    a = torch.ones(8, dtype=torch.float32, device="cuda")
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    s = _stream()
    # batch 0: no-op; n 0: zeros
    assert lib.radon_dot_f64_batched_noalloc(a.data_ptr(), a.data_ptr(), 8, 0, 0, out.data_ptr(), s) == 0
    assert lib.radon_dot_f64_batched_noalloc(a.data_ptr(), a.data_ptr(), 0, 3, 0, out.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert out[:3].cpu().tolist() == [0.0, 0.0, 0.0] and np.isnan(out[3].item())
    # beyond the fixed scratch: 1025 systems of >= 258048 elements need 65600 partials
    rc = lib.radon_dot_f64_batched_noalloc(a.data_ptr(), a.data_ptr(), 300000, 1025, 0,
                                           out.data_ptr(), s)
    assert rc == -8 and "scratch" in _lib.string(rc)
    # argument errors as radon_dot_f64_batched
    assert lib.radon_dot_f64_batched_noalloc(a.data_ptr(), a.data_ptr(), 8, 1, 7, out.data_ptr(), s) == -1
    assert lib.radon_dot_f64_batched_noalloc(a.data_ptr(), a.data_ptr(), -1, 1, 0, out.data_ptr(), s) == -1
    assert lib.radon_dot_f64_batched_noalloc(a.data_ptr() + 4, a.data_ptr(), 4, 1, 0, out.data_ptr(), s) == -2
