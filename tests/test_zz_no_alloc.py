"""tvs_quality_noalloc, the allocation-free variant of tvs_quality, through
the C-ABI: its results equal tvs_quality's bit for bit, on two calls in a row
(the second on a smaller image, so the shared static scratch holds the first
call's sums when the second starts), in both dtypes; a fresh context that
only calls the variant holds no device memory of its own afterwards."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    c = Context(0)
    yield c
    c.close()


def pair(n2, n1, seed, dtype):
    clean, noisy = synth.noisy_image(n2, n1, 0.1, seed)
    return (torch.tensor(noisy, dtype=dtype, device=DEV), torch.tensor(clean, dtype=dtype, device=DEV))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_equals_quality_on_two_calls(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    with Context(0) as fresh:
        big, small = pair(700, 900, 61, dtype), pair(37, 53, 62, dtype)
        q_big = fresh.quality_noalloc(*big)
        q_small = fresh.quality_noalloc(*small)
        torch.cuda.synchronize()
        # the variant used none of the context's lazily allocated buffers
        assert fresh.bytes() == 0
        ref_big = fresh.quality(*big)
        ref_small = fresh.quality(*small)
        assert fresh.bytes() > 0
    for q, r in ((q_big, ref_big), (q_small, ref_small)):
        for k in ("psnr", "mssim", "mse"):
            assert q[k] == r[k], (k, q[k], r[k])
    assert q_big["mse"] != q_small["mse"]


def test_noalloc_identical_images_and_errors(ctx):
    from paper_2602_17494_amd import TVS_EINVAL, TvsError
    x, _ = pair(64, 48, 63, torch.float32)
    q = ctx.quality_noalloc(x, x.clone())
    assert q["mse"] == 0.0 and q["psnr"] == float("inf")
    assert abs(q["mssim"] - 1.0) < 1e-12
    # a bad dtype code is refused before any device work
    import ctypes
    from paper_2602_17494_amd.tvs import load
    out = (ctypes.c_double * 3)()
    rc = load().tvs_quality_noalloc(ctx._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    64, 48, 7, out, None)
    assert rc == TVS_EINVAL
    with pytest.raises(TvsError):
        ctx.quality_noalloc(x[:0], x[:0])
