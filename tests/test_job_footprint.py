"""Host-side job footprints (no GPU needed): they grow with the image, double
from float32 to float64 for the resident state, and include the overlap
frames and plans a layout adds."""
import pytest

torch = pytest.importorskip("torch")


def fp(shape, dtype, lay, its=(2, 3)):
    from paper_2602_17494_amd import job_footprint, make_iters, make_layout
    return job_footprint(shape, dtype, make_layout(*lay), make_iters(*its))


def test_footprint_properties():
    try:
        from paper_2602_17494_amd import load
        load()
    except Exception as e:  # library not built here
        pytest.skip(str(e))
    a = fp((64, 64), torch.float32, (1, 1, 0, 0))
    b = fp((128, 128), torch.float32, (1, 1, 0, 0))
    assert 0 < a < b
    c = fp((128, 128), torch.float64, (1, 1, 0, 0))
    table = 8 * 130 * 130
    assert 1.9 * (b - table) < c - table < 2.1 * (b - table)
    d = fp((128, 128), torch.float32, (2, 2, 8, 8))
    assert d > b  # local frames and plans on top of the global ones
    with pytest.raises(Exception):
        fp((1, 8), torch.float32, (1, 1, 0, 0))


def test_footprint_refuses_sides_beyond_the_transform_limit():
    # image sides up to 5119 (Omega-tilde sides up to 5120, transforms of at
    # most 10240 points in one workgroup's LDS); larger ones are refused with
    # TVS_EINVAL before any device work
    try:
        from paper_2602_17494_amd import load
        load()
    except Exception as e:  # library not built here
        pytest.skip(str(e))
    from paper_2602_17494_amd import TVS_EINVAL, TvsError
    assert fp((5119, 300), torch.float32, (1, 1, 0, 0)) > 0
    assert fp((4096, 4096), torch.float64, (16, 16, 16, 16)) > 0
    for shape in [(5120, 300), (300, 5120), (6000, 6000)]:
        with pytest.raises(TvsError) as e:
            fp(shape, torch.float32, (1, 1, 0, 0))
        assert e.value.code == TVS_EINVAL and "5120" in str(e.value)
