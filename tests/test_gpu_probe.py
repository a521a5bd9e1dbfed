"""The bandwidth probe (a kernel with a streaming kernel's access mix and no
arithmetic) through the C ABI: a positive duration that grows with the bytes
moved, and rejection of stream counts out of range."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_stream():
    from paper_2306_09189_amd import hecnn
    ctx = hecnn.Context(10, 2, 60, 40, 1, 60, 1, 40, device=0)
    small = ctx.probe_stream(6, 2, 1 << 16, 5)
    big = ctx.probe_stream(6, 2, 1 << 24, 5)
    assert 0 < small < big
    # 1 GiB moved: at least 1 TB/s and no more than the 8 TB/s of HBM
    gbps = 8 * (1 << 24) * 8 / (big * 1e-6) / 1e9
    assert 1000 < gbps < 8000, gbps
    for nr, nw in ((0, 2), (9, 2), (6, 0), (6, 5)):
        with pytest.raises(hecnn.HecError) as e:
            ctx.probe_stream(nr, nw, 1 << 16, 1)
        assert e.value.status == hecnn.HEC_EINVAL
    with pytest.raises(hecnn.HecError):
        ctx.probe_stream(6, 2, 100, 1)
