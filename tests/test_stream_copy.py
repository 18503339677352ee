"""The streaming copy used as the measured HBM ceiling (fft3d_stream_copy):
it must copy every byte, including past the single-sweep grid."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fft3d():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (64 << 20) + 16, (4 << 30) + 32])
def test_copies_every_byte(fft3d, nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes % 1000)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros(nbytes + 16, dtype=torch.uint8, device="cuda")
    fft3d.stream_copy(src, dst[:nbytes])
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].max()) == 0   # nothing written past the end


def test_rejections(fft3d):
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        fft3d.stream_copy(a, a[:32])
    lib = fft3d._lib.lib()
    assert lib.fft3d_stream_copy(a.data_ptr(), a.data_ptr() + 32, 24, None) == -1
    assert lib.fft3d_stream_copy(a.data_ptr() + 8, a.data_ptr() + 32, 16, None) == -6
