"""The plain copy behind the HBM-ceiling measurement (dct_probe_copy): byte
for byte equal to its source at sizes around the workgroup and word sizes."""
import sys

import pytest


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


@pytest.fixture(scope="module")
def hip():
    from paper_1306_1373_amd import codec
    codec.load()
    return codec


@pytest.mark.parametrize("nbytes", [0, 16, 4096 + 16, 256 * 16 * 3 + 48, (1 << 22) + 4080])
def test_copy_exact(hip, nbytes):
    import torch
    print(f"[probe copy] {nbytes} bytes", file=sys.stderr, flush=True)
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.full((nbytes + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    hip.probe_copy(src[:nbytes], dst[:nbytes])
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert bool((dst[nbytes:] == 0xA5).all())   # nothing past the end


def test_copy_rejects_overlap_and_size(hip):
    import torch
    buf = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(hip.DctError):
        hip.probe_copy(buf[:512], buf[256:768])
    with pytest.raises(hip.DctError):
        hip.probe_copy(buf[:24], buf[512:536])
