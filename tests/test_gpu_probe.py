"""The HBM bandwidth probe kernels (reff_stream_probe) do what the header
says on small buffers, so the bandwidths the benchmark reports for them are
those of real copies, reads and writes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_probe_kernels_move_the_data():
    import torch
    from paper_2607_05818_amd import reff
    print("[case] stream probe kinds 0-4 on 1 MiB arrays", flush=True)
    nb = 1 << 20
    n = nb // 4
    src = torch.arange(3 * n, dtype=torch.float32, device="cuda") * 0.5
    for kind in (0, 4):
        dst = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
        reff.reff_stream_probe(kind, src, dst, nb, 37)
        torch.cuda.synchronize()
        assert torch.equal(dst[:n], src[:n]) and torch.all(dst[n:] == 0)
    dst = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    reff.reff_stream_probe(3, src, dst, nb, 64)
    torch.cuda.synchronize()
    a, b, c = src[:n], src[n:2 * n], src[2 * n:]
    assert torch.equal(dst[:n], a + b) and torch.equal(dst[n:], b - c)
    reff.reff_stream_probe(2, None, dst, nb, 16)
    torch.cuda.synchronize()
    assert torch.all(dst[:n] == 1.0)
    out = torch.zeros(16 * 256, dtype=torch.float32, device="cuda")
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    reff.reff_stream_probe(1, ones, out, nb, 16)
    torch.cuda.synchronize()
    assert float(out.sum()) == float(n)
    with pytest.raises(reff.ReffError):
        reff.reff_stream_probe(0, src, dst, 10, 16)
