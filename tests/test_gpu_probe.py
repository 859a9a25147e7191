"""The vector-ALU issue-rate probe (a diagnostic for the roofline peak of the path
kernels, in its own library libbmprobe.so) runs through its C entry point, rejects bad sizes, and reports a rate of the order
of the peak derived from the chip's unit counts and clock."""
from __future__ import annotations

import pytest

from helpers import say
from paper_1409_4923_amd import probe as PR

pytestmark = pytest.mark.gpu


def test_valu_probe_rates():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    n = 256 * 1024
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    peak = 256 * 64 * 2.4e9
    fma = PR.valu_probe(0, 2000, out.data_ptr(), n, stream)
    mixed = PR.valu_probe(1, 2000, out.data_ptr(), n, stream)
    trans = PR.valu_probe(2, 2000, out.data_ptr(), n, stream)
    say("VALU probe: FMA %.3g, FMA+compare+select %.3g, FMA+exp2 %.3g lane-ops/s (peak %.3g)"
        % (fma, mixed, trans, peak))
    assert 0.3 * peak < fma < 1.1 * peak
    assert mixed > 0.3 * peak
    assert trans > 0.05 * peak
    assert torch.isfinite(out).all()
    with pytest.raises(PR.ProbeError):
        PR.valu_probe(0, 10, out.data_ptr(), 100, stream)
    with pytest.raises(PR.ProbeError):
        PR.valu_probe(3, 10, out.data_ptr(), n, stream)
