"""The surrogate query without a workspace (bm_surrogate_query_noalloc), through the
C ABI, against bm_surrogate_query with a caller workspace on the same inputs: the
two run the same kernels, so mean, std, the routed count and the routed indices
must agree bit for bit.  Two calls in a row, the second smaller, so a stale
scratch from the first call would show; a third on fewer members."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import say
from oracle import mlp as M
from paper_1409_4923_amd import bmotor as B
from paper_1409_4923_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    B.lib()
    yield
    torch.cuda.synchronize()


def _query(s, xd, thr, noalloc):
    import torch
    n = xd.shape[0]
    mean = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    std = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    fidx = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    fcnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        B.bm_surrogate_query_noalloc(s.n, s.params.data_ptr(), s.wbf.data_ptr(), xd.data_ptr(), n, thr,
                                     mean.data_ptr(), std.data_ptr(), fidx.data_ptr(), fcnt.data_ptr(), stream)
    else:
        nb = B.bm_mlp_workspace_size(s.n, n, 0)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        B.bm_surrogate_query(s.n, s.params.data_ptr(), s.wbf.data_ptr(), xd.data_ptr(), n, thr, mean.data_ptr(),
                             std.data_ptr(), fidx.data_ptr(), fcnt.data_ptr(), ws.data_ptr(), nb, stream)
    torch.cuda.synchronize()
    c = int(fcnt.cpu().numpy()[0])
    return mean.cpu().numpy(), std.cpu().numpy(), c, fidx.cpu().numpy()[:max(c, 0)].astype(np.uint32)


def _same(a, b):
    assert a[0].tobytes() == b[0].tobytes(), "mean differs"
    assert a[1].tobytes() == b[1].tobytes(), "std differs"
    assert a[2] == b[2], "routed count differs"
    assert np.array_equal(a[3], b[3]), "routed indices differ"


@pytest.mark.parametrize("members,sizes", [(5, (70_001, 1_000)), (3, (200_000, 63))])
def test_noalloc_query_matches_workspace_query(members, sizes):
    import torch
    p = W.mlp_params(members, seed=31 + members)
    s = B.Surrogate(members, params=p)
    for i, n in enumerate(sizes):
        say("no-alloc query: %d members, %d rows (call %d)" % (members, n, i + 1))
        x = W.surrogate_queries(n, seed=40 + i)
        xd = torch.tensor(x, device="cuda")
        thr = 0.0
        ref = _query(s, xd, thr, noalloc=False)
        thr = float(np.median(ref[1]))              # about half the rows route
        ref = _query(s, xd, thr, noalloc=False)
        got = _query(s, xd, thr, noalloc=True)
        _same(got, ref)
        assert 0 < got[2] < n or n < 100
        assert np.array_equal(got[3], M.route(got[1], thr))


def test_noalloc_query_rejects_beyond_scratch():
    import torch
    s = B.Surrogate(16, seed=3)
    n = B.BM_QUERY_SCRATCH_BYTES // (16 * 4) + 1
    xd = torch.zeros((1, 5), dtype=torch.float32, device="cuda")
    out = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(B.BMError) as ei:
        B.bm_surrogate_query_noalloc(16, s.params.data_ptr(), s.wbf.data_ptr(), xd.data_ptr(), n, 0.0,
                                     out.data_ptr(), out.data_ptr(), out.data_ptr(), out.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == -3
