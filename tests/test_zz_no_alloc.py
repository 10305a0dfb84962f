"""gsr_ncc_noalloc (NCC with its scratch in a static device array, no
allocation) against gsr_ncc on the same inputs, over two calls in a row, the
second smaller, and against the oracle's NCC (Eq. 10) within 1e-4; sizes past
the static scratch are refused."""
import numpy as np
import pytest

from oracle import ncc as oncc

pytestmark = pytest.mark.gpu


def _pair(rng, P, H, W):
    q = rng.uniform(0.0, 1.0, (3, H, W)).astype(np.float32)
    a = rng.uniform(-1.0, 1.5, P)[:, None, None, None]
    noise = rng.normal(0.0, rng.uniform(0.05, 2.0, P)[:, None, None, None], (P, 3, H, W))
    return q, (a * q[None] + noise).astype(np.float32)


def test_ncc_noalloc_matches_ncc_two_calls():
    import torch
    from paper_2403_11367_amd import Context, GsrError
    ctx = Context(0)
    rng = np.random.default_rng(17)
    dev = torch.device("cuda", 0)
    for P, H, W in ((64, 376, 1408), (5, 37, 61)):  # the bench's batch, then a smaller ragged one
        print(f"ncc_noalloc: P {P}, {W}x{H}", flush=True)
        q, r = _pair(rng, P, H, W)
        qd, rd = torch.as_tensor(q, device=dev), torch.as_tensor(r, device=dev)
        ref = ctx.ncc(qd, rd)
        got = torch.full((P,), float("nan"), device=dev)
        ctx.ncc_noalloc(qd, rd, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)  # the same kernels on the same inputs
        exp = oncc.ncc(q, r)
        assert np.abs(got.cpu().numpy() - exp).max() <= 1e-4
    # scratch need 4 H W + 48 P ceil(H W / 4096) bytes > 8 MiB: refused, output untouched
    P, H, W = 2, 1024, 2100
    q, r = _pair(rng, P, H, W)
    out = torch.full((P,), 7.0, device=dev)
    with pytest.raises(GsrError, match="static scratch"):
        ctx.ncc_noalloc(torch.as_tensor(q, device=dev), torch.as_tensor(r, device=dev), out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    ctx.close()
