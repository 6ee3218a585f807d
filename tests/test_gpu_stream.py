"""The HBM streaming probe (pr_stream_probe): the copy reproduces its source, the read pass leaves it alone."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_stream_probe_copies_and_reads():
    import torch
    import paper_2204_01287_amd as pr

    ctx = pr.Context(0)
    rng = np.random.default_rng(3)
    for nbytes in (16, 4096, (1 << 20) + 48, 3 * (1 << 24) + 16 * 7):
        say(f"stream probe {nbytes} bytes")
        host = rng.integers(0, 256, nbytes + 32, dtype=np.uint8)
        src = torch.from_numpy(host).cuda()
        dst = torch.zeros(nbytes + 32, dtype=torch.uint8, device="cuda")
        pr.pr_stream_probe(ctx.handle, src, dst, nbytes)
        pr.pr_stream_probe(ctx.handle, src, None, nbytes)
        pr.pr_sync(ctx.handle)
        got = dst.cpu().numpy()
        assert np.array_equal(got[:nbytes], host[:nbytes])
        assert not got[nbytes:].any()  # nothing past the size
        assert np.array_equal(src.cpu().numpy(), host)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for args in ((buf, buf, 24), (buf.data_ptr() + 8, None, 16), (None, None, 16)):
        with pytest.raises(pr.PrError, match="PR_EINVAL"):
            pr.pr_stream_probe(ctx.handle, *args)
    ctx.close()
