"""The measurement kernels behind the roofline figures do what their
throughput is credited with: the global-atomic probe adds exactly
blocks x 256 x 8 x iters to its buffer (no add lost or duplicated) and spreads
them over the whole buffer, and the copy kernel used to calibrate the byte
counters copies every byte (ragged sizes included)."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01122_amd import capred
    return capred


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("log2w,blocks,iters", [(6, 3, 5), (12, 64, 7), (18, 512, 3)])
def test_global_atomic_probe_counts(cap, log2w, blocks, iters):
    note(f"global atomic probe 2^{log2w} words, {blocks} blocks, {iters} iters")
    counts = torch.zeros(1 << log2w, dtype=torch.int32, device="cuda")
    cap.probe_global_atomic(iters, blocks, counts)
    torch.cuda.synchronize()
    c = counts.cpu().to(torch.int64)
    total = blocks * 256 * 8 * iters
    assert int(c.sum()) == total
    assert int(c.min()) >= 0
    # pseudo-random addresses: with >= 4 adds per word on average every word is hit
    if total >= 4 * (1 << log2w) * 8:
        assert int((c == 0).sum()) == 0


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 22) + 16 * 7])
def test_copy_kernel(cap, nbytes):
    note(f"copy {nbytes} bytes")
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros_like(src)
    cap.copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src.cpu(), dst.cpu())
