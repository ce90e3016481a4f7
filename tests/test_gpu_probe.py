"""GPU test of the LDS-atomic measurement helper behind the benchmark's ceiling figure: every
workgroup's checksum equals what its adds must sum to, so the atomics the timing counts are issued."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_checksums():
    import torch

    from paper_1710_10789_amd import probe

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    blocks, iters = 300, 37
    print(f"[case] probe {blocks} workgroups x {iters} iterations", flush=True)
    out = probe.probe_lds_atomics(blocks, iters, device="cuda:0")
    torch.cuda.synchronize()
    # lane t adds t + 1, four times per iteration
    want = 4 * iters * sum(t + 1 for t in range(256))
    assert out.cpu().tolist() == [want] * blocks
