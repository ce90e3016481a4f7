"""GPU tests of the measurement helpers behind the benchmark's ceiling figures: every workgroup's
LDS-atomic checksum equals what its adds must sum to, and every lane of the FMA probe returns the
value of its sixteen chains computed with single-rounded FP32 FMAs on the host, so the work the
timings count is issued."""
import numpy as np
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


def test_fma_probe_values():
    import torch

    from paper_1710_10789_amd import probe

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    blocks, iters = 3, 50
    print(f"[case] fma probe {blocks} workgroups x {iters} iterations", flush=True)
    out = probe.probe_fma_f32(blocks, iters, device="cuda:0")
    torch.cuda.synchronize()
    # x * a + b in FP64 is exact for these operands (48-bit products, sums within 53 bits), so one
    # rounding to FP32 is the fused multiply-add's
    a, b = np.float32(0.999), np.float32(1e-4)
    tid = np.arange(256, dtype=np.float64)
    x = (tid[:, None] * np.float64(np.float32(1e-3)) + np.arange(16, dtype=np.float64)[None, :]).astype(np.float32)
    for _ in range(iters):
        x = (x.astype(np.float64) * np.float64(a) + np.float64(b)).astype(np.float32)
    s = np.zeros(256, dtype=np.float32)
    for c in range(16):
        s = (s + x[:, c]).astype(np.float32)
    got = out.cpu().numpy().reshape(blocks, 256)
    for blk in range(blocks):
        assert np.array_equal(got[blk], s), np.abs(got[blk] - s).max()
