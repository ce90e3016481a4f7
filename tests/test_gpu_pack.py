"""GPU test of the FP16 pack kernel (``tetra_pack_f16``, the precision variant's storage format):
per-band scale 2^ceil(log2 max |w|) from the exponent and mantissa fields of the largest magnitude
(clamped to 2^-126..2^126, 1 for an all-zero band), FP16 values w / scale rounded to nearest even.
Compared bit for bit with a numpy rendering of the same rule."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def numpy_pack(w):
    """The rule in numpy: float32 division by an exact power of two, then RNE to float16."""
    nb = w.shape[0]
    mx = np.abs(w).reshape(nb, -1).max(axis=1).astype(np.float32)
    bits = mx.view(np.uint32).astype(np.int64)
    ex, man = bits >> 23, bits & 0x7FFFFF
    e = np.where(ex == 0, -126, ex - 127 + (man != 0))
    e = np.clip(np.where(bits == 0, 0, e), -126, 126)
    scale = np.ldexp(np.float32(1.0), e).astype(np.float32)
    inv = np.ldexp(np.float32(1.0), -e).astype(np.float32)
    w16 = (w * inv[:, None, None]).astype(np.float16)
    return w16, scale


def _cases():
    rng = np.random.default_rng(31)
    a = rng.uniform(0, 1, (5, 3, 101)).astype(np.float32)
    a[1] = 0.0                                   # all-zero band: scale 1
    a[2, 1, 7] = 0.5                             # largest value an exact power of two
    a[2] = np.minimum(a[2], 0.5)
    a[3] *= np.float32(3e-6)                     # values in the FP16 subnormal range after scaling
    a[3, 0, :50] *= np.float32(1e-4)
    a[4] = -a[4] * 37.0                          # signed weights (general observables), |w| > 1
    b = rng.normal(size=(16, 16, 4096)).astype(np.float32) ** 2  # C3-like orbital weights
    c = rng.uniform(0, 1, (1, 1, 1)).astype(np.float32)
    d = np.full((2, 1, 3), 1e-39, dtype=np.float32)  # FP32-subnormal largest value: scale 2^-126
    return [a, b, c, d]


@pytest.mark.parametrize("case", range(4))
def test_pack_matches_numpy_bitwise(case):
    import torch

    import paper_1710_10789_amd as tetra

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = _cases()[case]
    print(f"[case] pack {w.shape}", flush=True)
    w16, scale = tetra.half_weights(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    r16, rs = numpy_pack(w)
    assert np.array_equal(scale.cpu().numpy().view(np.uint32), rs.view(np.uint32))
    assert np.array_equal(w16.cpu().numpy().view(np.uint16), r16.view(np.uint16))
    # second call into the same outputs: everything overwritten, same bits
    w16b, scaleb = tetra.half_weights(torch.from_numpy(w).cuda(), out=w16, scale=scale)
    torch.cuda.synchronize()
    assert np.array_equal(w16b.cpu().numpy().view(np.uint16), r16.view(np.uint16))
