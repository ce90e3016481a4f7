"""Full-size parity of the precision workload: 128^3 periodic grid (12.6 M tetrahedra), 16 bands x 16
orbitals (the paper's largest realistic model size, Sec. III.B), 2000 energies. Every output element
against the FP64 oracle, through the C ABI:

* FP32 weights, plain forward: max |D - D_ref| / max |D_ref| <= 1e-5;
* exact accumulation (TETRA_EXACT): <= 1e-5, and bitwise equal on a repeated call;
* FP16 weights with a per-band power-of-two scale (packed by the library's kernel): <= 1e-3 against the
  oracle on the FP32 weights and <= 1e-5 against the oracle on the dequantised weights, plain and exact.

The model's diagonalisation (2.1 M Hermitian 16 x 16 matrices) runs on the host's cores once per
module (cached on disk); each oracle pass takes a few seconds on 16 threads."""
import numpy as np
import pytest

import synth
from gates import dos_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def c3(oracle_lib):
    c = synth.config("k128_b16_e2000")
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    print(f"[case] k128_b16_e2000: diagonalising {grid} x {norb} orbitals", flush=True)
    eps, w = synth.band_structure(norb, c["seed"], grid, progress=True)
    e0, de = synth.energy_grid(eps, ne)
    ref, cnt = oracle_lib.dos(eps, w, grid, e0, de, ne)
    print(f"[case] oracle done: {cnt} in-window updates", flush=True)
    return grid, norb, ne, eps, w, e0, de, ref


def test_c3_fp32_plain_and_exact(torch_dev, c3):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne, eps, w, e0, de, ref = c3
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    print("[case] k128_b16_e2000 fp32 plain", flush=True)
    plain = tetra.dos_forward(te, tw, grid, e0, de, ne)
    print("[case] k128_b16_e2000 fp32 exact x2", flush=True)
    ex1 = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True)
    ex2 = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True)
    torch.cuda.synchronize()
    e_plain = dos_err(plain.cpu().numpy().astype(np.float64), ref)
    e_exact = dos_err(ex1.cpu().numpy().astype(np.float64), ref)
    print(f"[case] err plain {e_plain:.3e}, exact {e_exact:.3e}", flush=True)
    assert e_plain <= 1e-5
    assert e_exact <= 1e-5
    assert torch.equal(ex1, ex2)


def test_c3_fp16_weights(torch_dev, oracle_lib, c3):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne, eps, w, e0, de, ref32 = c3
    te = torch.from_numpy(eps).to(dev)
    w16, scale = tetra.half_weights(torch.from_numpy(w).to(dev))
    torch.cuda.synchronize()
    deq = (w16.float() * scale[:, None, None]).cpu().numpy()
    refdq, _ = oracle_lib.dos(eps, deq, grid, e0, de, ne)
    del deq
    for exact in (False, True):
        print(f"[case] k128_b16_e2000 fp16 weights exact={exact}", flush=True)
        got = tetra.dos_forward(te, w16, grid, e0, de, ne, w_scale=scale, exact=exact)
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.float64)
        e32, edq = dos_err(got, ref32), dos_err(got, refdq)
        print(f"[case] err vs fp32 weights {e32:.3e}, vs dequantised {edq:.3e}", flush=True)
        assert e32 <= 1e-3
        assert edq <= 1e-5
