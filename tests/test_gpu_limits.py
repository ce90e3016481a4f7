"""GPU tests at the largest energy grid the C ABI accepts (ne = 2^22): a tile-band's index range then
spans about a million bins, so every kernel makes hundreds of passes over its LDS histogram (or its
rows of G), and the FP32 window estimates work at the limit they are validated for.

Small k-grid (3 x 4 x 5, one tile), 4 bands x 4 orbitals over the band range +-10 %. DOS and
gradients against the FP64 oracle in full; the number of states and bin averages (the oracle is
dense in energy there) at sampled energies, and the number of states at the last energy, above
every band, against the mean orbital weight summed over bands. Gates as in the other GPU tests."""
import numpy as np
import pytest

import synth
from test_gpu_backward import gate

pytestmark = pytest.mark.gpu

GRID = (3, 4, 5)
NORB = 4
NE = 1 << 22


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def model():
    eps, w = synth.band_structure(NORB, 13, GRID)
    e0, de = synth.energy_grid(eps, NE)
    return eps, w, e0, de


def test_largest_energy_grid_dos_and_adjoint(torch_dev, oracle_lib, model):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    eps, w, e0, de = model
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    print(f"[case] DOS {GRID} x {NORB} x {NORB}, ne = 2^22", flush=True)
    got = tetra.dos_forward(te, tw, GRID, e0, de, NE)
    torch.cuda.synchronize()
    ref, _ = oracle_lib.dos(eps, w, GRID, e0, de, NE)
    err = np.abs(got.cpu().numpy().astype(np.float64) - ref).max() / np.abs(ref).max()
    print(f"[case] DOS err {err:.3e}", flush=True)
    assert err <= 1e-5
    G = np.random.default_rng(3).standard_normal((NE, NORB)).astype(np.float32)
    print("[case] adjoint, ne = 2^22", flush=True)
    ge, gw = tetra.dos_backward(te, tw, GRID, e0, de, torch.from_numpy(G).to(dev))
    torch.cuda.synchronize()
    re, rw = oracle_lib.dos_backward(eps, w, GRID, e0, de, G.astype(np.float64))
    oke, eb, _ = gate(ge.cpu().numpy(), re)
    okw, wb, _ = gate(gw.cpu().numpy(), rw)
    print(f"[case] grad_eps {eb:.2e}, grad_w {wb:.2e}", flush=True)
    assert oke and okw


def test_largest_energy_grid_number_of_states(torch_dev, oracle_lib, model):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    eps, w, e0, de = model
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    print("[case] number of states and bin averages, ne = 2^22", flush=True)
    n = tetra.nos_forward(te, tw, GRID, e0, de, NE).cpu().numpy().astype(np.float64)
    b = tetra.dos_binned(te, tw, GRID, e0, de, NE).cpu().numpy().astype(np.float64)
    mean_b = w.astype(np.float64).sum(axis=(0, 2)) / eps.shape[1]
    assert np.abs(n[-1] - mean_b).max() <= 1e-5 * np.abs(mean_b).max()
    assert np.abs(b.sum(axis=0) * de - mean_b).max() <= 1e-5 * np.abs(mean_b).max()
    bscale = np.abs(b).max()
    for j in np.random.default_rng(4).choice(NE, size=6, replace=False):
        E = e0 + int(j) * de
        rn = oracle_lib.nos(eps, w, GRID, E, de, 1)[0]
        rb = oracle_lib.dos_binned(eps, w, GRID, E, de, 1)[0]
        en = np.abs(n[j] - rn).max() / np.abs(mean_b).max()
        eb = np.abs(b[j] - rb).max() / bscale
        print(f"[case] j={j}: nos err {en:.3e}, binned err {eb:.3e}", flush=True)
        assert en <= 1e-5 and eb <= 1e-5
