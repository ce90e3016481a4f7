"""Full-size parity in every launch configuration the autotuner can pick: the headline workload
(64^3 periodic grid, 8 bands x 8 orbitals, 1000 energies) through each tile shape of the forward and
of the adjoint kernel, every output element against the FP64 oracle.

Gates as in the other GPU tests: forward max |D - D_ref| / max |D_ref| <= 1e-5; gradients per element
|g - g_ref| <= 1e-3 |g_ref| where |g_ref| >= 1e-3 max |g_ref|, else <= 1e-6 max |g_ref|."""
import numpy as np
import pytest

import synth
from test_gpu_backward import gate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def headline(oracle_lib):
    c = synth.config("k64_b8_e1000")
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    eps, w = synth.band_structure(norb, c["seed"], grid)
    teps, tw = synth.band_structure(norb, 1, grid)
    e0, de = synth.energy_grid(eps, ne)
    D, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    T, _ = oracle_lib.dos(teps, tw, grid, e0, de, ne)
    G = (2.0 * (D - T)).astype(np.float32)  # the loss gradient of the bench, from the oracle
    re, rw = oracle_lib.dos_backward(eps, w, grid, e0, de, G.astype(np.float64))
    return grid, ne, eps, w, e0, de, D, G, re, rw


def test_forward_every_tile_shape(torch_dev, headline):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, ne, eps, w, e0, de, D, _, _, _ = headline
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    scale = np.abs(D).max()
    for tile in range(len(tetra.TILE_SHAPES)):
        print(f"[case] forward 64^3 x 8 x 8 x 1000, tile {tetra.TILE_SHAPES[tile]}", flush=True)
        got = tetra.dos_forward(te, tw, grid, e0, de, ne, tile=tile)
        torch.cuda.synchronize()
        err = np.abs(got.cpu().numpy().astype(np.float64) - D).max() / scale
        print(f"[case] err {err:.3e}", flush=True)
        assert err <= 1e-5


def test_adjoint_every_tile_shape(torch_dev, headline):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, ne, eps, w, e0, de, _, G, re, rw = headline
    te, tw, tG = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(G).to(dev)
    for tile in range(len(tetra.TILE_SHAPES)):
        print(f"[case] adjoint 64^3 x 8 x 8 x 1000, tile {tetra.TILE_SHAPES[tile]}", flush=True)
        ge, gw = tetra.dos_backward(te, tw, grid, e0, de, tG, tile=tile)
        torch.cuda.synchronize()
        okw, wb, _ = gate(gw.cpu().numpy(), rw)
        oke, eb, _ = gate(ge.cpu().numpy(), re)
        print(f"[case] grad_w worst-rel {wb:.2e}; grad_eps worst-rel {eb:.2e}", flush=True)
        assert okw and oke
