"""GPU parity of every tile shape (forward and adjoint) and of the autotuner's choice."""
import numpy as np
import pytest

import synth
from gates import gate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _err(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / scale if scale > 0 else np.abs(got).max()


@pytest.mark.parametrize("tile", range(6))
@pytest.mark.parametrize("grid", [(9, 6, 21), (3, 17, 5), (1, 2, 40)])
def test_every_tile_shape_forward_and_backward(torch_dev, oracle_lib, tile, grid):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    print(f"[case] tile={tile} {tetra.TILE_SHAPES[tile]} grid={grid}", flush=True)
    eps, w = synth.band_structure(5, 40 + tile, grid)
    e0, de = synth.energy_grid(eps, 170)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    got = tetra.dos_forward(te, tw, grid, e0, de, 170, tile=tile)
    G = np.random.default_rng(tile).normal(size=(170, 5)).astype(np.float32)
    ge, gw = tetra.dos_backward(te, tw, grid, e0, de, torch.from_numpy(G).to(dev), tile=tile)
    torch.cuda.synchronize()
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, 170)
    assert _err(got.cpu().numpy().astype(np.float64), ref) <= 1e-5
    re, rw = oracle_lib.dos_backward(eps, w, grid, e0, de, G.astype(np.float64))
    oke, eb, en = gate(ge.cpu().numpy(), re)
    okw, wb, wn = gate(gw.cpu().numpy(), rw)
    print(f"[case] grad_eps worst-rel {eb:.2e} norm {en:.2e}; grad_w worst-rel {wb:.2e} norm {wn:.2e}", flush=True)
    assert oke and okw


def test_autotuner_picks_a_shape_and_caches_it(torch_dev, tmp_path, monkeypatch):
    torch, dev = torch_dev
    monkeypatch.setenv("TETRA_TUNE_CACHE", str(tmp_path / "tune.json"))
    import importlib

    import paper_1710_10789_amd.tune as tune

    tune = importlib.reload(tune)
    grid = (16, 16, 16)
    eps, w = synth.band_structure(8, 0, grid)
    e0, de = synth.energy_grid(eps, 200)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    best, times = tune.tune_forward(te, tw, grid, e0, de, 200, reps=1)
    assert 0 <= best < 6 and len(times) == 6 and times[best] == min(times)
    assert tune.best_tile("forward", te, tw, grid, 200) == best
    G = torch.ones(200, 8, device=dev)
    bbest, _ = tune.tune_backward(te, tw, grid, e0, de, G, reps=1)
    assert tune.best_tile("backward", te, tw, grid, 200) == bbest
    assert (tmp_path / "tune.json").exists()
