"""GPU tests of the batched persistent path (tetra_dos_batched) through the C ABI: every item against
the single-problem forward and the FP64 oracle; mixed orbital counts and more items than one launch
holds; capture in a HIP graph with repeated replays."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _err(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / scale if scale > 0 else np.abs(got).max()


def _problems(torch, dev, specs):
    probs, host = [], []
    for seed, grid, ne, norb in specs:
        eps, w = synth.band_structure(norb, seed, grid)
        e0, de = synth.energy_grid(eps, ne)
        probs.append((torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), grid, e0, de, ne))
        host.append((eps, w, grid, e0, de, ne))
    return probs, host


def test_batched_mixed_grids_match_single_and_oracle(torch_dev, oracle_lib):
    """The batched workload's mix (32 models, cubic grids of uneven size, 256-2048 energies) with
    grids scaled down so the oracle stays quick."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    specs = [(seed, grid, ne, 8) for seed, grid, ne in synth.batched_items(scale=0.25)]
    print(f"[case] batched {len(specs)} items, grids {sorted({s[1][0] for s in specs})}", flush=True)
    probs, host = _problems(torch, dev, specs)
    outs = tetra.dos_batched(probs)
    singles = [tetra.dos_forward(*p) for p in probs]
    torch.cuda.synchronize()
    for o, s, (eps, w, grid, e0, de, ne) in zip(outs, singles, host):
        got = o.cpu().numpy().astype(np.float64)
        assert _err(got, s.cpu().numpy().astype(np.float64)) <= 1e-6
        ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
        assert _err(got, ref) <= 1e-5


def test_batched_orbital_groups_and_many_items(torch_dev, oracle_lib):
    """40 items with three orbital counts: several persistent launches, one counter each."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    rng = np.random.default_rng(9)
    specs = []
    for i in range(40):
        n = int(rng.integers(2, 9))
        specs.append((300 + i, (n, int(rng.integers(1, 7)), int(rng.integers(3, 20))), int(rng.integers(50, 400)),
                      int(rng.choice([3, 8, 5]))))
    probs, host = _problems(torch, dev, specs)
    print(f"[case] {len(specs)} items, workspace {tetra.batched_workspace_bytes(probs)} bytes", flush=True)
    outs = tetra.dos_batched(probs)
    torch.cuda.synchronize()
    for o, (eps, w, grid, e0, de, ne) in zip(outs, host):
        ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
        assert _err(o.cpu().numpy().astype(np.float64), ref) <= 1e-5


def test_batched_fp16_weights(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    probs = []
    refs = []
    for seed, grid, ne in ((1, (6, 7, 20), 300), (2, (12, 4, 9), 700)):
        eps, w = synth.band_structure(8, seed, grid)
        e0, de = synth.energy_grid(eps, ne)
        w16, scale = (t.cpu() for t in tetra.half_weights(torch.from_numpy(w).cuda()))
        deq = (w16.float() * scale[:, None, None]).numpy()
        probs.append((torch.from_numpy(eps).to(dev), w16.to(dev), grid, e0, de, ne, scale.to(dev)))
        refs.append(oracle_lib.dos(eps, deq, grid, e0, de, ne)[0])
    outs = tetra.dos_batched(probs)
    torch.cuda.synchronize()
    for o, ref in zip(outs, refs):
        assert _err(o.cpu().numpy().astype(np.float64), ref) <= 1e-5


def test_batched_workspace_too_small(torch_dev):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    probs, _ = _problems(torch, dev, [(5, (4, 4, 4), 64, 3)])
    with pytest.raises(tetra.TetraError):
        tetra.dos_batched(probs, workspace=torch.empty(8, dtype=torch.uint8, device=dev))


def test_batched_graph_capture_replays(torch_dev):
    """One capture, several replays with eager work between them; every replay recomputes the
    cleared outputs exactly as the eager call did."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    specs = [(seed, grid, ne, 8) for seed, grid, ne in synth.batched_items(n_models=6, scale=0.2)]
    probs, _ = _problems(torch, dev, specs)
    ws = torch.empty(tetra.batched_workspace_bytes(probs), dtype=torch.uint8, device=dev)
    outs = [torch.empty((p[5], 8), device=dev) for p in probs]
    eager = [o.clone() for o in tetra.dos_batched(probs, workspace=ws, out=outs)]  # warm-up, eager result
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tetra.dos_batched(probs, workspace=ws, out=outs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        for o in outs:
            o.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.allclose(o, e, rtol=1e-6, atol=1e-6 * float(e.abs().max())), rep


def test_batched_per_item_tile_shapes(torch_dev, oracle_lib):
    """Items of one persistent launch may use different tile shapes."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    specs = [(60 + i, (5 + i, 7, 9 + 2 * i), 150 + 37 * i, 8) for i in range(6)]
    probs, host = _problems(torch, dev, specs)
    outs = tetra.dos_batched(probs, tiles=list(range(6)))
    torch.cuda.synchronize()
    for o, (eps, w, grid, e0, de, ne) in zip(outs, host):
        ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
        assert _err(o.cpu().numpy().astype(np.float64), ref) <= 1e-5


def test_batched_sixteen_orbitals_fp16(torch_dev, oracle_lib):
    """The largest orbital count through the persistent launch, with FP16 weights and per-item tiles."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    probs, refs = [], []
    for seed, grid, ne in ((21, (8, 9, 10), 700), (22, (12, 5, 16), 1300), (23, (3, 4, 33), 256)):
        eps, w = synth.band_structure(16, seed, grid)
        e0, de = synth.energy_grid(eps, ne)
        w16, scale = (t.cpu() for t in tetra.half_weights(torch.from_numpy(w).cuda()))
        deq = (w16.float() * scale[:, None, None]).numpy()
        probs.append((torch.from_numpy(eps).to(dev), w16.to(dev), grid, e0, de, ne, scale.to(dev)))
        refs.append(oracle_lib.dos(eps, deq, grid, e0, de, ne)[0])
    print(f"[case] batched norb 16 fp16, {len(probs)} items", flush=True)
    outs = tetra.dos_batched(probs, tiles=[5, 2, 0])
    torch.cuda.synchronize()
    for o, ref in zip(outs, refs):
        assert _err(o.cpu().numpy().astype(np.float64), ref) <= 1e-5
