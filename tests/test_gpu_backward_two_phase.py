"""GPU tests of the adjoint's two-phase output (``tetra_dos_backward_ws``): tile-boundary points go
through per-tile face slots and a gather pass instead of global atomics. Applies where every grid side
is a multiple of the tile's with more than one tile per axis.

* Parity with the FP64 oracle (the per-element gate of the adjoint tests) for every tile shape, one
  and several energy passes over G, 1, 3, 8 and 16 orbitals, FP16 weights and complex amplitudes;
* every output element is written (outputs pre-filled with NaN; nothing is zero-filled on this path),
  also for a band with no finite energy and for grad_eps or grad_w alone;
* bitwise reproducible from run to run (``deterministic=True`` accepted), and within 1e-6 of the
  largest gradient of the atomic path on the same inputs;
* forward and adjoint captured in one HIP graph and replayed four times with eager work between
  replays, every replay against the eager result;
* one caller-owned workspace reused across problems of different sizes and tile shapes, bit for bit
  the result of a fresh one."""
import numpy as np
import pytest

import synth
from gates import gate

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 16), (8, 8, 4), (4, 8, 8), (8, 4, 8), (4, 16, 4), (16, 4, 4)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _grid(tile, mult=(2, 2, 2)):
    return tuple(t * m for t, m in zip(SHAPES[tile], mult))


def _run(torch_dev, eps, w, grid, e0, de, G, tile, **kw):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    ge, gw = tetra.dos_backward(torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), grid, e0, de,
                                torch.from_numpy(np.ascontiguousarray(G, np.float32)).to(dev), tile=tile, **kw)
    torch.cuda.synchronize()
    return (ge.cpu().numpy() if ge is not None else None), (gw.cpu().numpy() if gw is not None else None)


@pytest.mark.parametrize("tile", range(6))
@pytest.mark.parametrize("norb,ne", [(3, 120), (8, 1500)])
def test_two_phase_parity_every_tile_shape(torch_dev, oracle_lib, tile, norb, ne):
    import paper_1710_10789_amd as tetra

    grid = _grid(tile, (2, 3, 2) if tile % 2 else (3, 2, 2))
    eps, w = synth.band_structure(norb, 40 + tile, grid, cache=False)
    e0, de = synth.energy_grid(eps, ne)
    assert tetra.backward_workspace_bytes(grid, eps.shape[0], norb, e0, de, ne, tile=tile) > 0
    G = np.random.default_rng(tile).normal(size=(ne, norb)).astype(np.float32)
    print(f"[case] two-phase tile {tile} grid {grid} norb {norb} ne {ne}", flush=True)
    re, rw = oracle_lib.dos_backward(eps, w, grid, e0, de, G.astype(np.float64))
    ge, gw = _run(torch_dev, eps, w, grid, e0, de, G, tile)
    oke, eb, _ = gate(ge, re)
    okw, wb, _ = gate(gw, rw)
    print(f"[case] grad_eps {eb:.2e} grad_w {wb:.2e}", flush=True)
    assert oke and okw


@pytest.mark.parametrize("norb", [1, 16])
def test_two_phase_parity_orbital_counts(torch_dev, oracle_lib, norb):
    grid = (8, 8, 32)
    eps, w = synth.band_structure(norb, 50 + norb, grid, cache=False)
    e0, de = synth.energy_grid(eps, 200)
    G = np.random.default_rng(norb).normal(size=(200, norb)).astype(np.float32)
    print(f"[case] two-phase norb {norb}", flush=True)
    re, rw = oracle_lib.dos_backward(eps, w, grid, e0, de, G.astype(np.float64))
    ge, gw = _run(torch_dev, eps, w, grid, e0, de, G, 0)
    assert gate(ge, re)[0] and gate(gw, rw)[0]


def test_two_phase_writes_every_element(torch_dev, oracle_lib):
    """Outputs full of NaN before the call; band 1 has no finite energy at all (its tile-bands end
    early and must still write zeros); grad_eps alone and grad_w alone."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (8, 8, 32)
    eps, w = synth.band_structure(4, 61, grid, cache=False)
    eps = eps.copy()
    eps[1] = np.nan
    e0, de = synth.energy_grid(eps[[0, 2, 3]], 150)
    G = np.random.default_rng(2).normal(size=(150, 4)).astype(np.float32)
    re, rw = oracle_lib.dos_backward(eps, w, grid, e0, de, G.astype(np.float64))
    te, tw, tG = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(G).to(dev)
    ge = torch.full(te.shape, float("nan"), device=dev)
    gw = torch.full(tw.shape, float("nan"), device=dev)
    print("[case] two-phase over NaN-filled outputs, one all-NaN band", flush=True)
    tetra.dos_backward(te, tw, grid, e0, de, tG, grad_eps=ge, grad_w=gw)
    torch.cuda.synchronize()
    ge, gw = ge.cpu().numpy(), gw.cpu().numpy()
    assert np.isfinite(ge).all() and np.isfinite(gw).all()
    assert (ge[1] == 0).all() and (gw[1] == 0).all()
    assert gate(ge, re)[0] and gate(gw, rw)[0]
    only_e, none_w = _run(torch_dev, eps, w, grid, e0, de, G, 0, need_w=False)
    none_e, only_w = _run(torch_dev, eps, w, grid, e0, de, G, 0, need_eps=False)
    assert none_w is None and none_e is None
    assert np.array_equal(only_e, ge) and np.array_equal(only_w, gw)


def test_two_phase_is_reproducible_and_matches_atomic_path(torch_dev):
    grid = (16, 8, 16)
    eps, w = synth.band_structure(8, 70, grid, cache=False)
    e0, de = synth.energy_grid(eps, 400)
    G = np.random.default_rng(3).normal(size=(400, 8)).astype(np.float32)
    print("[case] two-phase determinism, tile 3", flush=True)
    a = _run(torch_dev, eps, w, grid, e0, de, G, 3)
    b = _run(torch_dev, eps, w, grid, e0, de, G, 3, deterministic=True)
    c = _run(torch_dev, eps, w, grid, e0, de, G, 3, two_phase=False)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y)
        assert np.abs(x - z).max() <= 1e-6 * np.abs(z).max()


def test_deterministic_raises_without_two_phase(torch_dev):
    import paper_1710_10789_amd as tetra

    grid = (6, 7, 9)  # not a multiple of any tile shape
    eps, w = synth.band_structure(2, 71, grid, cache=False)
    e0, de = synth.energy_grid(eps, 50)
    G = np.zeros((50, 2), np.float32)
    with pytest.raises(tetra.TetraError):
        _run(torch_dev, eps, w, grid, e0, de, G, 0, deterministic=True)


def test_two_phase_fp16_and_amplitudes(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (8, 16, 16)
    eps, a = synth.amplitudes(5, 72, grid)
    b = (a.real.astype(np.float64) ** 2 + a.imag.astype(np.float64) ** 2).astype(np.float32)
    e0, de = synth.energy_grid(eps, 130)
    G = np.random.default_rng(4).normal(size=(130, 5)).astype(np.float32)
    re, rb = oracle_lib.dos_backward(eps, b, grid, e0, de, G.astype(np.float64))
    print("[case] two-phase complex amplitudes, tile 2", flush=True)
    ge, ga = tetra.dos_backward(torch.from_numpy(eps).to(dev), torch.from_numpy(a).to(dev), grid, e0, de,
                                torch.from_numpy(G).to(dev), tile=2)
    ga = ga.cpu().numpy()
    ra = 2.0 * a.astype(np.complex128) * rb
    assert gate(ge.cpu().numpy(), re)[0] and gate(ga.real, ra.real)[0] and gate(ga.imag, ra.imag)[0]
    # FP16 weights: the gradient is that of the dequantised weights
    w16, scale = (t.cpu() for t in tetra.half_weights(torch.from_numpy(b).cuda()))
    wd = (w16.float() * scale[:, None, None]).numpy()
    re, rw = oracle_lib.dos_backward(eps, wd, grid, e0, de, G.astype(np.float64))
    print("[case] two-phase FP16 weights, tile 2", flush=True)
    ge, gw = tetra.dos_backward(torch.from_numpy(eps).to(dev), w16.to(dev), grid, e0, de,
                                torch.from_numpy(G).to(dev), w_scale=scale.to(dev), tile=2)
    assert gate(ge.cpu().numpy(), re)[0] and gate(gw.cpu().numpy(), rw)[0]


def test_forward_and_two_phase_adjoint_in_one_graph(torch_dev):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (8, 8, 32)
    eps, w = synth.band_structure(8, 73, grid, cache=False)
    e0, de = synth.energy_grid(eps, 300)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    G = torch.from_numpy(np.random.default_rng(6).normal(size=(300, 8)).astype(np.float32)).to(dev)
    ws = torch.empty(tetra.backward_workspace_bytes(grid, 8, 8, e0, de, 300), dtype=torch.uint8, device=dev)
    dos = torch.empty((300, 8), device=dev)
    ge, gw = torch.empty_like(te), torch.empty_like(tw)

    def step():
        tetra.dos_forward(te, tw, grid, e0, de, 300, out=dos)
        tetra.dos_backward(te, tw, grid, e0, de, G, grad_eps=ge, grad_w=gw, workspace=ws)

    step()
    torch.cuda.synchronize()
    ref = [dos.clone(), ge.clone(), gw.clone()]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    print("[case] forward + two-phase adjoint graph capture", flush=True)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in (dos, ge, gw):
            t.fill_(float("nan"))  # eager work between replays
        ws.fill_(0xFF)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.allclose(dos, ref[0], rtol=1e-6, atol=1e-6 * float(ref[0].abs().max())), rep
        assert torch.equal(ge, ref[1]) and torch.equal(gw, ref[2]), rep  # the adjoint is reproducible


def test_workspace_reused_across_problems(torch_dev):
    """One caller-owned workspace, sized for the larger problem, used for two problems in a row (the
    second smaller, on another tile shape) and then for the first again: each result equals that of
    a fresh workspace bit for bit, so nothing depends on what the workspace held before."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    probs = []
    for grid, tile, ne, seed in (((8, 8, 32), 0, 200, 81), ((16, 8, 16), 3, 90, 82)):
        eps, w = synth.band_structure(4, seed, grid, cache=False)
        e0, de = synth.energy_grid(eps, ne)
        G = torch.from_numpy(np.random.default_rng(seed).normal(size=(ne, 4)).astype(np.float32)).to(dev)
        probs.append((torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), grid, e0, de, G, tile))
    sizes = [tetra.backward_workspace_bytes(p[2], p[0].shape[0], 4, p[3], p[4], p[5].shape[0], tile=p[6]) for p in probs]
    assert sizes[0] > sizes[1] > 0
    ws = torch.full((sizes[0],), 0xAB, dtype=torch.uint8, device=dev)
    print("[case] workspace reuse, two problems", flush=True)
    results = []
    for p in (probs[0], probs[1], probs[0]):
        te, tw, grid, e0, de, G, tile = p
        shared = tetra.dos_backward(te, tw, grid, e0, de, G, tile=tile, workspace=ws)
        fresh = tetra.dos_backward(te, tw, grid, e0, de, G, tile=tile, deterministic=True)
        torch.cuda.synchronize()
        assert torch.equal(shared[0], fresh[0]) and torch.equal(shared[1], fresh[1])
        results.append(shared)
    assert torch.equal(results[0][0], results[2][0]) and torch.equal(results[0][1], results[2][1])
    with pytest.raises(ValueError):
        te, tw, grid, e0, de, G, tile = probs[0]
        tetra.dos_backward(te, tw, grid, e0, de, G, tile=tile, workspace=ws[: sizes[0] - 1])
