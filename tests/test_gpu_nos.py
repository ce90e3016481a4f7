"""GPU tests of the orbital-resolved number of states and the bin-averaged DOS (``tetra_nos_forward``,
``tetra_dos_binned`` through the C ABI) against the FP64 oracle (``nos``, ``dos_binned``).

Small grids span several tiles with ragged edges in every direction, odd and even orbital counts,
energy grids that start inside the bands (so that whole tetrahedra lie below the first energy) and
end inside them, every tile shape, FP16 weights, signed weights (the 64-bit histogram form), grids
entirely below or above the bands, and a single energy. At the headline size (64^3 x 8 x 8 x 1000)
the oracle, which is dense in energy, is evaluated at sampled energies and bins, and properties that
hold at any size are checked on every output: N at an energy above every band equals the mean
orbital weight summed over bands, N is non-decreasing, and the bin averages times de sum to the
difference of N at the outer bin edges.

Gate (FP32 kernels against FP64): max |X - X_ref| / max |X_ref| <= 1e-5."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _grid_inside(eps, ne, lo_frac, hi_frac):
    lo, hi = float(np.min(eps)), float(np.max(eps))
    a, b = lo + lo_frac * (hi - lo), lo + hi_frac * (hi - lo)
    e0 = float(np.float32(a))
    de = float(np.float32((b - a) / (ne - 1) if ne > 1 else 0.01 * (hi - lo)))
    return e0, de


def _err(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got.astype(np.float64) - ref).max() / scale if scale > 0 else np.abs(got).max()


def _run(torch, dev, eps, w, grid, e0, de, ne, tile=None, w16=None, scale=None):
    import paper_1710_10789_amd as tetra

    te = torch.from_numpy(eps).to(dev)
    if w16 is not None:
        tw, ts = w16.to(dev), scale.to(dev)
    else:
        tw, ts = torch.from_numpy(w).to(dev), None
    n = tetra.nos_forward(te, tw, grid, e0, de, ne, w_scale=ts, tile=tile)
    b = tetra.dos_binned(te, tw, grid, e0, de, ne, w_scale=ts, tile=tile)
    torch.cuda.synchronize()
    return n.cpu().numpy(), b.cpu().numpy()


CASES = [
    # grid, norb (= bands), seed, ne, energy grid as fractions of the band range
    ((9, 7, 18), 5, 3, 150, (0.3, 0.8)),
    ((5, 6, 7), 8, 4, 77, (-0.1, 1.1)),
    ((16, 16, 16), 3, 5, 200, (0.05, 0.6)),
    ((6, 11, 4), 2, 6, 1, (0.5, 0.5)),
    ((3, 2, 1), 1, 7, 40, (0.2, 0.9)),
]


@pytest.mark.parametrize("grid,norb,seed,ne,frac", CASES)
def test_nos_and_binned_against_oracle(torch_dev, oracle_lib, grid, norb, seed, ne, frac):
    torch, dev = torch_dev
    eps, w = synth.band_structure(norb, seed, grid)
    e0, de = _grid_inside(eps, ne, *frac)
    print(f"[case] nos {grid} norb={norb} seed={seed} ne={ne} e0={e0} de={de}", flush=True)
    rn = oracle_lib.nos(eps, w, grid, e0, de, ne)
    rb = oracle_lib.dos_binned(eps, w, grid, e0, de, ne)
    gn, gb = _run(torch, dev, eps, w, grid, e0, de, ne)
    en, eb = _err(gn, rn), _err(gb, rb)
    print(f"[case] err nos {en:.3e} binned {eb:.3e}", flush=True)
    assert en <= TOL and eb <= TOL


def test_every_tile_shape(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne = (17, 9, 21), 4, 120
    eps, w = synth.band_structure(norb, 8, grid)
    e0, de = _grid_inside(eps, ne, 0.25, 0.75)
    rn = oracle_lib.nos(eps, w, grid, e0, de, ne)
    rb = oracle_lib.dos_binned(eps, w, grid, e0, de, ne)
    for tile in range(len(tetra.TILE_SHAPES)):
        print(f"[case] nos {grid} norb={norb} tile {tetra.TILE_SHAPES[tile]}", flush=True)
        gn, gb = _run(torch, dev, eps, w, grid, e0, de, ne, tile=tile)
        assert _err(gn, rn) <= TOL and _err(gb, rb) <= TOL


def test_fp16_weights(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne = (12, 10, 9), 7, 90
    eps, w = synth.band_structure(norb, 9, grid)
    e0, de = _grid_inside(eps, ne, 0.1, 0.9)
    w16, scale = (t.cpu() for t in tetra.half_weights(torch.from_numpy(w).cuda()))
    deq = (w16.float() * scale[:, None, None]).numpy()
    rn = oracle_lib.nos(eps, deq, grid, e0, de, ne)
    rb = oracle_lib.dos_binned(eps, deq, grid, e0, de, ne)
    print(f"[case] nos fp16 weights {grid} norb={norb}", flush=True)
    gn, gb = _run(torch, dev, eps, w, grid, e0, de, ne, w16=w16, scale=scale)
    assert _err(gn, rn) <= TOL and _err(gb, rb) <= TOL


def test_signed_weights(torch_dev, oracle_lib):
    """A general observable X in place of b (eq. BZintegral) may be negative: the histogram then
    takes its signed 64-bit form."""
    torch, dev = torch_dev
    grid, norb, ne = (8, 9, 10), 6, 64
    eps, w = synth.band_structure(norb, 10, grid)
    x = (w - np.float32(0.3)).astype(np.float32)
    e0, de = _grid_inside(eps, ne, 0.0, 1.0)
    rn = oracle_lib.nos(eps, x, grid, e0, de, ne)
    rb = oracle_lib.dos_binned(eps, x, grid, e0, de, ne)
    print(f"[case] nos signed weights {grid} norb={norb}", flush=True)
    gn, gb = _run(torch, dev, eps, x, grid, e0, de, ne)
    assert _err(gn, rn) <= TOL and _err(gb, rb) <= TOL


@pytest.mark.parametrize("signed", [False, True])
def test_many_energies_several_histogram_passes(torch_dev, oracle_lib, signed):
    """16 orbitals and 3000 energies: a tile-band's index range exceeds one LDS histogram, so the
    kernel makes several passes and each starts one index early to know the weights there."""
    torch, dev = torch_dev
    grid, norb, ne = (5, 7, 3), 16, 3000
    eps, w = synth.band_structure(norb, 12, grid)
    if signed:
        w = (w - np.float32(0.05)).astype(np.float32)
    e0, de = _grid_inside(eps, ne, 0.05, 0.95)
    print(f"[case] nos {grid} norb={norb} ne={ne} signed={signed}", flush=True)
    rn = oracle_lib.nos(eps, w, grid, e0, de, ne)
    rb = oracle_lib.dos_binned(eps, w, grid, e0, de, ne)
    gn, gb = _run(torch, dev, eps, w, grid, e0, de, ne)
    en, eb = _err(gn, rn), _err(gb, rb)
    print(f"[case] err nos {en:.3e} binned {eb:.3e}", flush=True)
    assert en <= TOL and eb <= TOL


def test_non_finite_energies_are_skipped(torch_dev, oracle_lib):
    """A tetrahedron-band with a non-finite corner energy contributes nothing, below or above."""
    torch, dev = torch_dev
    grid, norb, ne = (5, 4, 6), 4, 90
    eps, w = synth.band_structure(norb, 9, grid)
    eps = eps.copy()
    eps[0, 3] = np.nan
    eps[2, 17] = np.inf
    eps[3, 40] = -np.inf
    e0, de = _grid_inside(np.nan_to_num(eps, nan=0.0, posinf=0.0, neginf=0.0), ne, 0.2, 0.9)
    print("[case] nos with non-finite energies", flush=True)
    rn = oracle_lib.nos(eps, w, grid, e0, de, ne)
    rb = oracle_lib.dos_binned(eps, w, grid, e0, de, ne)
    gn, gb = _run(torch, dev, eps, w, grid, e0, de, ne)
    assert _err(gn, rn) <= TOL and _err(gb, rb) <= TOL


def test_graph_capture_replays(torch_dev):
    """Both entry points allocate nothing and clear their outputs with kernels: one capture, several
    replays with eager work between them, every replay equal to the eager result."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne = (9, 7, 18), 5, 150
    eps, w = synth.band_structure(norb, 3, grid)
    e0, de = _grid_inside(eps, ne, 0.3, 0.8)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    on = torch.empty((ne, norb), device=dev)
    ob = torch.empty((ne, norb), device=dev)
    tetra.nos_forward(te, tw, grid, e0, de, ne, out=on)
    tetra.dos_binned(te, tw, grid, e0, de, ne, out=ob)
    en, eb = on.clone(), ob.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    print("[case] nos graph capture", flush=True)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tetra.nos_forward(te, tw, grid, e0, de, ne, out=on)
            tetra.dos_binned(te, tw, grid, e0, de, ne, out=ob)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        on.fill_(-1.0)  # eager work between replays
        ob.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.allclose(on, en, rtol=1e-6, atol=1e-6 * float(en.abs().max())), rep
        assert torch.allclose(ob, eb, rtol=1e-6, atol=1e-6 * float(eb.abs().max())), rep


def test_grid_outside_the_bands(torch_dev, oracle_lib):
    torch, dev = torch_dev
    grid, norb, ne = (7, 8, 9), 4, 50
    eps, w = synth.band_structure(norb, 11, grid)
    lo, hi = float(np.min(eps)), float(np.max(eps))
    print("[case] nos grid below every band", flush=True)
    gn, gb = _run(torch, dev, eps, w, grid, float(np.float32(lo - 3.0)), 0.01, ne)
    assert not gn.any() and not gb.any()
    print("[case] nos grid above every band", flush=True)
    e0 = float(np.float32(hi + 0.5))
    gn, gb = _run(torch, dev, eps, w, grid, e0, 0.01, ne)
    mean_b = w.astype(np.float64).sum(axis=(0, 2)) / eps.shape[1]
    rn = oracle_lib.nos(eps, w, grid, e0, 0.01, 1)
    assert _err(gn[0], rn[0]) <= TOL
    assert np.abs(rn[0] - mean_b).max() <= 1e-12
    assert (gn == gn[0]).all()  # one step at the first energy, nothing after it
    assert not gb.any()  # every increment falls below the first bin


def test_headline_size_sampled(torch_dev, oracle_lib):
    torch, dev = torch_dev
    c = synth.config("k64_b8_e1000")
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    eps, w = synth.band_structure(norb, c["seed"], grid)
    e0, de = synth.energy_grid(eps, ne)
    print(f"[case] nos 64^3 x 8 x 8 x {ne}", flush=True)
    gn, gb = _run(torch, dev, eps, w, grid, e0, de, ne)
    gn64, gb64 = gn.astype(np.float64), gb.astype(np.float64)
    mean_b = w.astype(np.float64).sum(axis=(0, 2)) / eps.shape[1]
    scale = np.abs(mean_b).max()
    # above every band (the grid spans the band range +- 10 %)
    assert np.abs(gn64[-1] - mean_b).max() <= TOL * scale
    assert (np.diff(gn64, axis=0) >= -1e-6 * scale).all()
    # the bins cover [e0 - de/2, e0 + (ne - 1/2) de]: nothing below, everything inside
    assert np.abs(gb64.sum(axis=0) * de - mean_b).max() <= TOL * scale
    rng = np.random.default_rng(12)
    for j in sorted(rng.choice(ne, size=4, replace=False)):
        E = float(np.float32(e0)) + int(j) * float(np.float32(de))
        rn = oracle_lib.nos(eps, w, grid, E, de, 1)[0]
        rb = oracle_lib.dos_binned(eps, w, grid, E, de, 1)[0]
        en = np.abs(gn64[j] - rn).max() / scale
        eb = np.abs(gb64[j] - rb).max() / np.abs(gb64).max()
        print(f"[case] j={j}: nos err {en:.3e}, binned err {eb:.3e}", flush=True)
        assert en <= TOL and eb <= TOL
