"""GPU parity of the susceptibility kernel (tetra_chi_spectral, through the C ABI) against the FP64
oracle's spectral weight S_m(q, w) (Im chi_0 = -pi S), element by element.

Gate: max |S - S_ref| / max |S_ref| <= 1e-5 (FP32 arithmetic; the clipping at the Fermi energy runs in
FP32 on the kernel side). Cases: small and ragged grids (every tile shape on one of them), transfers of
both signs and zero, one to sixteen orbitals, a symmetric transfer-energy grid (both signs of w),
FP16 weights and complex amplitudes (against the oracle on the weights the kernel sees), non-finite
energies, bands that straddle E_F everywhere (every region clipped: the kernel's queue of regions to
clip at its capacity), and the 64^3 x 8 x 8 workload with 500 transfer energies in full. The binding
calls tetra_chi_spectral_ws (a first pass of per-(tile, band) energy ranges); its result is also
compared with tetra_chi_spectral's."""
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


def _grid_for(eps, nw, symmetric):
    """Transfer energies over the band width: w in [0, W] or symmetric [-W, W] (FP32 values)."""
    width = float(eps[np.isfinite(eps)].max() - eps[np.isfinite(eps)].min())
    if symmetric:
        dw = float(np.float32(2.0 * width / (nw - 1)))
        return float(np.float32(-(nw - 1) / 2 * dw)), dw
    return 0.0, float(np.float32(width / (nw - 1)))


def _run(torch_dev, eps, w, grid, q, ef, w0, dw, nw, tile=None, w_scale=None):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    te = torch.from_numpy(np.ascontiguousarray(eps)).to(dev)
    tw = w.to(dev) if isinstance(w, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(w)).to(dev)
    out = torch.full((nw, tw.shape[1]), float("nan"), device=dev)
    tetra.chi_spectral(te, tw, grid, q, ef, w0, dw, nw, out=out, tile=tile,
                       w_scale=w_scale.to(dev) if w_scale is not None else None)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


CASES = [  # grid, bands = orbitals, transfer, symmetric energy grid
    ((4, 3, 5), 2, (1, 0, 2), True),
    ((6, 5, 4), 3, (-2, 1, 0), False),
    ((8, 8, 8), 1, (3, 0, 0), True),
    ((5, 7, 3), 4, (0, 0, 0), True),
    ((9, 6, 21), 3, (4, -2, 7), False),
    ((12, 10, 8), 8, (3, 3, 0), False),
]


@pytest.mark.parametrize("grid,nb,q,symmetric", CASES)
def test_parity_small_and_ragged(torch_dev, oracle_lib, grid, nb, q, symmetric):
    eps, w = synth.band_structure(nb, 5 + nb, grid)
    ef = float(np.float32(np.median(eps)))
    nw = 120
    w0, dw = _grid_for(eps, nw, symmetric)
    print(f"[case] chi grid={grid} nb=norb={nb} q={q} nw={nw} symmetric={symmetric}", flush=True)
    ref, nsub = oracle_lib.chi(eps, w, grid, q, ef, w0, dw, nw)
    got = _run(torch_dev, eps, w, grid, q, ef, w0, dw, nw)
    err = dos_err(got, ref)
    print(f"[case] err {err:.3e} (oracle: {nsub} updates, max |S| {np.abs(ref).max():.3e})", flush=True)
    assert np.abs(ref).max() > 0
    assert err <= 1e-5


@pytest.mark.parametrize("norb", [1, 5, 16])
def test_orbital_counts(torch_dev, oracle_lib, norb):
    grid = (6, 6, 6)
    eps, w = synth.band_structure(norb, 30 + norb, grid)
    ef = float(np.float32(np.mean(eps)))
    w0, dw = _grid_for(eps, 90, True)
    print(f"[case] chi grid={grid} norb={norb}", flush=True)
    ref, _ = oracle_lib.chi(eps, w, grid, (2, 1, 3), ef, w0, dw, 90)
    got = _run(torch_dev, eps, w, grid, (2, 1, 3), ef, w0, dw, 90)
    assert dos_err(got, ref) <= 1e-5


def test_every_tile_shape(torch_dev, oracle_lib):
    grid = (16, 16, 16)
    eps, w = synth.band_structure(4, 2, grid)
    ef = float(np.float32(np.median(eps)))
    w0, dw = _grid_for(eps, 150, False)
    ref, _ = oracle_lib.chi(eps, w, grid, (4, 0, 0), ef, w0, dw, 150)
    for tile in range(6):
        print(f"[case] chi 16^3 nb=4 tile={tile}", flush=True)
        got = _run(torch_dev, eps, w, grid, (4, 0, 0), ef, w0, dw, 150, tile=tile)
        assert dos_err(got, ref) <= 1e-5


def test_fp16_weights_and_complex_amplitudes(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (8, 6, 10)
    nb = 4
    eps, w = synth.band_structure(nb, 12, grid)
    ef = float(np.float32(np.median(eps)))
    w0, dw = _grid_for(eps, 100, True)
    w16, scale = tetra.half_weights(torch.from_numpy(w).to(dev))
    deq = (w16.float() * scale[:, None, None]).cpu().numpy()
    ref16, _ = oracle_lib.chi(eps, deq, grid, (3, 2, 1), ef, w0, dw, 100)
    print("[case] chi fp16 weights", flush=True)
    got16 = _run(torch_dev, eps, w16, grid, (3, 2, 1), ef, w0, dw, 100, w_scale=scale)
    assert dos_err(got16, ref16) <= 1e-5
    eps_a, amp = synth.amplitudes(nb, 12, grid)
    wa = (np.abs(amp) ** 2).astype(np.float32)
    refa, _ = oracle_lib.chi(eps_a, wa, grid, (3, 2, 1), ef, w0, dw, 100)
    print("[case] chi complex amplitudes", flush=True)
    gota = _run(torch_dev, eps_a, torch.from_numpy(amp), grid, (3, 2, 1), ef, w0, dw, 100)
    assert dos_err(gota, refa) <= 1e-5


def test_non_finite_energies_drop_their_pairs(torch_dev, oracle_lib):
    grid = (5, 4, 6)
    eps, w = synth.band_structure(3, 9, grid)
    eps = eps.copy()
    eps[0, 3] = np.nan
    eps[2, 17] = np.inf
    fin = eps[np.isfinite(eps)]
    ef = float(np.float32(np.median(fin)))
    w0, dw = _grid_for(fin, 80, True)
    ref, _ = oracle_lib.chi(eps, w, grid, (1, 1, 1), ef, w0, dw, 80)
    got = _run(torch_dev, eps, w, grid, (1, 1, 1), ef, w0, dw, 80)
    assert np.all(np.isfinite(got))
    assert dos_err(got, ref) <= 1e-5


def test_full_size_64cube_8x8_500w(torch_dev, oracle_lib):
    c = synth.config("chi_k64_b8_w500")
    grid, norb, nw = c["grid"], c["norb"], c["nw"]
    eps, w = synth.band_structure(norb, c["seed"], grid)
    ef, w0, dw = synth.chi_grid(eps, nw)
    print(f"[case] chi {grid} 8x8 q={c['q']} nw={nw}", flush=True)
    ref, nsub = oracle_lib.chi(eps, w, grid, c["q"], ef, w0, dw, nw)
    got = _run(torch_dev, eps, w, grid, c["q"], ef, w0, dw, nw)
    err = dos_err(got, ref)
    print(f"[case] err {err:.3e}, {nsub} updates", flush=True)
    assert err <= 1e-5


def test_signed_weights_use_the_signed_accumulator(torch_dev, oracle_lib):
    """General observables in place of b (negative products W): one signed 64-bit histogram."""
    rng = np.random.default_rng(31)
    grid = (7, 6, 5)
    eps, w = synth.band_structure(3, 17, grid)
    w = (w * rng.choice([-1.0, 1.0], size=w.shape)).astype(np.float32)
    ef = float(np.float32(np.median(eps)))
    w0, dw = _grid_for(eps, 100, True)
    ref, _ = oracle_lib.chi(eps, w, grid, (2, 3, 1), ef, w0, dw, 100)
    print("[case] chi signed weights", flush=True)
    got = _run(torch_dev, eps, w, grid, (2, 3, 1), ef, w0, dw, 100)
    assert np.abs(ref).max() > 0
    assert dos_err(got, ref) <= 1e-5


def test_every_region_clipped(torch_dev, oracle_lib):
    """Both bands a little random noise around E_F at every point: nearly every region of every
    tetrahedron straddles a Fermi plane, so the kernel queues both regions of nearly all six
    tetrahedra of every cube (its queue's capacity) and works the clipped pieces off in many rounds
    of the whole workgroup; 16^3 grid, 2 bands, 3 orbitals, both signs of w."""
    rng = np.random.default_rng(47)
    grid = (16, 16, 16)
    nb, norb, nk = 2, 3, 16 * 16 * 16
    eps = (0.05 * rng.standard_normal((nb, nk))).astype(np.float32)
    w = rng.random((nb, norb, nk)).astype(np.float32)
    ef = 0.0
    w0, dw = _grid_for(eps, 64, True)
    print("[case] chi every region clipped 16^3 nb=2 norb=3", flush=True)
    ref, nsub = oracle_lib.chi(eps, w, grid, (2, 1, 0), ef, w0, dw, 64)
    got = _run(torch_dev, eps, w, grid, (2, 1, 0), ef, w0, dw, 64)
    err = dos_err(got, ref)
    print(f"[case] err {err:.3e}, {nsub} updates", flush=True)
    assert np.abs(ref).max() > 0
    assert err <= 1e-5


@pytest.mark.parametrize("case", ["ragged", "clipped", "full"])
def test_first_pass_ranges_match_the_plain_call(torch_dev, oracle_lib, case):
    """tetra_chi_spectral_ws (a first pass writes every (tile, band)'s energy ranges; units that cannot
    contribute leave before loading anything) against tetra_chi_spectral on the same inputs: equal
    within the order of the float atomics that add the units' partial sums (1e-5 of the largest value;
    a unit skipped wrongly moves its bins by far more), and the ranges path against the oracle."""
    torch, dev = torch_dev
    if case == "ragged":
        grid, nb, q, symmetric = (9, 6, 21), 3, (4, -2, 7), True
        eps, w = synth.band_structure(nb, 8, grid)
        ef = float(np.float32(np.median(eps)))
        nw = 120
        w0, dw = _grid_for(eps, nw, symmetric)
    elif case == "clipped":
        rng = np.random.default_rng(53)
        grid, q, nw = (16, 16, 8), (3, 0, 1), 64
        eps = (0.05 * rng.standard_normal((2, 16 * 16 * 8))).astype(np.float32)
        w = rng.random((2, 3, 16 * 16 * 8)).astype(np.float32)
        ef = 0.0
        w0, dw = _grid_for(eps, nw, True)
    else:
        c = synth.config("chi_k64_b8_w500")
        grid, nw, q = c["grid"], c["nw"], c["q"]
        eps, w = synth.band_structure(c["norb"], c["seed"], grid)
        ef, w0, dw = synth.chi_grid(eps, nw)
    import paper_1710_10789_amd as tetra

    te, tw = torch.from_numpy(np.ascontiguousarray(eps)).to(dev), torch.from_numpy(np.ascontiguousarray(w)).to(dev)
    print(f"[case] chi first-pass ranges, {case}: grid {grid} nb {eps.shape[0]} norb {w.shape[1]}", flush=True)
    for tile in (0, 3):
        plain = tetra.chi_spectral(te, tw, grid, q, ef, w0, dw, nw, tile=tile, ranges=False)
        ws = torch.empty(tetra.chi_workspace_bytes(grid, eps.shape[0], w.shape[1], w0, dw, nw, tile=tile),
                         dtype=torch.uint8, device=dev)
        fast = tetra.chi_spectral(te, tw, grid, q, ef, w0, dw, nw, tile=tile, workspace=ws)
        torch.cuda.synchronize()
        a, b = fast.cpu().numpy().astype(np.float64), plain.cpu().numpy().astype(np.float64)
        diff = np.abs(a - b).max() / np.abs(b).max()
        print(f"[case] tile {tile}: ranges vs plain {diff:.2e}", flush=True)
        assert np.abs(b).max() > 0 and diff <= 1e-5
    ref, _ = oracle_lib.chi(eps, w, grid, q, ef, w0, dw, nw)
    assert dos_err(a, ref) <= 1e-5
