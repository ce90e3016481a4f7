"""GPU parity of the forward kernel (through the C ABI) against the FP64 oracle.

Gate: err = max_{j,m} |D_gpu - D_ref| / max_{j,m} |D_ref| <= 1e-5 for FP32 (pointwise relative error
is undefined where the DOS vanishes)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _gpu_dos(torch_dev, eps, w, grid, e0, de, ne):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    out = tetra.dos_forward(torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), grid, e0, de, ne)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _err(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / scale if scale > 0 else np.abs(got).max()


def _check(torch_dev, oracle_lib, eps, w, grid, e0, de, ne, tol=TOL_F32):
    print(f"[case] grid={grid} nb={eps.shape[0]} norb={w.shape[1]} ne={ne} e0={e0} de={de}", flush=True)
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    got = _gpu_dos(torch_dev, eps, w, grid, e0, de, ne)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    err = _err(got, ref)
    print(f"[case] err={err:.3e}", flush=True)
    assert err <= tol, err
    return got, ref


def test_parity_16cube_8orb_200E(torch_dev, oracle_lib):
    c = synth.config("k16_b8_e200")
    eps, w = synth.band_structure(c["norb"], c["seed"], c["grid"])
    e0, de = synth.energy_grid(eps, c["ne"])
    _check(torch_dev, oracle_lib, eps, w, c["grid"], e0, de, c["ne"])


@pytest.mark.parametrize("norb", [1, 3, 8, 16])
@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 1, 3), (5, 7, 3), (9, 6, 21)])
def test_parity_small_and_ragged_grids(torch_dev, oracle_lib, grid, norb):
    eps, w = synth.band_structure(norb, 7 + norb, grid)
    e0, de = synth.energy_grid(eps, 150)
    _check(torch_dev, oracle_lib, eps, w, grid, e0, de, 150)


def test_parity_energy_chunking(torch_dev, oracle_lib):
    """A dense energy grid makes a tile-band span more bins than one LDS histogram pass holds."""
    grid = (6, 5, 20)
    eps, w = synth.band_structure(16, 3, grid)
    e0, de = synth.energy_grid(eps, 6000)
    _check(torch_dev, oracle_lib, eps, w, grid, e0, de, 6000)


def test_flat_and_separable_bands(torch_dev, oracle_lib):
    grid = (6, 4, 5)
    nk = 120
    rng = np.random.default_rng(1)
    f = rng.uniform(-1, 1, 6).astype(np.float32)
    eps = np.stack([np.full(nk, 0.25, np.float32),  # flat band: contributes nothing
                    np.repeat(f, 20).astype(np.float32)])
    w = np.ones((2, 1, nk), np.float32)
    got, ref = _check(torch_dev, oracle_lib, eps, w, grid, -1.2, 0.0137, 180)
    assert np.abs(ref).max() > 0


def test_non_finite_energies_are_skipped(torch_dev, oracle_lib):
    grid = (5, 4, 6)
    eps, w = synth.band_structure(4, 9, grid)
    eps = eps.copy()
    eps[0, 3] = np.nan
    eps[2, 17] = np.inf
    eps[3, 40] = -np.inf
    e0, de = synth.energy_grid(np.nan_to_num(eps, nan=0.0, posinf=0.0, neginf=0.0), 120)
    _check(torch_dev, oracle_lib, eps, w, grid, e0, de, 120)


def test_energy_grid_outside_bands_gives_zero(torch_dev, oracle_lib):
    grid = (4, 4, 4)
    eps, w = synth.band_structure(3, 2, grid)
    got = _gpu_dos(torch_dev, eps, w, grid, 100.0, 0.1, 50)
    assert np.all(got == 0)
    got = _gpu_dos(torch_dev, eps, w, grid, -100.0, 0.1, 50)
    assert np.all(got == 0)


def test_single_energy_and_output_overwritten(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (4, 5, 6)
    eps, w = synth.band_structure(5, 4, grid)
    E = float(np.float32(np.median(eps)))
    ref, _ = oracle_lib.dos(eps, w, grid, E, 1.0, 1)
    out = torch.full((1, 5), 123.0, device=dev)
    tetra.dos_forward(torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), grid, E, 1.0, 1, out=out)
    torch.cuda.synchronize()
    assert _err(out.cpu().numpy(), ref) <= TOL_F32


def test_parity_64cube_8orb_1000E_full(torch_dev, oracle_lib):
    """The headline workload at full size, every output element against the oracle, plus the spread
    between repeated runs (float atomics make the summation order vary)."""
    c = synth.config("k64_b8_e1000")
    eps, w = synth.band_structure(c["norb"], c["seed"], c["grid"])
    e0, de = synth.energy_grid(eps, c["ne"])
    got, ref = _check(torch_dev, oracle_lib, eps, w, c["grid"], e0, de, c["ne"])
    again = _gpu_dos(torch_dev, eps, w, c["grid"], e0, de, c["ne"])
    assert _err(again, got) <= 1e-6


def test_signed_weights_use_the_wide_accumulator(torch_dev, oracle_lib):
    """Weights of both signs (a general observable in place of b): every bin's sum stays exact."""
    grid = (6, 5, 20)
    eps, w = synth.band_structure(3, 4, grid)
    w = (w - 0.4).astype(np.float32)
    e0, de = synth.energy_grid(eps, 180)
    _check(torch_dev, oracle_lib, eps, w, grid, e0, de, 180)


def test_nearly_flat_band(torch_dev, oracle_lib):
    """Spans far below the energy step: point values spike, and the workgroup bound is dominated by
    narrow tetrahedra."""
    grid = (8, 6, 20)
    rng = np.random.default_rng(3)
    eps = (0.3 + 1e-4 * rng.standard_normal((2, 960))).astype(np.float32)
    eps[1] += 0.2
    w = rng.uniform(0, 1, (2, 4, 960)).astype(np.float32)
    _check(torch_dev, oracle_lib, eps, w, grid, 0.25, 0.013, 30)


def _fp16_inputs(w):
    """Per-band power-of-two scale (exact), FP16 mantissa rounding: the precision variant's weights."""
    import torch

    import paper_1710_10789_amd as tetra

    w16, scale = (t.cpu() for t in tetra.half_weights(torch.from_numpy(w).cuda()))
    deq = (w16.float() * scale[:, None, None]).numpy()
    return w16, scale, deq


def test_fp16_weights(torch_dev, oracle_lib):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (12, 10, 16)
    eps, w = synth.band_structure(16, 5, grid)
    e0, de = synth.energy_grid(eps, 400)
    w16, scale, deq = _fp16_inputs(w)
    got = tetra.dos_forward(torch.from_numpy(eps).to(dev), w16.to(dev), grid, e0, de, 400, w_scale=scale.to(dev))
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    ref32, _ = oracle_lib.dos(eps, w, grid, e0, de, 400)     # against the FP32 weights: FP16 gate
    refdq, _ = oracle_lib.dos(eps, deq, grid, e0, de, 400)   # against the dequantised weights: FP32 gate
    e32, edq = _err(got, ref32), _err(got, refdq)
    print(f"[case] fp16 err vs fp32 weights {e32:.3e}, vs dequantised {edq:.3e}", flush=True)
    assert e32 <= 1e-3 and edq <= TOL_F32


@pytest.mark.parametrize("grid,norb,ne", [((16, 16, 16), 8, 200), ((5, 7, 3), 3, 150), ((9, 6, 21), 16, 3000)])
def test_exact_accumulation_mode(torch_dev, oracle_lib, grid, norb, ne):
    """TETRA_EXACT: exact cross-workgroup sums; parity with the oracle and bitwise reproducibility."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    eps, w = synth.band_structure(norb, 2, grid)
    e0, de = synth.energy_grid(eps, ne)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    a = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True)
    b = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True)
    torch.cuda.synchronize()
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    err = _err(a.cpu().numpy().astype(np.float64), ref)
    print(f"[case] exact-mode err {err:.3e}", flush=True)
    assert err <= TOL_F32
    assert torch.equal(a, b)


def test_exact_mode_every_tile_shape_and_graph_replays(torch_dev, oracle_lib):
    """TETRA_EXACT on every tile shape: oracle parity and bitwise repeats; the exact forward (set-up,
    bound pass, main pass, conversion, all plain kernels into the caller's workspace) captured in a
    HIP graph and replayed several times with eager work in between, every replay bitwise equal to
    the eager call."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne = (16, 16, 32), 8, 300
    eps, w = synth.band_structure(norb, 6, grid)
    e0, de = synth.energy_grid(eps, ne)
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    for tile in range(len(tetra.TILE_SHAPES)):
        print(f"[case] exact mode, tile {tile}", flush=True)
        a = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True, tile=tile)
        b = tetra.dos_forward(te, tw, grid, e0, de, ne, deterministic=True, tile=tile)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert _err(a.cpu().numpy().astype(np.float64), ref) <= TOL_F32
    nbytes = tetra.forward_workspace_bytes(grid, norb, norb, e0, de, ne, exact=True)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.empty((ne, norb), device=dev)
    eager = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True, workspace=ws).clone()
    print("[case] exact mode in a HIP graph", flush=True)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True, workspace=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(3):
        out.fill_(float("nan"))
        ws.fill_(0xA5)  # stale workspace contents must not matter
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), r
        tetra.dos_forward(te, tw * 0.5, grid, e0, de, ne)  # eager work in between
        torch.cuda.synchronize()
