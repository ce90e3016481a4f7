"""GPU test of the allocation-free forward (tetra_dos_forward_noalloc, the exact path on the library's
static device scratch): through the C ABI, its result equals that of tetra_dos_forward_ws with a
caller-owned workspace bit for bit (the exact accumulation is order-independent), and matches the FP64
oracle to the DOS gate, on two calls in a row, the second with a smaller problem (fewer energies and
orbitals, another grid), so that the scratch left by the first call must not leak into the second."""
import ctypes

import numpy as np
import pytest

import synth
from gates import dos_err

pytestmark = pytest.mark.gpu

CASES = [  # (grid, norb, ne, seed): the second is smaller in every size
    ((16, 16, 16), 8, 400, 0),
    ((12, 10, 8), 5, 150, 3),
]


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _ws_call(tetra, torch, dev, eps, w, grid, e0, de, ne, flags):
    """The existing entry point, tetra_dos_forward_ws, with a workspace of the size it asks for."""
    nb, norb, _ = w.shape
    d = tetra.make_desc(grid, nb, norb, e0, de, ne)
    need = tetra.lib().tetra_dos_forward_workspace(ctypes.byref(d), flags)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = torch.full((ne, norb), float("nan"), device=dev)
    st = tetra.lib().tetra_dos_forward_ws(ctypes.byref(d), eps.data_ptr(), w.data_ptr(), 0, None, out.data_ptr(),
                                          flags, ws.data_ptr(), ws.numel(), ctypes.c_void_p(0))
    assert st == 0, tetra.lib().tetra_status_string(st)
    return out


def _noalloc_call(tetra, torch, dev, eps, w, grid, e0, de, ne, flags):
    nb, norb, _ = w.shape
    d = tetra.make_desc(grid, nb, norb, e0, de, ne)
    out = torch.full((ne, norb), float("nan"), device=dev)
    st = tetra.lib().tetra_dos_forward_noalloc(ctypes.byref(d), eps.data_ptr(), w.data_ptr(), 0, None,
                                               out.data_ptr(), flags, ctypes.c_void_p(0))
    assert st == 0, tetra.lib().tetra_status_string(st)
    return out


@pytest.mark.parametrize("flags", [1, 2 | (3 << 8)], ids=["exact", "deterministic-tile3"])
def test_noalloc_matches_workspace_entry_point_on_two_calls(torch_dev, oracle_lib, flags):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    for grid, norb, ne, seed in CASES:
        eps, w = synth.band_structure(norb, seed, grid)
        e0, de = synth.energy_grid(eps, ne)
        ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
        te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
        print(f"[case] noalloc flags={flags:#x} grid={grid} norb={norb} ne={ne} seed={seed}", flush=True)
        got = _noalloc_call(tetra, torch, dev, te, tw, grid, e0, de, ne, flags)
        want = _ws_call(tetra, torch, dev, te, tw, grid, e0, de, ne, flags)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        err = dos_err(got.cpu().numpy().astype(np.float64), ref)
        print(f"[case] err vs oracle {err:.3e}", flush=True)
        assert err <= 1e-5


def test_noalloc_plain_path_and_binding(torch_dev, oracle_lib):
    """Without the exact flags the scratch is unused: the plain forward, within the DOS gate; the
    Python binding's wrapper calls the same entry point and rejects an exact problem beyond the
    scratch."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne, seed = CASES[1]
    eps, w = synth.band_structure(norb, seed, grid)
    e0, de = synth.energy_grid(eps, ne)
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    te, tw = torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev)
    out = torch.empty((ne, norb), device=dev)
    tetra.dos_forward_noalloc(te, tw, grid, e0, de, ne, out)
    torch.cuda.synchronize()
    assert dos_err(out.cpu().numpy().astype(np.float64), ref) <= 1e-5
    ex = torch.empty((ne, norb), device=dev)
    tetra.dos_forward_noalloc(te, tw, grid, e0, de, ne, ex, exact=True)
    want = tetra.dos_forward(te, tw, grid, e0, de, ne, exact=True)
    torch.cuda.synchronize()
    assert torch.equal(ex, want)
    big_ne = tetra.NOALLOC_MAX_BINS // norb + 1
    big = torch.empty((big_ne, norb), device=dev)
    with pytest.raises(tetra.TetraError) as info:
        tetra.dos_forward_noalloc(te, tw, grid, e0, de, big_ne, big, exact=True)
    assert info.value.status == tetra.TETRA_ERR_SCRATCH
