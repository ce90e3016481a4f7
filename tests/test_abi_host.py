"""Host-side checks of the C ABI (no GPU): the library loads, exports every function declared in
include/tetra.h, and rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_1710_10789_amd as tetra

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tetra.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tetra_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(tetra.library_path()):
        from paper_1710_10789_amd import build

        build.build()
    return tetra.lib()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("tetra_dos_forward", "tetra_dos_forward_ws", "tetra_dos_forward_workspace", "tetra_dos_backward",
              "tetra_dos_backward_ws", "tetra_dos_backward_workspace", "tetra_dos_batched",
              "tetra_dos_batched_workspace", "tetra_pack_f16",
              "tetra_nos_forward", "tetra_dos_binned", "tetra_status_string", "tetra_last_hip_error",
              "tetra_version"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_measurement_probe_is_not_in_the_product_library(L):
    """The LDS-atomic and FMA probes are benchmark helpers of their own library, not part of the C ABI."""
    assert "tetra_probe" not in open(HEADER).read()
    assert not hasattr(L, "tetra_probe_lds_atomics")
    assert not hasattr(L, "tetra_probe_fma_f32")


def test_status_strings(L):
    assert L.tetra_status_string(0) == b"ok"
    assert L.tetra_status_string(-1) == b"invalid argument"
    assert L.tetra_status_string(-2) == b"unsupported request"
    assert L.tetra_status_string(-3) == b"workspace missing or too small"
    assert L.tetra_status_string(-4) == b"HIP runtime error"
    assert b"static scratch" in L.tetra_status_string(-5)
    assert L.tetra_status_string(123) == b"unknown status"
    assert L.tetra_version() >= 100


FAKE = 0x1000  # never dereferenced: validation fails before any launch


def _fwd(L, d, eps=FAKE, w=FAKE, wtype=0, scale=None, dos=FAKE, flags=0):
    return L.tetra_dos_forward(ctypes.byref(d) if d is not None else None, eps, w, wtype, scale, dos, flags, None)


def _bwd(L, d, gd=FAKE, ge=FAKE, gw=FAKE, flags=0, wtype=0, scale=None):
    return L.tetra_dos_backward(ctypes.byref(d), FAKE, FAKE, wtype, scale, gd, ge, gw, flags, None)


def good():
    return tetra.make_desc((4, 4, 4), 2, 3, -1.0, 0.01, 100)


@pytest.mark.parametrize(
    "field,value,status",
    [
        ("n1", 0, -1), ("n2", -3, -1), ("n3", 0, -1), ("nb", 0, -1), ("norb", 0, -1), ("ne", 0, -1),
        ("de", 0.0, -1), ("de", -0.5, -1), ("de", float("nan"), -1), ("e0", float("inf"), -1),
        ("e0", float("nan"), -1), ("norb", 17, -2), ("ne", (1 << 22) + 1, -1), ("n1", 1 << 28, -1),
    ],
)
def test_forward_rejects_bad_descriptors(L, field, value, status):
    d = good()
    setattr(d, field, value)
    assert _fwd(L, d) == status


def test_forward_rejects_bad_pointers_and_flags(L):
    assert _fwd(L, None) == -1
    assert _fwd(L, good(), eps=None) == -1
    assert _fwd(L, good(), w=None) == -1
    assert _fwd(L, good(), dos=None) == -1
    assert _fwd(L, good(), wtype=7) == -1
    assert _fwd(L, good(), wtype=0, scale=FAKE) == -1  # FP32 weights take no scale
    assert _fwd(L, good(), wtype=1, scale=None) == -1  # FP16 weights need a scale
    assert _fwd(L, good(), flags=8) == -1
    d = good()
    d.e0, d.de, d.ne = 3.0e38, 1.0e37, 1000  # last grid energy overflows FP32
    assert _fwd(L, d) == -1
    assert _fwd(L, good(), flags=7 << 8) == -1  # no such tile shape
    assert _fwd(L, good(), flags=15 << 8) == -1
    assert _fwd(L, good(), flags=1) == -3  # exact mode needs a workspace
    assert _fwd(L, good(), flags=2 | (3 << 8)) == -3  # deterministic (= exact) mode likewise


def _fwd_ws(L, d, ws, ws_bytes, flags=0):
    return L.tetra_dos_forward_ws(ctypes.byref(d), FAKE, FAKE, 0, None, FAKE, flags, ws, ws_bytes, None)


def test_forward_workspace_sizes_and_checks(L):
    d = good()
    need = 256 + 8 * d.ne * d.norb
    for flags in (1, 2, 3, 1 | (5 << 8)):
        assert L.tetra_dos_forward_workspace(ctypes.byref(d), flags) == need
    assert L.tetra_dos_forward_workspace(ctypes.byref(d), 0) == 0
    assert L.tetra_dos_forward_workspace(ctypes.byref(d), 3 << 8) == 0
    assert L.tetra_dos_forward_workspace(ctypes.byref(d), 0x10) == 0  # unknown flag
    assert L.tetra_dos_forward_workspace(ctypes.byref(d), 1 | (6 << 8)) == 0  # no such tile shape
    bad = good()
    bad.de = -1.0
    assert L.tetra_dos_forward_workspace(ctypes.byref(bad), 1) == 0
    assert tetra.forward_workspace_bytes((4, 4, 4), 2, 3, -1.0, 0.01, 100, exact=True) == need
    assert _fwd_ws(L, d, FAKE, need - 1, flags=1) == -3  # too small
    assert _fwd_ws(L, d, None, need, flags=1) == -3  # missing
    assert _fwd_ws(L, d, FAKE + 8, need, flags=1) == -1  # misaligned
    assert _fwd_ws(L, bad, FAKE, need, flags=1) == -1
    assert _fwd_ws(L, d, FAKE, need, flags=0x40) == -1  # unknown flag


def _fwd_na(L, d, flags=0, eps=FAKE, dos=FAKE):
    return L.tetra_dos_forward_noalloc(ctypes.byref(d) if d is not None else None, eps, FAKE, 0, None, dos, flags,
                                       None)


def test_noalloc_forward_rejects_before_any_hip_call(L):
    """The allocation-free forward validates like tetra_dos_forward_ws and refuses exact problems
    beyond its static scratch (TETRA_NOALLOC_MAX_BINS) with TETRA_ERR_SCRATCH, all without a GPU."""
    text = open(HEADER).read()
    assert f"#define TETRA_NOALLOC_MAX_BINS {tetra.NOALLOC_MAX_BINS}" in text
    d = good()
    assert _fwd_na(L, None) == -1
    assert _fwd_na(L, d, eps=None) == -1
    assert _fwd_na(L, d, dos=None) == -1
    assert _fwd_na(L, d, flags=0x40) == -1  # unknown flag
    assert _fwd_na(L, d, flags=1 | (6 << 8)) == -1  # no such tile shape
    big = good()
    big.norb, big.ne = 16, tetra.NOALLOC_MAX_BINS // 16 + 1
    for flags in (1, 2, 3, 1 | (2 << 8)):
        assert _fwd_na(L, big, flags=flags) == -5
    bad = good()
    bad.de = 0.0
    assert _fwd_na(L, bad, flags=1) == -1


def test_chi_rejects_bad_arguments(L):
    f = L.tetra_chi_spectral

    def call(d=None, ef=0.0, eps=FAKE, w=FAKE, wtype=0, scale=None, out=FAKE, flags=0):
        return f(ctypes.byref(d if d is not None else good()), 1, 0, -1, ef, eps, w, wtype, scale, out, flags, None)

    assert call(ef=float("nan")) == -1
    assert call(ef=float("inf")) == -1
    assert call(eps=None) == -1
    assert call(w=None) == -1
    assert call(out=None) == -1
    assert call(wtype=1) == -1  # FP16 weights need their scale
    assert call(wtype=0, scale=FAKE) == -1
    assert call(flags=0x40) == -1
    assert call(flags=7 << 8) == -1
    assert call(flags=1) == -2  # no exact accumulation here
    assert call(flags=2) == -2
    bad = good()
    bad.de = -1.0
    assert call(d=bad) == -1
    many = good()
    many.n1, many.n2, many.n3, many.nb, many.norb = 64, 64, 64, 8000, 1  # nb^2 x tiles workgroups >= 2^31
    assert call(d=many) == -2


def test_chi_workspace_sizes_and_checks(L):
    """tetra_chi_spectral_workspace: 16 nb T bytes (two 8-byte energy ranges per (tile, band)), 0 for
    bad arguments; tetra_chi_spectral_ws rejects a short or misaligned workspace before any launch and
    validates the rest as tetra_chi_spectral does."""
    shapes = [(4, 4, 16), (8, 8, 4), (4, 8, 8), (8, 4, 8), (4, 16, 4), (16, 4, 4)]
    for sid, (a, b, c) in enumerate(shapes):
        for grid in ((64, 64, 64), (9, 6, 21), (1, 1, 1)):
            d = tetra.make_desc(grid, 3, 2, 0.0, 0.01, 100)
            tiles = -(-grid[0] // a) * -(-grid[1] // b) * -(-grid[2] // c)
            assert L.tetra_chi_spectral_workspace(ctypes.byref(d), sid << 8) == 16 * 3 * tiles, (sid, grid)
            assert tetra.chi_workspace_bytes(grid, 3, 2, 0.0, 0.01, 100, tile=sid) == 16 * 3 * tiles
    assert L.tetra_chi_spectral_workspace(ctypes.byref(good()), 1) == 0  # no exact accumulation here
    assert L.tetra_chi_spectral_workspace(ctypes.byref(good()), 6 << 8) == 0  # no such tile shape
    bad = good()
    bad.nb = 0
    assert L.tetra_chi_spectral_workspace(ctypes.byref(bad), 0) == 0
    f = L.tetra_chi_spectral_ws
    d = good()
    need = L.tetra_chi_spectral_workspace(ctypes.byref(d), 0)
    assert need > 0

    def call(ws, ws_bytes, ef=0.0, eps=FAKE, flags=0):
        return f(ctypes.byref(d), 1, 0, -1, ef, eps, FAKE, 0, None, FAKE, flags, ws, ws_bytes, None)

    assert call(FAKE, need - 1) == -3  # too small
    assert call(FAKE + 8, need) == -1  # misaligned
    assert call(FAKE, need, ef=float("nan")) == -1
    assert call(FAKE, need, eps=None) == -1
    assert call(FAKE, need, flags=1) == -2


def test_pack_f16_rejects_bad_arguments(L):
    f = L.tetra_pack_f16
    assert f(0, 2, 3, FAKE, FAKE, FAKE, None) == -1
    assert f(2, 0, 3, FAKE, FAKE, FAKE, None) == -1
    assert f(2, 2, -1, FAKE, FAKE, FAKE, None) == -1
    assert f(2, 2, 3, None, FAKE, FAKE, None) == -1
    assert f(2, 2, 3, FAKE, None, FAKE, None) == -1
    assert f(2, 2, 3, FAKE, FAKE, None, None) == -1
    assert f(1 << 16, 1 << 8, 1 << 7, FAKE, FAKE, FAKE, None) == -1  # 2^31 elements


def test_backward_rejects_bad_arguments(L):
    assert _bwd(L, good(), gd=None) == -1
    assert _bwd(L, good(), ge=None, gw=None) == -1
    d = good()
    d.norb = 40
    assert _bwd(L, d) == -2
    assert _bwd(L, good(), flags=4) == -1
    assert _bwd(L, good(), flags=9 << 8) == -1
    assert _bwd(L, good(), flags=2) == -2  # no deterministic adjoint


@pytest.mark.parametrize("name", ["tetra_nos_forward", "tetra_dos_binned"])
def test_number_of_states_rejects_bad_arguments(L, name):
    f = getattr(L, name)

    def call(d=None, eps=FAKE, w=FAKE, wtype=0, scale=None, out=FAKE, flags=0):
        d = good() if d is None else d
        return f(ctypes.byref(d), eps, w, wtype, scale, out, flags, None)

    assert f(None, FAKE, FAKE, 0, None, FAKE, 0, None) == -1
    assert call(eps=None) == -1
    assert call(w=None) == -1
    assert call(out=None) == -1
    assert call(wtype=1) == -1  # FP16 weights need a scale
    assert call(scale=FAKE) == -1  # FP32 weights take no scale
    assert call(flags=4) == -1
    assert call(flags=6 << 8) == -1  # no such tile shape
    assert call(flags=1) == -2  # no exact mode
    assert call(flags=2) == -2
    d = good()
    d.ne = 0
    assert call(d=d) == -1
    d = good()
    d.norb = 17
    assert call(d=d) == -2


def test_batched_rejects_bad_arguments(L):
    assert L.tetra_dos_batched(None, 1, 0, 0, None, 0, None) == -1
    items = (tetra.TetraItem * 1)()
    assert L.tetra_dos_batched(items, 0, 0, 0, None, 0, None) == -1
    items[0].d = good()
    items[0].eps, items[0].w, items[0].dos = FAKE, FAKE, FAKE
    items[0].tile = 6  # no such tile shape
    assert L.tetra_dos_batched(items, 1, 0, 0, FAKE, 4096, None) == -1
    items[0].tile = 0
    assert L.tetra_dos_batched(items, 1, 0, 1, FAKE, 4096, None) == -2  # no exact mode in batches
    assert L.tetra_dos_batched(items, 1, 0, 2, FAKE, 4096, None) == -2
    assert L.tetra_dos_batched(items, 1, 0, 0, FAKE, 8, None) == -3  # workspace too small
    assert L.tetra_dos_batched_workspace(items, 1, 0, 0) == 256


def test_complex_amplitudes_flags(L):
    d = good()
    assert L.tetra_dos_forward(ctypes.byref(d), FAKE, FAKE, 2, FAKE, FAKE, 0, None) == -1  # no scale for C32
    assert L.tetra_dos_forward(ctypes.byref(d), FAKE, FAKE, 3, None, FAKE, 0, None) == -1  # no such type
    assert L.tetra_dos_backward(ctypes.byref(d), FAKE, FAKE, 2, FAKE, FAKE, FAKE, FAKE, 0, None) == -1
    assert L.tetra_nos_forward(ctypes.byref(d), FAKE, FAKE, 2, FAKE, FAKE, 0, None) == -1


def test_from_eigh_layouts():
    """The binding's layout helper (no GPU): eigenvalues [nk, nb] and eigenvectors [nk, norb, nb] to
    eps [nb, nk] and weights |a|^2 or amplitudes a, both [nb, norb, nk]."""
    import numpy as np
    import torch

    rng = np.random.default_rng(0)
    m = rng.standard_normal((6, 3, 3)) + 1j * rng.standard_normal((6, 3, 3))
    h = torch.from_numpy(m + np.conj(np.swapaxes(m, 1, 2)))
    ev, vec = torch.linalg.eigh(h)
    eps, w = tetra.from_eigh(ev, vec)
    eps2, a = tetra.from_eigh(ev, vec, amplitudes=True)
    assert eps.shape == (3, 6) and w.shape == (3, 3, 6) and a.shape == (3, 3, 6)
    assert a.dtype == torch.complex64 and w.dtype == torch.float32
    assert torch.equal(eps, eps2)
    assert torch.allclose(a.abs() ** 2, w, atol=1e-6)
    assert torch.allclose(a[1, 2, 4].to(torch.complex128), vec[4, 2, 1], atol=1e-6)


def test_probe_rejects_bad_arguments():
    from paper_1710_10789_amd import probe

    P = probe.lib()
    assert P.tetra_probe_lds_atomics(0, 10, FAKE, None) == -1
    assert P.tetra_probe_lds_atomics(4, 0, FAKE, None) == -1
    assert P.tetra_probe_lds_atomics(4, 10, None, None) == -1
    assert P.tetra_probe_lds_atomics((1 << 24) + 1, 10, FAKE, None) == -1
    assert P.tetra_probe_fma_f32(0, 10, FAKE, None) == -1
    assert P.tetra_probe_fma_f32(4, 0, FAKE, None) == -1
    assert P.tetra_probe_fma_f32(4, 10, None, None) == -1
    assert P.tetra_probe_fma_f32(4, (1 << 24) + 1, FAKE, None) == -1


def test_backward_workspace_sizes(L):
    """tetra_dos_backward_workspace: 4 (norb + 1) F nb T bytes where the two-phase output applies
    (grid sides multiples of the tile's, more than one tile per axis), else 0."""
    shapes = [(4, 4, 16), (8, 8, 4), (4, 8, 8), (8, 4, 8), (4, 16, 4), (16, 4, 4)]
    for sid, (a, b, c) in enumerate(shapes):
        faces = 2 * (b + 1) * (c + 1) + 2 * (a - 1) * (c + 1) + 2 * (a - 1) * (b - 1)
        assert faces == (a + 1) * (b + 1) * (c + 1) - (a - 1) * (b - 1) * (c - 1)
        d = tetra.make_desc((64, 64, 64), 8, 8, -1.0, 0.01, 1000)
        tiles = (64 // a) * (64 // b) * (64 // c)
        assert L.tetra_dos_backward_workspace(ctypes.byref(d), sid << 8) == 4 * 9 * faces * 8 * tiles
        assert tetra.backward_workspace_bytes((64, 64, 64), 8, 8, -1.0, 0.01, 1000, tile=sid) == 4 * 9 * faces * 8 * tiles
        for grid in ((a, 2 * b, 2 * c), (2 * a, 2 * b, c), (2 * a + 1, 2 * b, 2 * c), (2 * a, 2 * b, 3 * c - 1)):
            d = tetra.make_desc(grid, 2, 3, -1.0, 0.01, 100)
            assert L.tetra_dos_backward_workspace(ctypes.byref(d), sid << 8) == 0, (sid, grid)
    d = good()
    d.ne = 0
    assert L.tetra_dos_backward_workspace(ctypes.byref(d), 0) == 0
    assert L.tetra_dos_backward_workspace(ctypes.byref(good()), 0x10) == 0  # unknown flag
    assert L.tetra_dos_backward_workspace(ctypes.byref(good()), 6 << 8) == 0  # no such tile shape


def _bwd_ws(L, d, ws, ws_bytes, flags=0):
    return L.tetra_dos_backward_ws(ctypes.byref(d), FAKE, FAKE, 0, None, FAKE, FAKE, FAKE, flags, ws, ws_bytes, None)


def test_backward_ws_rejects_before_launch(L):
    d = tetra.make_desc((8, 8, 32), 2, 3, -1.0, 0.01, 100)
    need = L.tetra_dos_backward_workspace(ctypes.byref(d), 0)
    assert need > 0
    assert _bwd_ws(L, d, FAKE, need - 1) == -3  # too small
    assert _bwd_ws(L, d, FAKE + 4, need) == -1  # misaligned
    ragged = tetra.make_desc((6, 8, 32), 2, 3, -1.0, 0.01, 100)
    assert _bwd_ws(L, ragged, FAKE, 1 << 30) == -3  # the two-phase output does not apply
    assert _bwd_ws(L, ragged, None, 0, flags=2) == -2  # deterministic needs the two-phase output
    assert _bwd_ws(L, d, None, 0, flags=2) == -2
    bad = tetra.make_desc((8, 8, 32), 2, 3, -1.0, 0.0, 100)
    assert _bwd_ws(L, bad, FAKE, need) == -1
    assert L.tetra_dos_backward_ws(ctypes.byref(d), FAKE, FAKE, 0, None, FAKE, None, None, 0, FAKE, need, None) == -1
