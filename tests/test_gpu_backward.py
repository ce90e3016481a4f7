"""GPU parity of the adjoint kernel (through the C ABI) against the FP64 oracle's analytic gradient and
against central finite differences of the FP64 oracle loss.

Gate (per element): |g_gpu - g_ref| <= 1e-3 |g_ref| where |g_ref| >= 1e-3 max|g_ref|, otherwise
|g_gpu - g_ref| <= 1e-6 max|g_ref|."""
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


def _gpu_grads(torch_dev, eps, w, grid, e0, de, G):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    ge, gw = tetra.dos_backward(torch.from_numpy(eps).to(dev), torch.from_numpy(w).to(dev), grid, e0, de,
                                torch.from_numpy(np.ascontiguousarray(G, np.float32)).to(dev))
    torch.cuda.synchronize()
    return ge.cpu().numpy(), gw.cpu().numpy()


def _check(torch_dev, oracle_lib, eps, w, grid, e0, de, G):
    print(f"[case] grid={grid} nb={eps.shape[0]} norb={w.shape[1]} ne={G.shape[0]}", flush=True)
    G32 = np.asarray(G, np.float32).astype(np.float64)  # both sides see the same FP32 G
    re, rw = oracle_lib.dos_backward(eps, w, grid, e0, de, G32)
    ge, gw = _gpu_grads(torch_dev, eps, w, grid, e0, de, G32)
    okw, wb, wn = gate(gw, rw)
    oke, eb, en = gate(ge, re)
    print(f"[case] grad_w worst-rel {wb:.2e} norm {wn:.2e}; grad_eps worst-rel {eb:.2e} norm {en:.2e}", flush=True)
    assert okw and oke
    return ge, gw, re, rw


@pytest.mark.parametrize("norb", [1, 3, 8, 16])
@pytest.mark.parametrize("grid", [(2, 2, 2), (2, 1, 3), (5, 7, 3), (9, 6, 21)])
def test_gradient_parity_small_and_ragged(torch_dev, oracle_lib, grid, norb):
    eps, w = synth.band_structure(norb, 11 + norb, grid)
    e0, de = synth.energy_grid(eps, 90)
    G = np.random.default_rng(norb).normal(size=(90, norb))
    _check(torch_dev, oracle_lib, eps, w, grid, e0, de, G)


def test_gradient_parity_energy_chunking(torch_dev, oracle_lib):
    grid = (6, 5, 20)
    eps, w = synth.band_structure(16, 3, grid)
    e0, de = synth.energy_grid(eps, 3000)
    G = np.random.default_rng(5).normal(size=(3000, 16))
    _check(torch_dev, oracle_lib, eps, w, grid, e0, de, G)


def test_gradient_with_non_finite_energies(torch_dev, oracle_lib):
    grid = (5, 4, 6)
    eps, w = synth.band_structure(4, 9, grid)
    eps = eps.copy()
    eps[0, 3] = np.nan
    eps[2, 17] = np.inf
    e0, de = synth.energy_grid(np.nan_to_num(eps, nan=0.0, posinf=0.0), 80)
    G = np.random.default_rng(2).normal(size=(80, 4))
    ge, gw, re, rw = _check(torch_dev, oracle_lib, eps, w, grid, e0, de, G)
    assert np.all(np.isfinite(ge)) and np.all(np.isfinite(gw))


def _incident(grid, k):
    """(cube origin, tetrahedron corner slots) of the 24 tetrahedra having k-point k as a corner."""
    tab = [(0, 1, 2, 5), (1, 2, 3, 5), (0, 2, 4, 5), (2, 3, 5, 7), (2, 4, 5, 6), (2, 5, 6, 7)]  # Table I - 1
    n1, n2, n3 = grid
    i1, i2, i3 = k // (n2 * n3), (k // n3) % n2, k % n3
    out = []
    for s in range(8):
        o = (s & 1, (s >> 1) & 1, s >> 2)
        cube = ((i1 - o[0]) % n1, (i2 - o[1]) % n2, (i3 - o[2]) % n3)
        for t in tab:
            if s in t:
                out.append((cube, t))
    return out


def _tet_kpoints(grid, cube, slots):
    n1, n2, n3 = grid
    return [(((cube[0] + (s & 1)) % n1) * n2 + (cube[1] + ((s >> 1) & 1)) % n2) * n3 + (cube[2] + (s >> 2)) % n3
            for s in slots]


def _local_delta(oracle_lib, eps, w, grid, n, k, e0, de, ne, new_eps=None, new_w=None):
    """Change of DOS[j][m] when eps[n,k] (or w[n,:,k]) changes: only the 24 incident tetrahedra move."""
    nk = eps.shape[1]
    vol = 1.0 / (6 * nk)
    norb = w.shape[1]
    delta = np.zeros((ne, norb))
    Ej = e0 + de * np.arange(ne)
    for cube, slots in _incident(grid, k):
        ks = _tet_kpoints(grid, cube, slots)
        e_old = eps[n, ks].astype(np.float64)
        e_new = e_old.copy()
        b_old = w[n][:, ks].astype(np.float64)
        b_new = b_old.copy()
        for pos, kk in enumerate(ks):
            if kk == k:
                if new_eps is not None:
                    e_new[pos] = new_eps
                if new_w is not None:
                    b_new[:, pos] = new_w
        lo = min(e_old.min(), e_new.min())
        hi = max(e_old.max(), e_new.max())
        for j in np.nonzero((Ej > lo) & (Ej < hi))[0]:
            for m in range(norb):
                delta[j, m] += (oracle_lib.tet_dos(e_new, b_new[m], Ej[j], vol)
                                - oracle_lib.tet_dos(e_old, b_old[m], Ej[j], vol))
    return delta


def test_fit_workload_64cube_500E(torch_dev, oracle_lib):
    """loss = sum (DOS - DOS_target)^2 on the differentiation workload (64^3, 8 bands x 8 orbitals,
    500 energies; target = model seed 1): all gradient elements against the oracle's analytic
    gradient, and 100 + 100 random entries against central differences of the FP64 loss."""
    torch, dev = torch_dev
    c = synth.config("k64_b8_e500_fit")
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    eps, w = synth.band_structure(norb, c["seed"], grid)
    teps, tw = synth.band_structure(norb, c["target_seed"], grid)
    e0, de = synth.energy_grid([eps, teps], ne)
    D, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    T, _ = oracle_lib.dos(teps, tw, grid, e0, de, ne)
    R = D - T
    G = 2.0 * R
    ge, gw, re, rw = _check(torch_dev, oracle_lib, eps, w, grid, e0, de, G)

    rng = np.random.default_rng(7)
    h = 1e-4
    Ej = e0 + de * np.arange(ne)
    nk = eps.shape[1]
    fd_e, an_e, fd_w, an_w = [], [], [], []
    while len(fd_e) < 100:
        n, k = int(rng.integers(8)), int(rng.integers(nk))
        x = float(eps[n, k])
        partners = {q for cube, slots in _incident(grid, k) for q in _tet_kpoints(grid, cube, slots)} - {k}
        pe = np.array([float(eps[n, q]) for q in partners])
        if np.min(np.abs(Ej - x)) < 10 * h or np.min(np.abs(pe - x)) < 10 * h:
            continue  # kink within reach of the perturbation
        dp = _local_delta(oracle_lib, eps, w, grid, n, k, e0, de, ne, new_eps=x + h)
        dm = _local_delta(oracle_lib, eps, w, grid, n, k, e0, de, ne, new_eps=x - h)
        Lp = (dp * (2 * R + dp)).sum()
        Lm = (dm * (2 * R + dm)).sum()
        fd_e.append((Lp - Lm) / (2 * h))
        an_e.append(ge[n, k])
    while len(fd_w) < 100:
        n, m, k = int(rng.integers(8)), int(rng.integers(norb)), int(rng.integers(nk))
        b = w[n, :, k].astype(np.float64)
        bp, bm = b.copy(), b.copy()
        bp[m] += h
        bm[m] -= h
        dp = _local_delta(oracle_lib, eps, w, grid, n, k, e0, de, ne, new_w=bp)
        dm = _local_delta(oracle_lib, eps, w, grid, n, k, e0, de, ne, new_w=bm)
        fd_w.append(((dp * (2 * R + dp)).sum() - (dm * (2 * R + dm)).sum()) / (2 * h))
        an_w.append(gw[n, m, k])
    fd_e, an_e, fd_w, an_w = map(np.array, (fd_e, an_e, fd_w, an_w))
    scale_e = np.abs(re).max()
    scale_w = np.abs(rw).max()
    for fd, an, scale in ((fd_e, an_e, scale_e), (fd_w, an_w, scale_w)):
        big = np.abs(fd) >= 1e-3 * scale
        err = np.abs(an - fd)
        print(f"[fd] worst rel {float((err[big] / np.abs(fd[big])).max()) if big.any() else 0:.2e}, "
              f"{int(big.sum())} large entries", flush=True)
        assert np.all(np.where(big, err <= 1e-3 * np.abs(fd), err <= 1e-6 * scale + 1e-3 * np.abs(fd)))


def test_autograd_function_matches_backward(torch_dev):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (6, 6, 8)
    eps_np, w_np = synth.band_structure(4, 21, grid)
    e0, de = synth.energy_grid(eps_np, 70)
    eps = torch.from_numpy(eps_np).to(dev).requires_grad_(True)
    w = torch.from_numpy(w_np).to(dev).requires_grad_(True)
    target = torch.rand(70, 4, device=dev)
    d = tetra.dos(eps, w, grid, e0, de, 70)
    loss = ((d - target) ** 2).sum()
    loss.backward()
    G = (2 * (d.detach() - target)).contiguous()
    ge, gw = tetra.dos_backward(eps.detach(), w.detach(), grid, e0, de, G)
    torch.cuda.synchronize()
    assert torch.allclose(eps.grad, ge, rtol=1e-5, atol=1e-6 * float(ge.abs().max()))
    assert torch.allclose(w.grad, gw, rtol=1e-5, atol=1e-6 * float(gw.abs().max()))


def test_gradient_with_fp16_weights(torch_dev, oracle_lib):
    """The adjoint of the FP16-weight forward: gradients with respect to the dequantised weights."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid = (9, 6, 21)
    eps, w = synth.band_structure(16, 6, grid)
    e0, de = synth.energy_grid(eps, 120)
    w16, scale = (t.cpu() for t in tetra.half_weights(torch.from_numpy(w).cuda()))
    deq = (w16.float() * scale[:, None, None]).numpy()
    G = np.random.default_rng(4).normal(size=(120, 16)).astype(np.float32).astype(np.float64)
    re, rw = oracle_lib.dos_backward(eps, deq, grid, e0, de, G)
    ge, gw = tetra.dos_backward(torch.from_numpy(eps).to(dev), w16.to(dev), grid, e0, de,
                                torch.from_numpy(G.astype(np.float32)).to(dev), w_scale=scale.to(dev))
    torch.cuda.synchronize()
    okw, _, _ = gate(gw.cpu().numpy(), rw)
    oke, _, _ = gate(ge.cpu().numpy(), re)
    assert okw and oke
