"""GPU tests of complex amplitude input (``TETRA_W_C32``): the kernels form the orbital weights
b = |a|^2 (eq. matrixelements) from the eigenvector components a^m_n(k), as the paper's kernel does,
and the adjoint returns the gradient with respect to their real and imaginary parts, 2 a dL/db.
Chained to ``torch.linalg.eigh``, that adjoint gives the derivative of a DOS loss with respect to the
parameters of a tight-binding Hamiltonian.

References: the FP64 oracle on b = |a|^2 (formed in FP64 from the FP32 parts, then rounded to FP32,
one rounding from what the kernels form); for gradients, 2 a times the oracle's analytic dL/db. For
the eigh chain, the oracle's analytic dL/deps and dL/db contracted with central differences (FP64
numpy eigh, a smooth function of the parameter) of the eigenpairs.

Gates: DOS, number of states and bin averages max |X - X_ref| / max |X_ref| <= 1e-5; gradients per
element as in the adjoint tests (1e-3 relative where |g_ref| >= 1e-3 max |g_ref|, else 1e-6 max);
the chained derivative within 1e-3 relative."""
import numpy as np
import pytest

import synth
from gates import gate

pytestmark = pytest.mark.gpu

GRID = (9, 7, 10)
NORB = 5
NE = 120


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def model():
    eps, a = synth.amplitudes(NORB, 3, GRID)
    b = (a.real.astype(np.float64) ** 2 + a.imag.astype(np.float64) ** 2).astype(np.float32)
    e0, de = synth.energy_grid(eps, NE)
    return eps, a, b, e0, de


def _err(got, ref):
    return np.abs(got.astype(np.float64) - ref).max() / np.abs(ref).max()


def test_forward_kernels_square_the_amplitudes(torch_dev, oracle_lib, model):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    eps, a, b, e0, de = model
    te, ta = torch.from_numpy(eps).to(dev), torch.from_numpy(a).to(dev)
    print(f"[case] amplitudes {GRID} norb={NORB} ne={NE}: DOS, number of states, bin averages", flush=True)
    d = tetra.dos_forward(te, ta, GRID, e0, de, NE)
    dk = tetra.dos_forward(te, ta, GRID, e0, de, NE, exact=True)
    n = tetra.nos_forward(te, ta, GRID, e0, de, NE)
    nb_ = tetra.dos_binned(te, ta, GRID, e0, de, NE)
    torch.cuda.synchronize()
    ref, _ = oracle_lib.dos(eps, b, GRID, e0, de, NE)
    assert _err(d.cpu().numpy(), ref) <= 1e-5
    assert _err(dk.cpu().numpy(), ref) <= 1e-5
    assert _err(n.cpu().numpy(), oracle_lib.nos(eps, b, GRID, e0, de, NE)) <= 1e-5
    assert _err(nb_.cpu().numpy(), oracle_lib.dos_binned(eps, b, GRID, e0, de, NE)) <= 1e-5


def test_batched_amplitudes(torch_dev, oracle_lib, model):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    eps, a, b, e0, de = model
    eps2, a2 = synth.amplitudes(NORB, 4, (5, 6, 7))
    b2 = (a2.real.astype(np.float64) ** 2 + a2.imag.astype(np.float64) ** 2).astype(np.float32)
    e02, de2 = synth.energy_grid(eps2, 70)
    probs = [(torch.from_numpy(eps).to(dev), torch.from_numpy(a).to(dev), GRID, e0, de, NE),
             (torch.from_numpy(eps2).to(dev), torch.from_numpy(a2).to(dev), (5, 6, 7), e02, de2, 70)]
    print("[case] batched amplitudes, 2 items", flush=True)
    outs = tetra.dos_batched(probs)
    torch.cuda.synchronize()
    assert _err(outs[0].cpu().numpy(), oracle_lib.dos(eps, b, GRID, e0, de, NE)[0]) <= 1e-5
    assert _err(outs[1].cpu().numpy(), oracle_lib.dos(eps2, b2, (5, 6, 7), e02, de2, 70)[0]) <= 1e-5


def test_adjoint_gradient_of_the_amplitudes(torch_dev, oracle_lib, model):
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    eps, a, b, e0, de = model
    G = np.random.default_rng(5).standard_normal((NE, NORB)).astype(np.float32)
    te, ta, tG = torch.from_numpy(eps).to(dev), torch.from_numpy(a).to(dev), torch.from_numpy(G).to(dev)
    print("[case] adjoint with amplitudes", flush=True)
    ge, ga = tetra.dos_backward(te, ta, GRID, e0, de, tG)
    torch.cuda.synchronize()
    assert ga.dtype == torch.complex64
    re, rb = oracle_lib.dos_backward(eps, b, GRID, e0, de, G.astype(np.float64))
    ra = 2.0 * a.astype(np.complex128) * rb
    oke, eb, _ = gate(ge.cpu().numpy(), re)
    ga = ga.cpu().numpy()
    okr, rr, _ = gate(ga.real, ra.real)
    oki, ri, _ = gate(ga.imag, ra.imag)
    print(f"[case] grad_eps {eb:.2e}; grad re(a) {rr:.2e}; grad im(a) {ri:.2e}", flush=True)
    assert oke and okr and oki


def test_eigh_chain_derivative(torch_dev, oracle_lib):
    """L(s) = sum (DOS(s) - target)^2 for H(k; s) = H_0(k) + s H_x(k), H_x the +-x hoppings: dL/ds by
    autograd through torch.linalg.eigh (FP64, on the host) and the adjoint kernel on complex
    amplitudes, against the oracle's analytic DOS gradient chained with eigenpair differences."""
    torch, dev = torch_dev
    import paper_1710_10789_amd as tetra

    grid, norb, ne = (6, 5, 7), 4, 80
    hops = synth.hoppings(norb, 21)
    hx = {r: (t if r in ((1, 0, 0), (-1, 0, 0)) else np.zeros_like(t)) for r, t in hops.items()}
    h0 = {r: (np.zeros_like(t) if r in ((1, 0, 0), (-1, 0, 0)) else t) for r, t in hops.items()}
    H0, Hx = synth.hamiltonians(h0, grid), synth.hamiltonians(hx, grid)
    eps1, w1 = synth.band_structure(norb, 21, grid, cache=False)
    teps, tw = synth.band_structure(norb, 22, grid, cache=False)
    e0, de = synth.energy_grid([eps1, teps], ne)
    target, _ = oracle_lib.dos(teps, tw, grid, e0, de, ne)

    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    H = torch.from_numpy(H0) + s * torch.from_numpy(Hx)
    evals, evecs = torch.linalg.eigh(H)
    eps_t, a_t = tetra.from_eigh(evals, evecs, amplitudes=True)
    print(f"[case] eigh chain {grid} norb={norb} ne={ne}", flush=True)
    dos = tetra.dos(eps_t.to(dev), a_t.to(dev), grid, e0, de, ne)
    loss = ((dos.double() - torch.from_numpy(target).to(dev)) ** 2).sum()
    loss.backward()
    got = float(s.grad)

    def pairs(sv):
        ev, vec = np.linalg.eigh(H0 + sv * Hx)
        return ev.T, (np.abs(vec) ** 2).transpose(2, 1, 0)

    e_c, b_c = pairs(1.0)
    e32, b32 = e_c.astype(np.float32), b_c.astype(np.float32)
    D, _ = oracle_lib.dos(e32, b32, grid, e0, de, ne)
    ge, gb = oracle_lib.dos_backward(e32, b32, grid, e0, de, 2.0 * (D - target))
    h = 1e-5
    ep, bp = pairs(1.0 + h)
    em, bm = pairs(1.0 - h)
    want = float((ge * (ep - em)).sum() + (gb * (bp - bm)).sum()) / (2 * h)
    print(f"[case] dL/ds autograd {got:.8e}, reference {want:.8e}", flush=True)
    assert abs(got - want) <= 1e-3 * abs(want)
