"""Bethe-Salpeter exchange kernel Kx through the C-ABI against the oracle:
FP64 to 1e-12 and split BF16 to 1e-9 on a ragged small case (K = 138 pairs,
Ng = 181) with G = 0 first, elsewhere in the list, or absent; a BSE-like
case (48^3 grid, Ng = 1500, K = 4096 pairs) on sampled rows, Hermiticity of
the full result, split against FP64; the workspace query."""

import numpy as np
import pytest

import oracle
from paper_1111_4429_amd import bgw, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
SPLIT_TOL = 1e-9


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def handle(torch_dev):
    h = bgw.Handle(0)
    yield h
    h.close()


def dev(torch_dev, a):
    torch, d = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


@pytest.fixture(scope="module")
def small():
    s = synth.small_system(n=16, ngw=300, ng=181, nv=3, nc=23, nk=2, seed=31)
    q = s["qs"][0]
    M = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"])
    v = oracle.vcoul(s["bmat"], q["q"], q["ge"])
    pf = 1.0 / (s["nk"] * s["vol"])
    return M, v, pf


@pytest.mark.parametrize("precision", [bgw.FP64, bgw.SPLIT_BF16])
@pytest.mark.parametrize("head", [0, 5, -1])
def test_kx_small_vs_oracle(torch_dev, handle, small, precision, head):
    M, v, pf = small
    assert M.shape == (138, 181)
    vv = v.copy()
    if head == 5:
        vv[5], vv[0] = vv[0], vv[5]  # the large 1/q0^2 term now sits at index 5
    if head == -1:
        vv[0] = v[1]  # all G kept: a Coulomb factor without the q0 -> 0 divergence, as at a finite q
    ref = oracle.bse_kx(M, vv, head, pf)
    kx = handle.bse_kx(dev(torch_dev, M), dev(torch_dev, vv), head=head, prefactor=pf, precision=precision)
    got = kx.cpu().numpy()
    assert rel(got, ref) <= (TOL if precision == bgw.FP64 else SPLIT_TOL), (precision, head)
    assert np.array_equal(got, got.conj().T)


def test_kx_bse_like_sampled(torch_dev, handle):
    torch = torch_dev[0]
    wl = synth.Workload("bse-like", n=48, ng=1500, ngw=1500, nv=4, nc=16, nk=64)
    s = synth.make_system(wl)
    q = s["qs"][0]
    M = handle.pair_density(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    v = dev(torch_dev, oracle.vcoul(s["bmat"], q["q"], q["ge"]))
    pf = 1.0 / (s["nk"] * s["vol"])
    K = M.shape[0]
    assert K == 4096
    k64 = handle.bse_kx(M, v, head=0, prefactor=pf, precision=bgw.FP64)
    ksp = handle.bse_kx(M, v, head=0, prefactor=pf, precision=bgw.SPLIT_BF16)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([[0, 1, K - 1], rng.integers(0, K, 13)]))
    ref = oracle.bse_kx(M.cpu().numpy(), v.cpu().numpy(), 0, pf, rows=rows)
    ri = torch.from_numpy(rows).to(M.device)
    assert rel(k64[ri].cpu().numpy(), ref) <= TOL
    assert rel(ksp[ri].cpu().numpy(), ref) <= SPLIT_TOL
    assert float(torch.linalg.vector_norm(ksp - k64) / torch.linalg.vector_norm(k64)) <= SPLIT_TOL
    assert bool(torch.equal(k64, k64.conj().T))
    assert float(torch.diagonal(k64).real.min()) >= 0.0


def test_kx_workspace_query(torch_dev, handle, small):
    torch = torch_dev[0]
    M, v, pf = small
    for precision in (bgw.FP64, bgw.SPLIT_BF16):
        h = bgw.Handle(0)
        Md, vd = dev(torch_dev, M), dev(torch_dev, v)
        kx = torch.empty((M.shape[0], M.shape[0]), dtype=torch.complex128, device=Md.device)
        need = h.bse_kx_workspace(Md, vd, head=0, prefactor=pf, precision=precision, kx=kx)
        h.bse_kx(Md, vd, head=0, prefactor=pf, precision=precision, kx=kx)
        torch.cuda.synchronize()
        assert h.workspace_bytes() == need
        h.close()


def test_kx_rejects_bad_arguments(torch_dev, handle, small):
    M, v, pf = small
    Md, vd = dev(torch_dev, M), dev(torch_dev, v)
    with pytest.raises(bgw.BgwError):
        handle.bse_kx(Md, vd, head=181, prefactor=pf)
