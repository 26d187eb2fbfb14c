"""The largest supported dielectric sphere, Ng = 12288: the chi-sum in both
precisions against the oracle on sampled blocks (head row/column included),
and the inversion, whose cooperative panels then take 48 workgroups per
matrix, checked by its residual eps eps^-1 - 1 (the oracle's own elimination
at this size would take the better part of an hour)."""

import numpy as np
import pytest

import oracle
from paper_1111_4429_amd import bgw

pytestmark = pytest.mark.gpu

NG = 12288


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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_chi_and_eps_inv_at_largest_ng(torch_dev, handle):
    torch, d = torch_dev
    print(f"[large-ng] Ng = {NG}", flush=True)
    rng = np.random.default_rng(5)
    nk, nv, nc = 1, 4, 128
    K = nk * nv * nc
    env = np.exp(-np.arange(NG) / 4000.0) / np.sqrt(NG)
    M = (rng.standard_normal((K, NG)) + 1j * rng.standard_normal((K, NG))) * env
    ev = np.sort(rng.uniform(-10.0, 0.0, (nk, nv)), axis=1)
    ec = np.sort(rng.uniform(1.0, 20.0, (nk, nc)), axis=1)
    pf = 0.01
    Md = torch.from_numpy(M).to(d)
    ent = dict(M=Md, ev=torch.from_numpy(ev).to(d), ec=torch.from_numpy(ec).to(d), nk=nk, nv=nv, nc=nc, head=0,
               prefactor=pf)
    (chi,) = handle.chi0([ent], [0.0])
    (chis,) = handle.chi0([ent], [0.0], precision=bgw.SPLIT_BF16)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, 1, 4095, 8191, NG - 1], rng.integers(0, NG, 12)]))
    cols = np.unique(np.concatenate([[0, 2, 6000, NG - 2], rng.integers(0, NG, 12)]))
    allc = np.unique(np.concatenate([rows, cols]))
    pos = {int(c): i for i, c in enumerate(allc)}
    w = oracle.weights(ev, ec, [0.0])
    ref = oracle.chi(np.ascontiguousarray(M[:, allc]), w, pf, rows=[pos[int(r)] for r in rows],
                     cols=[pos[int(c)] for c in cols])[0]
    ri, ci = torch.from_numpy(rows).to(d), torch.from_numpy(cols).to(d)
    assert rel(chi[0][ri][:, ci].cpu().numpy(), ref) <= 1e-12
    assert rel(chis[0][ri][:, ci].cpu().numpy(), ref) <= 1e-9
    del chis
    # eps = 1 - v chi is close to the identity here (well conditioned)
    g = np.arange(NG, dtype=np.float64)
    v = torch.from_numpy(4.0 * np.pi / (1.0 + g ** (2.0 / 3.0))).to(d)
    einv = torch.empty_like(chi)
    info = torch.empty(1, dtype=torch.int32, device=d)
    handle.eps_inv(v, chi, epsinv=einv, info=info)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    eye = torch.eye(NG, dtype=torch.complex128, device=d)
    eps = eye - v[:, None] * chi[0]
    res = eps @ einv[0] - eye
    assert float(res.abs().max()) <= 1e-12
