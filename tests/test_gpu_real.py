"""Real flavor through the C-ABI against the oracle: real coefficients ->
real M (the complex definition's values, which are real) -> real symmetric
chi for several q and frequencies in one call (FP64, 1e-12), accumulation,
the workspace query, and a silicon-like real workload on sampled blocks with
the real rank-K update against the complex one on the same M."""

import numpy as np
import pytest

import oracle
from paper_1111_4429_amd import bgw, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


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
    s = synth.small_system(n=16, ngw=300, ng=181, nv=4, nc=37, nk=3, seed=17, flavor="real")
    q = s["qs"][0]
    Mo = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"])
    return s, q, Mo


def test_pair_density_real(torch_dev, handle, small):
    s, q, Mo = small
    M = handle.pair_density_real(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    assert M.dtype == torch_dev[0].float64
    assert rel(M.cpu().numpy(), Mo.real) <= TOL


def test_chi0_real_batch(torch_dev, handle, small):
    """Two q entries (the second with fewer G) and three frequencies in one call."""
    torch = torch_dev[0]
    s, q, Mo = small
    pf = 1.0 / (s["nk"] * s["vol"])
    om = np.array([0.0, 2.0, 30.0])
    Mr = np.ascontiguousarray(Mo.real)
    ents = [dict(M=dev(torch_dev, Mr), ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"],
                 nv=s["nv"], nc=s["nc"], head=0, prefactor=pf),
            dict(M=dev(torch_dev, Mr[:, :100]), ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"],
                 nv=s["nv"], nc=s["nc"], head=0, prefactor=pf)]
    chis = handle.chi0_real(ents, om)
    torch.cuda.synchronize()
    w = oracle.weights(q["ev"], s["ec"], om)
    for c, Mq in zip(chis, (Mr, Mr[:, :100])):
        ref = oracle.chi(Mq, w, pf)
        assert np.all(ref.imag == 0.0)
        got = c.cpu().numpy()
        for i in range(len(om)):
            assert rel(got[i], ref[i].real) <= TOL
            assert np.array_equal(got[i], got[i].T)


def test_chi0_real_accumulate_and_workspace(torch_dev, small):
    torch = torch_dev[0]
    s, q, Mo = small
    pf = 1.0 / (s["nk"] * s["vol"])
    Mr = np.ascontiguousarray(Mo.real)
    nk, nv, nc = s["nk"], s["nv"], s["nc"]
    per_k = nv * nc
    ev, ec = q["ev"].reshape(nk, nv), s["ec"].reshape(nk, nc)
    h = bgw.Handle(0)
    full = [dict(M=dev(torch_dev, Mr), ev=dev(torch_dev, ev), ec=dev(torch_dev, ec), nk=nk, nv=nv, nc=nc,
                 prefactor=pf)]
    need = h.chi0_real_workspace(full, [1.0])
    (one,) = h.chi0_real(full, [1.0])
    torch.cuda.synchronize()
    assert h.workspace_bytes() == need
    acc = torch.zeros_like(one)
    for a, b in ((0, 1), (1, nk)):
        part = [dict(M=dev(torch_dev, Mr[a * per_k:b * per_k]), ev=dev(torch_dev, ev[a:b]), ec=dev(torch_dev, ec[a:b]),
                     nk=b - a, nv=nv, nc=nc, prefactor=pf)]
        h.chi0_real(part, [1.0], accumulate=True, chis=[acc])
    torch.cuda.synchronize()
    assert rel(acc.cpu().numpy(), one.cpu().numpy()) <= 1e-13
    # the real flavor is FP64 on the imaginary axis: other requests are refused
    d, outs, keep = h._chi_desc(full, [1.0], bgw.SPLIT_BF16, False, None, False, real=True)
    with pytest.raises(bgw.BgwError):
        bgw._check(bgw.lib().bgw_chi0_real(h._h, bgw.ctypes.byref(d), bgw._stream()))
    d.precision, d.axis = bgw.FP64, 1
    with pytest.raises(bgw.BgwError):
        bgw._check(bgw.lib().bgw_chi0_real(h._h, bgw.ctypes.byref(d), bgw._stream()))
    del keep, outs
    h.close()


def test_silicon_like_real_sampled(torch_dev, handle):
    """The silicon-like workload in the real flavor: real M against the oracle
    on sampled pairs, real chi against the oracle on sampled blocks and against
    the complex FP64 chi of the same M (cast to complex)."""
    torch = torch_dev[0]
    s = synth.make_system(synth.WORKLOADS["silicon-like-48-real"])
    q = s["qs"][0]
    M = handle.pair_density_real(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    pairs = np.array([0, 1, 4095, 40000, 102399])
    Mo = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"], pairs=pairs)
    assert rel(M[torch.from_numpy(pairs).to(M.device)].cpu().numpy(), Mo.real) <= TOL
    pf = 1.0 / (s["nk"] * s["vol"])
    ent = dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"], nc=s["nc"],
               head=0, prefactor=pf)
    (cr,) = handle.chi0_real([ent], [0.0])
    (cc,) = handle.chi0([dict(ent, M=M.to(torch.complex128).contiguous())], [0.0])
    torch.cuda.synchronize()
    assert float(torch.linalg.vector_norm(cr - cc.real) / torch.linalg.vector_norm(cc.real)) <= TOL
    assert float(torch.abs(cc.imag).max()) <= 1e-14 * float(torch.abs(cc.real).max())
    rng = np.random.default_rng(2)
    rows = np.unique(np.concatenate([[0, 1499], rng.integers(0, 1500, 10)]))
    cols = np.unique(np.concatenate([[0, 777], rng.integers(0, 1500, 10)]))
    allc = np.unique(np.concatenate([rows, cols]))
    sub = M[:, torch.from_numpy(allc).to(M.device)].cpu().numpy()
    pos = {int(c): i for i, c in enumerate(allc)}
    w = oracle.weights(q["ev"], s["ec"], [0.0])
    ref = oracle.chi(sub, w, pf, rows=[pos[int(r)] for r in rows], cols=[pos[int(c)] for c in cols])[0]
    got = cr[0][torch.from_numpy(rows).to(M.device)][:, torch.from_numpy(cols).to(M.device)].cpu().numpy()
    assert rel(got, ref.real) <= TOL
