"""Full-frequency (real-axis) chi^r/a(q; E) and its inverse dielectric matrix
through the C-ABI against the oracle: the complex weights of the
retarded/advanced dielectric equation on the paper's real-frequency grid,
both precisions, both functions, the head row in FP64, accumulation, graph
replay, and a silicon-like full-size check on sampled blocks."""

import numpy as np
import pytest

import oracle
from paper_1111_4429_amd import bgw, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
SPLIT_TOL = 1e-9
DELTA = 0.5  # eV


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
def small(torch_dev, handle):
    """ng = 181 (ragged tiles), K = 4 * 4 * 120 = 1920 pairs, E on the paper's grid.
    The split form's error grows like sqrt(ng / K) times the cancellation of
    the real part of the weight across the resonance E = |Delta|, so K is
    kept well above ng, as in the workloads."""
    s = synth.small_system(n=16, ngw=300, ng=181, nv=4, nc=120, nk=4, seed=44)
    q = s["qs"][0]
    M = handle.pair_density(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    torch_dev[0].cuda.synchronize()
    Mo = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"])
    E = bgw.ff_grid(2.0, 6.0, 40.0, 3.0)
    pf = 1.0 / (s["nk"] * s["vol"])
    ent = dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"], nc=s["nc"],
               head=0, prefactor=pf)
    ref = {k: oracle.chi(Mo, oracle.weights_real(q["ev"], s["ec"], E, DELTA, k), pf) for k in ("retarded", "advanced")}
    return dict(s=s, q=q, M=M, Mo=Mo, E=E, pf=pf, ent=ent, ref=ref)


def test_ff_grid_matches_oracle():
    for args in ((2.0, 6.0, 40.0, 3.0), (0.5, 2.0, 5.0, 0.5), (0.1, 1.3, 30.0, 0.05), (1.0, 10.0, 10.0, 0.0)):
        assert np.allclose(bgw.ff_grid(*args), oracle.ff_grid(*args), rtol=1e-15, atol=1e-14), args


def test_pair_density(small):
    assert rel(small["M"].cpu().numpy(), small["Mo"]) <= TOL


@pytest.mark.parametrize("precision", [bgw.FP64, bgw.SPLIT_BF16])
@pytest.mark.parametrize("kind", ["retarded", "advanced"])
def test_chi_real_axis(torch_dev, handle, small, precision, kind):
    (chi,) = handle.chi0([small["ent"]], small["E"], precision=precision, axis=kind, broadening=DELTA)
    got = chi.cpu().numpy()
    ref = small["ref"][kind]
    tol = TOL if precision == bgw.FP64 else SPLIT_TOL
    for i in range(len(small["E"])):
        assert rel(got[i], ref[i]) <= tol, (kind, i)
        # head row and column in FP64 in both precisions
        assert rel(got[i][0], ref[i][0]) <= TOL
        assert rel(got[i][:, 0], ref[i][:, 0]) <= TOL


@pytest.mark.parametrize("precision", [bgw.FP64, bgw.SPLIT_BF16])
def test_advanced_is_adjoint_of_retarded(torch_dev, handle, small, precision):
    kw = dict(precision=precision, broadening=DELTA)
    (cr,) = handle.chi0([small["ent"]], small["E"], axis="retarded", **kw)
    (ca,) = handle.chi0([small["ent"]], small["E"], axis="advanced", **kw)
    cr, ca = cr.cpu().numpy(), ca.cpu().numpy()
    for i in range(len(small["E"])):
        if precision == bgw.FP64:
            assert np.array_equal(ca[i], cr[i].conj().T)
        else:
            # the BF16 MFMA's FP32 accumulation is not sign-symmetric in its last
            # bit, so a few elements of the split form may differ by one rounding
            assert rel(ca[i], cr[i].conj().T) <= 1e-14
        anti = (cr[i] - cr[i].conj().T) / 2j
        lam = np.linalg.eigvalsh(0.5 * (anti + anti.conj().T))
        if small["E"][i] > 0:
            assert lam.max() <= 1e-13 * np.abs(lam).max()


def test_accumulate_and_graph(torch_dev, handle, small):
    """K-chunked accumulation (two calls on the two halves of the pairs) and
    graph replay give the one-call result."""
    torch = torch_dev[0]
    s, ent = small["s"], small["ent"]
    (one,) = handle.chi0([ent], small["E"], axis="retarded", broadening=DELTA)
    nk, nv, nc = s["nk"], s["nv"], s["nc"]
    per_k = nv * nc  # pairs are ordered (k, v, c): the first k-point's pairs come first
    ev, ec = ent["ev"].reshape(nk, nv), ent["ec"].reshape(nk, nc)
    a = dict(ent, M=ent["M"][:per_k].contiguous(), ev=ev[:1].contiguous(), ec=ec[:1].contiguous(), nk=1)
    b = dict(ent, M=ent["M"][per_k:].contiguous(), ev=ev[1:].contiguous(), ec=ec[1:].contiguous(), nk=nk - 1)
    acc = torch.zeros_like(one)
    handle.chi0([a], small["E"], axis="retarded", broadening=DELTA, chis=[acc], accumulate=True)
    handle.chi0([b], small["E"], axis="retarded", broadening=DELTA, chis=[acc], accumulate=True)
    torch.cuda.synchronize()
    assert rel(acc.cpu().numpy(), one.cpu().numpy()) <= 1e-13
    g = torch.empty_like(one)
    for rep in range(3):
        handle.chi0([ent], small["E"], axis="retarded", broadening=DELTA, chis=[g], use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy(), one.cpu().numpy()), rep
        g.zero_()


@pytest.mark.parametrize("precision", [bgw.FP64, bgw.SPLIT_BF16])
def test_eps_inv_real_axis(torch_dev, handle, small, precision):
    s, q = small["s"], small["q"]
    (chi,) = handle.chi0([small["ent"]], small["E"], precision=precision, axis="retarded", broadening=DELTA)
    v = bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"])
    einv, info = handle.eps_inv(dev(torch_dev, v), chi)
    assert np.all(info.cpu().numpy() == 0)
    ref, rinfo = oracle.eps_inv(v, chi.cpu().numpy())
    assert np.all(rinfo == 0)
    for i in range(len(small["E"])):
        assert rel(einv[i].cpu().numpy(), ref[i]) <= TOL


def test_silicon_like_real_axis_sampled(torch_dev, handle):
    """Silicon-like workload (Ng = 1500, K = 102400), four real frequencies
    around the absorption onset: both precisions against the oracle on
    sampled blocks of G, G' (the oracle from the GPU M, which other tests
    check), split against FP64 as a whole, and the inverse by its residual."""
    torch = torch_dev[0]
    s = synth.make_system(synth.WORKLOADS["silicon-like-48"])
    q = s["qs"][0]
    M = handle.pair_density(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    pf = 1.0 / (s["nk"] * s["vol"])
    ent = dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"], nc=s["nc"],
               head=0, prefactor=pf)
    E = np.array([0.0, 2.5, 9.0, 30.0])
    (c64,) = handle.chi0([ent], E, precision=bgw.FP64, axis="retarded", broadening=0.2)
    (csp,) = handle.chi0([ent], E, precision=bgw.SPLIT_BF16, axis="retarded", broadening=0.2)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([[0, 1, 1499], rng.integers(0, 1500, 20)]))
    cols = np.unique(np.concatenate([[0, 2, 1499], rng.integers(0, 1500, 20)]))
    allc = np.unique(np.concatenate([rows, cols]))
    sub = M[:, torch.from_numpy(allc).to(M.device)].cpu().numpy()
    pos = {int(c): i for i, c in enumerate(allc)}
    w = oracle.weights_real(q["ev"], s["ec"], E, 0.2, "retarded")
    ref = oracle.chi(sub, w, pf, rows=[pos[int(r)] for r in rows], cols=[pos[int(c)] for c in cols])
    ri, ci = torch.from_numpy(rows).to(M.device), torch.from_numpy(cols).to(M.device)
    for i in range(len(E)):
        assert rel(c64[i][ri][:, ci].cpu().numpy(), ref[i]) <= TOL
        assert rel(csp[i][ri][:, ci].cpu().numpy(), ref[i]) <= SPLIT_TOL
        assert float(torch.linalg.vector_norm(csp[i] - c64[i]) / torch.linalg.vector_norm(c64[i])) <= SPLIT_TOL
    v = dev(torch_dev, bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"]))
    einv, info = handle.eps_inv(v, c64)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    eye = torch.eye(1500, dtype=c64.dtype, device=c64.device)
    for i in range(len(E)):
        r = (eye - v[:, None] * c64[i]) @ einv[i] - eye
        assert float(torch.linalg.vector_norm(r)) / np.sqrt(1500) <= 1e-11
