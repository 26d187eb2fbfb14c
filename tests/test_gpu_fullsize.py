"""Full-size runs of the supercell, imaginary-frequency and uneven-q workloads
through the C-ABI, checked stage by stage on samples the oracle can compute:

  (i)   M for sampled pairs (every q) from the coefficients;
  (ii)  chi on sampled (G, G') blocks, including the head row/column and the
        last index, computed by the oracle from the GPU-produced M (already
        checked by (i)), for FP64 (<= 1e-12) and split (<= 1e-9) precision;
        the whole split chi against the whole FP64 chi (<= 1e-9);
  (iii) eps^-1 by its residual in the symmetrised form
        V^-1/2 (eps eps^-1 - I) V^1/2 (eps = 1 - V chi, V = diag v), which is
        well conditioned at any size because V^1/2 chi V^1/2 is Hermitian and
        negative semi-definite.
"""

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


def check_M_samples(torch_dev, s, q, M, npairs=24, seed=0):
    K = s["nk"] * s["nv"] * s["nc"]
    rng = np.random.default_rng(seed)
    pairs = np.unique(np.concatenate([[0, K - 1], rng.integers(0, K, npairs - 2)]))
    ref = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"], pairs=pairs)
    got = M[torch_dev[0].from_numpy(pairs).to(M.device)].cpu().numpy()
    assert rel(got, ref) <= TOL


def sample_index(ng, n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, 1, ng - 1], rng.integers(0, ng, n)])).astype(np.int64)


def oracle_block(torch_dev, M, w, pf, rows, cols):
    """chi[rows][cols] by the oracle from the GPU M, gathering only the needed columns."""
    torch = torch_dev[0]
    cols_all = np.unique(np.concatenate([rows, cols]))
    sub = M[:, torch.from_numpy(cols_all).to(M.device)].cpu().numpy()
    pos = {int(c): i for i, c in enumerate(cols_all)}
    r = np.array([pos[int(x)] for x in rows], dtype=np.int32)
    c = np.array([pos[int(x)] for x in cols], dtype=np.int32)
    return oracle.chi(sub, w, pf, rows=r, cols=c)


def check_eps_inv(torch_dev, v, chi, einv):
    """Residual of the symmetrised inverse, per matrix."""
    torch = torch_dev[0]
    ng = chi.shape[-1]
    vs = torch.sqrt(v)
    eye = torch.eye(ng, dtype=chi.dtype, device=chi.device)
    for w in range(chi.shape[0]):
        eps = eye - v[:, None] * chi[w]
        r = eps @ einv[w] - eye
        rs = r * (vs[None, :] / vs[:, None])
        res = float(torch.linalg.vector_norm(rs)) / np.sqrt(ng)
        assert res <= 1e-12, f"symmetrised residual {res:.3e} (frequency {w})"


def test_supercell_96_full(torch_dev, handle):
    """96^3 grid, Ng = 8000, K = 256000: M samples, chi blocks (FP64 and split),
    split vs FP64 over the whole matrix, eps^-1 residual."""
    torch = torch_dev[0]
    s = synth.make_system(synth.WORKLOADS["supercell-96"])
    q = s["qs"][0]
    ng = q["ng"]
    M = handle.pair_density(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    torch.cuda.synchronize()
    check_M_samples(torch_dev, s, q, M, npairs=16)
    pf = 1.0 / (s["nk"] * s["vol"])
    ent = [dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"], nc=s["nc"],
                head=0, prefactor=pf)]
    (c64,) = handle.chi0(ent, [0.0], precision=bgw.FP64)
    (csp,) = handle.chi0(ent, [0.0], precision=bgw.SPLIT_BF16)
    torch.cuda.synchronize()
    assert float(torch.linalg.vector_norm(csp - c64) / torch.linalg.vector_norm(c64)) <= SPLIT_TOL
    rows, cols = sample_index(ng, 29, 1), sample_index(ng, 29, 2)
    w = oracle.weights(q["ev"], s["ec"], [0.0])
    ref = oracle_block(torch_dev, M, w, pf, rows, cols)[0]
    ri, ci = torch.from_numpy(rows).to(M.device), torch.from_numpy(cols).to(M.device)
    assert rel(c64[0][ri][:, ci].cpu().numpy(), ref) <= TOL
    assert rel(csp[0][ri][:, ci].cpu().numpy(), ref) <= SPLIT_TOL
    assert rel(csp[0][0].cpu().numpy(), c64[0][0].cpu().numpy()) <= 1e-13  # FP64 head row in split mode
    del M
    v = dev(torch_dev, bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"]))
    einv, info = handle.eps_inv(v, csp)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    check_eps_inv(torch_dev, v, csp, einv)


def test_imag_freq_64_full(torch_dev, handle):
    """64^3 grid, Ng = 4000, K = 512000: all 32 Gauss-Legendre frequencies in
    one split-precision call (the workload's precision) against the oracle
    on sampled blocks of every frequency; FP64 at the first, 16th and last
    frequency in one batched call, against the oracle and the split result."""
    torch = torch_dev[0]
    s = synth.make_system(synth.WORKLOADS["imag-freq-64"])
    q = s["qs"][0]
    ng = q["ng"]
    om_all = s["omega"]
    assert len(om_all) == 32
    pick = [0, 15, 31]
    M = handle.pair_density(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    torch.cuda.synchronize()
    check_M_samples(torch_dev, s, q, M, npairs=16, seed=3)
    pf = 1.0 / (s["nk"] * s["vol"])
    ent = [dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"], nc=s["nc"],
                head=0, prefactor=pf)]
    (csp,) = handle.chi0(ent, om_all, precision=bgw.SPLIT_BF16)
    (c64,) = handle.chi0(ent, om_all[pick], precision=bgw.FP64)
    torch.cuda.synchronize()
    rows, cols = sample_index(ng, 21, 4), sample_index(ng, 21, 5)
    w = oracle.weights(q["ev"], s["ec"], om_all)
    ref = oracle_block(torch_dev, M, w, pf, rows, cols)
    ri, ci = torch.from_numpy(rows).to(M.device), torch.from_numpy(cols).to(M.device)
    for i in range(len(om_all)):
        assert rel(csp[i][ri][:, ci].cpu().numpy(), ref[i]) <= SPLIT_TOL, i
        assert rel(csp[i][0].cpu().numpy(), csp[i][:, 0].conj().cpu().numpy()) == 0.0
    for j, i in enumerate(pick):
        assert rel(c64[j][ri][:, ci].cpu().numpy(), ref[i]) <= TOL
        assert float(torch.linalg.vector_norm(csp[i] - c64[j]) / torch.linalg.vector_norm(c64[j])) <= SPLIT_TOL
        assert rel(csp[i][0].cpu().numpy(), c64[j][0].cpu().numpy()) <= 1e-13  # FP64 head row in split mode
    # |chi_GG(i omega)| decreases with omega
    d = torch.diagonal(csp, dim1=1, dim2=2).abs()
    assert bool((d[1:] <= d[:-1]).all())
    del M, c64
    v = dev(torch_dev, bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"]))
    einv, info = handle.eps_inv(v, csp)
    torch.cuda.synchronize()
    assert int(info.cpu().max()) == 0 and int(info.cpu().min()) == 0
    check_eps_inv(torch_dev, v, csp, einv)


def test_uneven_q_48_full(torch_dev, handle):
    """48^3 grid, Ngw = 6000, K = 518400 per q: the q with the smallest,
    median and largest Ng of the 64 (q0 included when it is one of them),
    chi for all three in one batched call, both precisions."""
    torch = torch_dev[0]
    wl = synth.WORKLOADS["uneven-q-48"]
    sizes = synth.uneven_q_sizes(wl)
    order = np.argsort(sizes, kind="stable")
    pick = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    s = synth.make_system(wl, q_subset=pick)
    assert [q["ng"] for q in s["qs"]] == [int(sizes[i]) for i in pick]
    pf = 1.0 / (s["nk"] * s["vol"])
    ents, Ms = [], []
    for j, q in enumerate(s["qs"]):
        M = handle.pair_density(s["n"], s["gw"], q["ge"], dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
        torch.cuda.synchronize()
        check_M_samples(torch_dev, s, q, M, npairs=12, seed=10 + j)
        Ms.append(M)
        ents.append(dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"],
                         nc=s["nc"], head=0, prefactor=pf))
    c64s = handle.chi0(ents, [0.0], precision=bgw.FP64)
    csps = handle.chi0(ents, [0.0], precision=bgw.SPLIT_BF16)
    torch.cuda.synchronize()
    for j, q in enumerate(s["qs"]):
        ng = q["ng"]
        c64, csp = c64s[j], csps[j]
        assert float(torch.linalg.vector_norm(csp - c64) / torch.linalg.vector_norm(c64)) <= SPLIT_TOL
        rows, cols = sample_index(ng, 17, 20 + j), sample_index(ng, 17, 30 + j)
        w = oracle.weights(q["ev"], s["ec"], [0.0])
        ref = oracle_block(torch_dev, Ms[j], w, pf, rows, cols)[0]
        ri, ci = torch.from_numpy(rows).to(c64.device), torch.from_numpy(cols).to(c64.device)
        assert rel(c64[0][ri][:, ci].cpu().numpy(), ref) <= TOL
        assert rel(csp[0][ri][:, ci].cpu().numpy(), ref) <= SPLIT_TOL
    del Ms, ents
    for j, q in enumerate(s["qs"]):
        v = dev(torch_dev, bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"]))
        einv, info = handle.eps_inv(v, c64s[j])
        torch.cuda.synchronize()
        assert int(info.cpu()[0]) == 0
        check_eps_inv(torch_dev, v, c64s[j], einv)
