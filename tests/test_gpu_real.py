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


# --- real coefficients from complex ones -----------------------------------

def _unitary(rng, d):
    q, r = np.linalg.qr(rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _groups(e, tol):
    """(b0, d) of every degenerate group of one k: neighbours within tol."""
    out, b0 = [], 0
    while b0 < len(e):
        b1 = b0 + 1
        while b1 < len(e) and e[b1] - e[b1 - 1] <= tol:
            b1 += 1
        out.append((b0, b1 - b0))
        b0 = b1
    return out


def _complexify(R, e, tol, seed):
    """Complex states a plane-wave code could return for the real states R
    [nk][nb][ngw]: a random phase on each state, a random unitary within each
    degenerate group."""
    rng = np.random.default_rng(seed)
    C = R * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, R.shape[:2]))[..., None]
    for k in range(R.shape[0]):
        for b0, d in _groups(e[k], tol):
            if d > 1:
                C[k, b0:b0 + d] = _unitary(rng, d) @ R[k, b0:b0 + d]
    return C


def _same_group_bases(torch_dev, a, b, e, tol, atol):
    """a and b (device f64 [nk][nb][ngw]) are orthonormal per k and span the
    same subspace for every degenerate group: S = a b^T is orthogonal and zero
    outside the group blocks."""
    torch = torch_dev[0]
    S = torch.bmm(a, b.transpose(1, 2).contiguous())
    nk, nb = S.shape[:2]
    mask = np.zeros((nk, nb, nb), dtype=bool)
    for k in range(nk):
        for b0, d in _groups(e[k], tol):
            mask[k, b0:b0 + d, b0:b0 + d] = True
    off = S.masked_fill(torch.from_numpy(mask).to(S.device), 0.0)
    eye = torch.eye(nb, dtype=S.dtype, device=S.device).expand(nk, nb, nb)
    assert float(off.abs().max()) <= atol
    assert float((torch.bmm(S, S.transpose(1, 2).contiguous()) - eye).abs().max()) <= atol
    assert float((torch.bmm(a, a.transpose(1, 2).contiguous()) - eye).abs().max()) <= atol


def test_realify_matches_oracle(torch_dev, handle):
    """Groups of 1 .. 32 states (the largest supported) at ngw = 300, not a
    multiple of the block size: the same real groups as the oracle's, phases
    of single states removed up to sign."""
    torch = torch_dev[0]
    s = synth.small_system(n=16, ngw=300, ng=181, nv=2, nc=40, nk=3, seed=23, flavor="real")
    R = s["cc"]
    e = s["ec"].reshape(3, 40).copy()
    for k, b0, d in ((0, 1, 2), (0, 4, 3), (0, 10, 5), (0, 39, 1), (1, 4, 32), (2, 38, 2)):
        e[k, b0:b0 + d] = e[k, b0]
    tol = 1e-9
    C = _complexify(R, e, tol, 5)
    ro, bad = oracle.realify(C, e, tol)
    assert bad == 0
    r, nbad = handle.realify(dev(torch_dev, C), e, tol)
    torch.cuda.synchronize()
    assert nbad == 0
    _same_group_bases(torch_dev, r, dev(torch_dev, ro), e, tol, 1e-12)
    _same_group_bases(torch_dev, r, dev(torch_dev, R), e, tol, 1e-12)
    # single states: the oracle's vector up to sign
    got, single = r.cpu().numpy(), [(k, b0) for k in range(3) for b0, d in _groups(e[k], tol) if d == 1]
    for k, b in single:
        sgn = np.sign(got[k, b] @ ro[k, b])
        assert np.abs(got[k, b] - sgn * ro[k, b]).max() <= 1e-13


def test_realify_counts_groups_that_are_not_real(torch_dev, handle):
    """Generic complex orthonormal states: a single state, and a group of d,
    span more real dimensions than they have states; real states mixed by a
    unitary do not.  The count equals the oracle's."""
    torch = torch_dev[0]
    rng = np.random.default_rng(8)
    ngw = 517
    Z = np.linalg.qr(rng.standard_normal((ngw, 12)) + 1j * rng.standard_normal((ngw, 12)))[0].T
    R = np.linalg.qr(rng.standard_normal((ngw, 12)))[0].T
    C = np.stack([Z, R * 1j, Z])
    C[2, 6:] = _unitary(rng, 6) @ R[6:]
    e = np.array([[0, 1, 2, 2, 3, 3, 3, 4, 5, 6, 7, 8],
                  [0] * 12,
                  [0, 0, 0, 1, 2, 3, 4, 4, 4, 4, 4, 4]], dtype=np.float64)
    ro, bad = oracle.realify(C, e, 1e-9)
    assert bad == 9 + 0 + 4
    r, nbad = handle.realify(dev(torch_dev, C), e, 1e-9)
    torch.cuda.synchronize()
    assert nbad == bad
    # the real groups still come out right
    got = r.cpu().numpy()
    P = got[1].T @ got[1]
    assert np.abs(P - R.T @ R).max() <= 1e-12
    assert np.abs(got[2, 6:].T @ got[2, 6:] - R[6:].T @ R[6:]).max() <= 1e-12


def test_realify_then_real_chi_equals_complex_chi(torch_dev, handle):
    """Complex degenerate states -> real states on the GPU -> real M -> real
    chi, against the oracle's chi of the complex states (FP64, 1e-12): each
    group is rotated within itself and the weights depend only on energies."""
    torch = torch_dev[0]
    s = synth.small_system(n=16, ngw=300, ng=181, nv=4, nc=24, nk=2, seed=31, flavor="real")
    q = s["qs"][0]
    nk, nv, nc = 2, 4, 24
    ev = q["ev"].reshape(nk, nv).copy()
    ec = s["ec"].reshape(nk, nc).copy()
    ev[0, 1:3] = ev[0, 1]
    ev[1, 0:4] = ev[1, 0]
    ec[0, 3:6] = ec[0, 3]
    ec[1, 0:2] = ec[1, 0]
    ec[1, 10:17] = ec[1, 10]
    tol = 1e-9
    Cv = _complexify(q["cv"], ev, tol, 11)
    Cc = _complexify(s["cc"], ec, tol, 12)
    om = [0.0, 3.0]
    pf = 1.0 / (nk * s["vol"])
    ref = oracle.chi(oracle.pair_density(s["gw"], q["ge"], Cv, Cc), oracle.weights(ev, ec, om), pf)
    assert np.abs(ref.imag).max() <= 1e-14 * np.abs(ref.real).max()
    rv, bv = handle.realify(dev(torch_dev, Cv), ev, tol)
    rc, bc = handle.realify(dev(torch_dev, Cc), ec, tol)
    M = handle.pair_density_real(s["n"], s["gw"], q["ge"], rv, rc)
    ent = dict(M=M, ev=dev(torch_dev, ev), ec=dev(torch_dev, ec), nk=nk, nv=nv, nc=nc, head=0, prefactor=pf)
    (got,) = handle.chi0_real([ent], om)
    torch.cuda.synchronize()
    assert bv == 0 and bc == 0
    got = got.cpu().numpy()
    for i in range(len(om)):
        assert rel(got[i], ref[i].real) <= TOL


def test_realify_silicon_like_conduction_states(torch_dev, handle):
    """The silicon-like real workload's 64 x 400 conduction states at 1500
    plane waves, complexified with degenerate groups of 2 .. 6 every few
    bands: GPU against the oracle and against the real states."""
    torch = torch_dev[0]
    s = synth.make_system(synth.WORKLOADS["silicon-like-48-real"])
    R = s["cc"]
    nk, nc = R.shape[:2]
    e = s["ec"].reshape(nk, nc).copy()
    rng = np.random.default_rng(3)
    for k in range(nk):
        b = int(rng.integers(0, 4))
        while b < nc:
            d = int(rng.integers(1, 7))
            e[k, b:b + d] = e[k, b]
            b += d + int(rng.integers(1, 6))
    tol = 1e-9
    C = _complexify(R, e, tol, 4)
    ro, bad = oracle.realify(C, e, tol)
    assert bad == 0
    r, nbad = handle.realify(dev(torch_dev, C), e, tol)
    torch.cuda.synchronize()
    assert nbad == 0
    _same_group_bases(torch_dev, r, dev(torch_dev, ro), e, tol, 1e-12)
    _same_group_bases(torch_dev, r, dev(torch_dev, R), e, tol, 1e-12)
    assert handle.workspace_bytes() >= handle.realify_workspace(nk, nc, R.shape[2], e, tol)
