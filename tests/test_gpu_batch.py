"""Batched chi0 through the C-ABI: many q with uneven Ng and many frequencies
in one call (one persistent FP64 launch), HIP-graph capture and replay, and
the autotuner.  Every (q, omega) result is checked against the oracle on the
same M: <= 1e-12 (FP64), <= 1e-9 (split)."""

import json
import os

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


def dev(torch_dev, a):
    torch, d = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


@pytest.fixture(scope="module")
def uneven(torch_dev):
    """Five q of an uneven batch (Ng_q ~ U{40..300}, generic q vectors), the
    q = q0 entry first; M per q from the oracle's convolution."""
    wl = synth.Workload("uneven-small", n=24, ng=300, ngw=300, nv=3, nc=7, nk=2, nq=5, ng_range=(40, 300))
    s = synth.make_system(wl, seed=3)
    qs = []
    for q in s["qs"]:
        M = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"])
        qs.append(dict(Mh=M, ev=q["ev"], ng=q["ng"], head=0))
    pf = 1.0 / (s["nk"] * s["vol"])
    om = np.array([0.0, 1.5, 30.0])
    return dict(s=s, qs=qs, pf=pf, om=om)


def entries(torch_dev, u, Ms=None):
    s = u["s"]
    out = []
    for i, q in enumerate(u["qs"]):
        M = dev(torch_dev, q["Mh"]) if Ms is None else Ms[i]
        out.append(dict(M=M, ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"],
                        nc=s["nc"], head=q["head"], prefactor=u["pf"]))
    return out


def refs(u):
    s = u["s"]
    return [oracle.chi(q["Mh"], oracle.weights(q["ev"], s["ec"], u["om"]), u["pf"]) for q in u["qs"]]


@pytest.mark.parametrize("tile", [None, "32", "64"])
def test_uneven_batch_fp64_vs_oracle(torch_dev, uneven, tile, monkeypatch):
    torch = torch_dev[0]
    if tile:
        monkeypatch.setenv("BGW_HERK_TILE", tile)
    h = bgw.Handle(0)
    ngs = [q["ng"] for q in uneven["qs"]]
    assert len(set(ngs)) == len(ngs) and min(ngs) < 64 < max(ngs)
    chis = h.chi0(entries(torch_dev, uneven), uneven["om"])
    torch.cuda.synchronize()
    for c, r in zip(chis, refs(uneven)):
        c = c.cpu().numpy()
        for i in range(len(uneven["om"])):
            assert rel(c[i], r[i]) <= TOL
            assert np.array_equal(c[i], c[i].conj().T)
    # the batch equals the same problems launched one q at a time (to rounding)
    for qi, e in enumerate(entries(torch_dev, uneven)):
        (one,) = h.chi0([e], uneven["om"])
        torch.cuda.synchronize()
        assert rel(one.cpu().numpy(), chis[qi].cpu().numpy()) <= 1e-14
    h.close()


def test_uneven_batch_accumulate(torch_dev, uneven):
    torch = torch_dev[0]
    h = bgw.Handle(0)
    ents = entries(torch_dev, uneven)
    chis = h.chi0(ents, uneven["om"])
    h.chi0(ents, uneven["om"], accumulate=True, chis=chis)
    torch.cuda.synchronize()
    for c, r in zip(chis, refs(uneven)):
        assert rel(c.cpu().numpy(), 2 * r) <= TOL
    h.close()


def test_uneven_batch_split_vs_oracle(torch_dev, uneven):
    torch = torch_dev[0]
    h = bgw.Handle(0)
    chis = h.chi0(entries(torch_dev, uneven), uneven["om"], precision=bgw.SPLIT_BF16)
    torch.cuda.synchronize()
    for c, r in zip(chis, refs(uneven)):
        c = c.cpu().numpy()
        for i in range(len(uneven["om"])):
            assert rel(c[i], r[i]) <= SPLIT_TOL
            assert rel(c[i][0], r[i][0]) <= 1e-13  # FP64 head row
    h.close()


@pytest.mark.parametrize("precision", [bgw.FP64, bgw.SPLIT_BF16])
def test_graph_replay_matches_eager(torch_dev, uneven, precision):
    """Capture on first use, then replays with eager work and synchronisation
    in between; every replay equals the eager result bitwise, and a replay
    after the inputs change follows the new inputs (the graph holds addresses)."""
    torch = torch_dev[0]
    h = bgw.Handle(0)
    Ms = [dev(torch_dev, q["Mh"]) for q in uneven["qs"]]
    ents = entries(torch_dev, uneven, Ms)
    eager = [c.clone() for c in h.chi0(ents, uneven["om"], precision=precision)]
    outs = [torch.empty_like(c) for c in eager]
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        h.chi0(ents, uneven["om"], precision=precision, chis=outs, use_graph=True)
        junk = torch.randn(512, 512, dtype=torch.float64, device=Ms[0].device)
        (junk @ junk).sum().item()  # eager work and a synchronisation between replays
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), f"replay {rep}"
    # new data behind the same addresses
    for M in Ms:
        M.mul_(2.0)
    h.chi0(ents, uneven["om"], precision=precision, chis=outs, use_graph=True)
    torch.cuda.synchronize()
    tol = TOL if precision == bgw.FP64 else SPLIT_TOL
    for o, r in zip(outs, refs(uneven)):
        assert rel(o.cpu().numpy(), 4 * r) <= tol
    h.close()


def test_autotune_and_cache(torch_dev, uneven, tmp_path):
    torch = torch_dev[0]
    cache = tmp_path / "tune.jsonl"
    os.environ["BGW_TUNE_CACHE"] = str(cache)
    try:
        h = bgw.Handle(0)
        ents = entries(torch_dev, uneven)
        K = uneven["s"]["nk"] * uneven["s"]["nv"] * uneven["s"]["nc"]
        for prec in (bgw.FP64, bgw.SPLIT_BF16):
            assert not h.tuned_config(prec, uneven["qs"][0]["ng"], K)["tuned"]
            h.autotune(ents, uneven["om"], precision=prec)
            for q in uneven["qs"]:
                cfg = h.tuned_config(prec, q["ng"], K)
                assert cfg["tuned"]
                assert cfg["tile"] in (32, 64) and cfg["items_per_cu"] in (2, 8, 32)
                if prec == bgw.SPLIT_BF16:
                    assert cfg["split_nsplit"] in (1, 2, 4, 8, 16)
            # tuned plans still match the oracle
            chis = h.chi0(ents, uneven["om"], precision=prec)
            torch.cuda.synchronize()
            tol = TOL if prec == bgw.FP64 else SPLIT_TOL
            for c, r in zip(chis, refs(uneven)):
                assert rel(c.cpu().numpy(), r) <= tol
        h.close()
        lines = [json.loads(l) for l in cache.read_text().splitlines()]
        classes = {(l["precision"], l["ng_class"], l["k_log2"]) for l in lines}
        assert {0, 1} == {c[0] for c in classes}
        assert all(l["ng_class"] % 512 == 0 and l["ms"] > 0 for l in lines)
        # a new handle reads the cache back
        h2 = bgw.Handle(0)
        assert h2.tuned_config(bgw.FP64, uneven["qs"][0]["ng"], K)["tuned"]
        h2.close()
    finally:
        del os.environ["BGW_TUNE_CACHE"]


def test_split_partials_fully_written(torch_dev, tmp_path, monkeypatch):
    """A K-split count that does not divide the chunk count (7 splits of the
    10 chunks of K = 960 pairs) on a handle whose workspace already holds an
    earlier call's partial sums: every partial sum the finalize adds must be
    written by this call's GEMM."""
    torch = torch_dev[0]
    s = synth.small_system(n=16, ngw=300, ng=150, nv=4, nc=60, nk=4, seed=5)
    q = s["qs"][0]
    K = s["nk"] * s["nv"] * s["nc"]
    assert K == 960
    M = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"])
    pf = 1.0 / (s["nk"] * s["vol"])
    om = np.array([0.0, 2.0, 20.0])
    ent = dict(M=dev(torch_dev, M), ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"], nv=s["nv"],
               nc=s["nc"], head=0, prefactor=pf)
    ref = oracle.chi(M, oracle.weights(q["ev"], s["ec"], om), pf)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("BGW_TUNE_CACHE", str(cache))
    h = bgw.Handle(0)
    h.autotune([ent], om, precision=bgw.SPLIT_BF16)
    h.close()
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    extra = [dict(l, nsplit=7) for l in lines if l["precision"] == bgw.SPLIT_BF16]
    assert extra
    with open(cache, "a") as f:
        for l in extra:
            f.write(json.dumps(l) + "\n")
    h2 = bgw.Handle(0)
    assert h2.tuned_config(bgw.SPLIT_BF16, q["ng"], K)["split_nsplit"] == 7
    # an accumulating FP64 call leaves its partial sums in the workspace
    acc = torch.zeros((len(om), q["ng"], q["ng"]), dtype=torch.complex128, device=ent["M"].device)
    h2.chi0([ent], om, chis=[acc], accumulate=True)
    for rep in range(2):
        (c,) = h2.chi0([ent], om, precision=bgw.SPLIT_BF16)
        torch.cuda.synchronize()
        c = c.cpu().numpy()
        for i in range(len(om)):
            assert rel(c[i], ref[i]) <= SPLIT_TOL, (rep, i)
    h2.close()


def test_many_frequencies_one_launch(torch_dev):
    """32 Gauss-Legendre frequencies of one q in one call; each frequency vs
    the oracle, and |chi_GG(i omega)| decreasing in omega."""
    torch = torch_dev[0]
    s = synth.small_system(n=16, ngw=181, ng=130, nv=3, nc=9, nk=3, seed=21, nw=32, freq="gauss-legendre-0-100eV")
    q = s["qs"][0]
    M = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"])
    pf = 1.0 / (s["nk"] * s["vol"])
    h = bgw.Handle(0)
    h.set_timing(True)
    (chi,) = h.chi0([dict(M=dev(torch_dev, M), ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"],
                          nv=s["nv"], nc=s["nc"], head=0, prefactor=pf)], s["omega"])
    torch.cuda.synchronize()
    t = h.timing()
    assert t["herk"][1] == 1 and t["weights"][1] == 1 and t["finalize"][1] == 1  # one launch each
    ref = oracle.chi(M, oracle.weights(q["ev"], s["ec"], s["omega"]), pf)
    chi = chi.cpu().numpy()
    for i in range(32):
        assert rel(chi[i], ref[i]) <= TOL
    d = np.abs(np.einsum("wii->wi", chi))
    assert np.all(np.diff(d, axis=0) <= 1e-15 * d[:-1])
    h.close()
