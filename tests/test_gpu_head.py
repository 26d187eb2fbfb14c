"""Position of G = 0 in the dielectric list.  The split path recomputes row
and column `head` of chi in FP64 (k_headwing) and the finalize leaves them
alone; these tests put G = 0 at index 5 of a permuted list (head = 5) and
drop the FP64 head recomputation altogether (head = -1), through
pair densities, chi0 in both precisions and eps^-1, against the oracle."""

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
def permuted(torch_dev, handle):
    """ng = 150 (three 64-tiles, ragged), G = 0 moved to index 5."""
    s = synth.small_system(n=16, ngw=300, ng=150, nv=4, nc=40, nk=2, seed=31)
    q = s["qs"][0]
    rng = np.random.default_rng(5)
    perm = rng.permutation(q["ng"])
    perm = np.concatenate([perm[perm != 0][:5], [0], perm[perm != 0][5:]])
    ge = np.ascontiguousarray(q["ge"][perm])
    assert tuple(ge[5]) == (0, 0, 0)
    M = handle.pair_density(s["n"], s["gw"], ge, dev(torch_dev, q["cv"]), dev(torch_dev, s["cc"]))
    torch_dev[0].cuda.synchronize()
    Mo = oracle.pair_density(s["gw"], ge, q["cv"], s["cc"])
    om = np.array([0.0, 7.0])
    pf = 1.0 / (s["nk"] * s["vol"])
    ref = oracle.chi(Mo, oracle.weights(q["ev"], s["ec"], om), pf)
    return dict(s=s, q=q, ge=ge, M=M, Mo=Mo, om=om, pf=pf, ref=ref)


def run_chi(torch_dev, handle, P, head, precision):
    s, q = P["s"], P["q"]
    (chi,) = handle.chi0([dict(M=P["M"], ev=dev(torch_dev, q["ev"]), ec=dev(torch_dev, s["ec"]), nk=s["nk"],
                               nv=s["nv"], nc=s["nc"], head=head, prefactor=P["pf"])], P["om"], precision=precision)
    torch_dev[0].cuda.synchronize()
    return chi


def test_pair_density_permuted_list(permuted):
    assert rel(permuted["M"].cpu().numpy(), permuted["Mo"]) <= TOL


@pytest.mark.parametrize("precision", [bgw.FP64, bgw.SPLIT_BF16])
def test_chi_head_5(torch_dev, handle, permuted, precision):
    chi = run_chi(torch_dev, handle, permuted, 5, precision).cpu().numpy()
    ref = permuted["ref"]
    tol = TOL if precision == bgw.FP64 else SPLIT_TOL
    for w in range(ref.shape[0]):
        assert rel(chi[w], ref[w]) <= tol
        # row and column 5 are FP64 in both precisions (the split path recomputes
        # them with the FP64 head kernel): the FP64 bar, also for split
        assert rel(chi[w][5], ref[w][5]) <= TOL
        assert rel(chi[w][:, 5], ref[w][:, 5]) <= TOL
        assert np.array_equal(chi[w][5], np.conj(chi[w][:, 5]))
        assert chi[w][5, 5].imag == 0.0
        # Hermitian with an exactly real diagonal
        assert np.array_equal(chi[w], chi[w].conj().T)


def test_chi_head_absent_split(torch_dev, handle, permuted):
    """head = -1: no FP64 recomputation, every entry from the split GEMM."""
    chi = run_chi(torch_dev, handle, permuted, -1, bgw.SPLIT_BF16).cpu().numpy()
    ref = permuted["ref"]
    for w in range(ref.shape[0]):
        assert rel(chi[w], ref[w]) <= SPLIT_TOL
        assert np.array_equal(chi[w], chi[w].conj().T)
    fp = run_chi(torch_dev, handle, permuted, -1, bgw.FP64).cpu().numpy()
    for w in range(ref.shape[0]):
        assert rel(fp[w], ref[w]) <= TOL


def test_eps_inv_permuted_list(torch_dev, handle, permuted):
    s, q = permuted["s"], permuted["q"]
    chi = run_chi(torch_dev, handle, permuted, 5, bgw.FP64)
    v = bgw.vcoul_bulk(s["bmat"], q["q"], permuted["ge"])
    einv, info = handle.eps_inv(dev(torch_dev, v), chi)
    assert np.all(info.cpu().numpy() == 0)
    ref, rinfo = oracle.eps_inv(v, chi.cpu().numpy())
    assert np.all(rinfo == 0)
    for w in range(ref.shape[0]):
        assert rel(einv[w].cpu().numpy(), ref[w]) <= TOL
