"""bgw_eps_inv_noalloc (the inversion with the library's fixed device
scratch) against bgw_eps_inv through the C-ABI: two calls in a row, the
first with more matrices than one launch of the fixed scratch holds at
Ng = 1200 (so the matrices go in several launches), the second smaller;
results to the FP64 bar, info identical."""

import numpy as np
import pytest

from paper_1111_4429_amd import bgw

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def system(torch, d, ng, nw, seed):
    """chi_w = -s_w X X^H / ng (Hermitian, negative definite), v(G) = 4 pi / (1 + |G|^2)-like: eps = 1 - v chi is
    well conditioned, and every frequency gets its own matrix."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng))
    C = -(X @ X.conj().T) / ng
    g2 = np.arange(ng, dtype=np.float64)
    v = 4 * np.pi / (1.0 + g2)
    s = 0.05 + 0.5 * rng.random(nw)
    C_d = torch.from_numpy(C).to(d)
    chi = torch.stack([float(si) * C_d for si in s]).contiguous()
    return torch.from_numpy(v).to(d), chi


def rel(torch, a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def test_noalloc_matches_eps_inv(torch_dev):
    torch, d = torch_dev
    h = bgw.Handle(0)
    for ng, nw, seed in ((1200, 60, 1), (300, 3, 2)):
        print(f"[no-alloc] ng={ng} nw={nw} seed={seed}", flush=True)
        v, chi = system(torch, d, ng, nw, seed)
        ref, rinfo = h.eps_inv(v, chi)
        out = torch.full_like(chi, float("nan"))
        info = torch.full((nw,), -7, dtype=torch.int32, device=d)
        h.eps_inv_noalloc(v, chi, out, info)
        torch.cuda.synchronize()
        assert torch.equal(info.cpu(), rinfo.cpu()) and int(info.abs().max()) == 0
        for w in range(nw):
            assert rel(torch, out[w], ref[w]) <= TOL, (ng, w)
    h.close()


def test_noalloc_rejects_oversize(torch_dev):
    torch, d = torch_dev
    h = bgw.Handle(0)
    z = torch.zeros(1, dtype=torch.float64, device=d)
    # an Ng above the library's largest (12288): refused on the host before any
    # launch, so the one-element buffers are never touched
    with pytest.raises(bgw.BgwError) as e:
        bgw._check(bgw.lib().bgw_eps_inv_noalloc(h._h, 13000, 1, bgw._dptr(z), bgw._dptr(z), bgw._dptr(z),
                                                 bgw._dptr(z), bgw._stream()))
    assert e.value.code == bgw.BGW_ERR_UNSUPPORTED
    assert "12288" in str(e.value)
    h.close()
