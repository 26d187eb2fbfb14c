"""Seeded synthetic inputs for the polarizability hot path.

This module only *draws* inputs: G-vector lists, orthonormal plane-wave
coefficients, band energies, the frequency list and the cell.  It holds
none of the method's arithmetic (no matrix elements, no weights, no chi,
no dielectric matrix), so the oracle and the GPU path can both be fed from
it without sharing any computation.

Conventions (see the paper's Appendix on wavefunction files for the
G-vector and normalisation conventions, and the epsilon section for the
two k-grids used at small q):

* G-vectors are integer Miller triples in reciprocal-lattice units with
  components in [-n/2, n/2).  One global list is ordered by
  (m.m, m_x, m_y, m_z); the wavefunction sphere is its first ``ngw``
  entries and each dielectric sphere its first ``ng`` entries, so G=0 is
  always index 0 and the dielectric sphere is contained in the
  wavefunction sphere.
* Coefficients: Re and Im ~ N(0, exp(-m.m/8)/2), then orthonormalised
  per k-point in band order (valence first) so that the squared
  coefficients of every band sum to 1.  The orthonormalisation is a QR
  factorisation whose R has a real positive diagonal, i.e. exactly the
  Gram-Schmidt result in exact arithmetic.
* Valence states at k+q for a small q0 (the shifted grid used for the
  q->0 head): orthonormalise (C_v,k + |q| xi_v/|xi_v|) over the valence
  bands only, xi_v an extra draw from the same envelope; energies at
  k+q0 equal those at k.  This makes |M_vc(G=0)| proportional to |q|.
* Valence states at a generic q (uneven-q batch, q index >= 1) are
  independent orthonormal sets with independent energies.
* Energies (eV): E_v ~ U[-10, 0], E_c ~ U[1, 20], sorted per k-point.
* Cell: cubic, V_uc = 67.5 * Nv bohr^3, reciprocal basis (2 pi / L) I.
* numpy PCG64 ``default_rng(seed)``; draw order: C (k, band, G, re/im),
  then xi, then E_v, E_c, then the uneven-q sizes and q vectors.
"""

from __future__ import annotations

import dataclasses
import hashlib
from typing import Dict, List, Optional, Sequence

import numpy as np

Q0_CRYSTAL = (0.001, 0.0, 0.0)


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes of one synthetic workload."""

    name: str
    n: int                 # FFT grid is n x n x n
    ng: int                # dielectric sphere size (fixed-size workloads)
    ngw: int               # wavefunction sphere size
    nv: int
    nc: int
    nk: int
    nw: int = 1            # number of frequencies
    freq: str = "static"   # "static" or "gauss-legendre-0-100eV"
    nq: int = 1
    ng_range: Optional[tuple] = None  # uneven q batch: Ng_q ~ U{lo..hi}
    precision: str = "fp64"
    flavor: str = "complex"  # "real": real coefficients (inversion + time-reversal symmetry)

    @property
    def npairs(self) -> int:
        return self.nv * self.nc * self.nk


# The five workloads, named by what they are.
WORKLOADS: Dict[str, Workload] = {
    "tiny-static-16": Workload("tiny-static-16", n=16, ng=300, ngw=300, nv=4, nc=16, nk=1),
    "silicon-like-48": Workload("silicon-like-48", n=48, ng=1500, ngw=1500, nv=4, nc=400, nk=64),
    "supercell-96": Workload("supercell-96", n=96, ng=8000, ngw=8000, nv=128, nc=2000, nk=1,
                             precision="split"),
    "imag-freq-64": Workload("imag-freq-64", n=64, ng=4000, ngw=4000, nv=64, nc=1000, nk=8,
                             nw=32, freq="gauss-legendre-0-100eV", precision="split"),
    "uneven-q-48": Workload("uneven-q-48", n=48, ng=6000, ngw=6000, nv=32, nc=600, nk=27,
                            nq=64, ng_range=(500, 6000), precision="split"),
    # Bethe-Salpeter exchange kernel over K = 4 x 64 x 64 = 16384 pairs of the silicon-like cell
    "bse-kx-48": Workload("bse-kx-48", n=48, ng=1500, ngw=1500, nv=4, nc=64, nk=64),
    # static self-energy of the silicon-like cell: 404 inner states (4 occupied), 64 outer states, one q
    "sigma-48": Workload("sigma-48", n=48, ng=1500, ngw=1500, nv=4, nc=400, nk=1),
    # the silicon-like cell on the real frequency axis (retarded chi on the full-frequency grid)
    "realaxis-48": Workload("realaxis-48", n=48, ng=1500, ngw=1500, nv=4, nc=400, nk=64, precision="split"),
    # the silicon-like workload in the real flavor (real coefficients)
    "silicon-like-48-real": Workload("silicon-like-48-real", n=48, ng=1500, ngw=1500, nv=4, nc=400, nk=64,
                                     flavor="real"),
}


def gvector_list(count: int) -> np.ndarray:
    """First ``count`` Miller triples ordered by (m.m, m_x, m_y, m_z)."""
    if count <= 0:
        return np.zeros((0, 3), dtype=np.int32)
    r = 1
    while (2 * r + 1) ** 3 * 0.5 < count:  # sphere of radius r holds ~ 4.19 r^3
        r += 1
    r += 2
    ax = np.arange(-r, r + 1, dtype=np.int64)
    m = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    mm = (m * m).sum(axis=1)
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], mm))
    sel = m[order[:count]]
    # make sure the cube was large enough: the last shell taken must be complete
    assert mm[order[count - 1]] < r * r, "cube too small for requested sphere"
    return np.ascontiguousarray(sel.astype(np.int32))


def _envelope(g: np.ndarray) -> np.ndarray:
    mm = (g.astype(np.float64) ** 2).sum(axis=1)
    return np.sqrt(np.exp(-mm / 8.0) / 2.0)


def _draw_coeffs(rng: np.random.Generator, shape: Sequence[int], g: np.ndarray, real: bool = False) -> np.ndarray:
    z = rng.standard_normal(tuple(shape) + (g.shape[0], 2))
    if real:  # the same variance per coefficient in one real component
        return z[..., 0] * np.sqrt(2.0) * _envelope(g)
    c = (z[..., 0] + 1j * z[..., 1]) * _envelope(g)
    return c


def orthonormalise(vectors: np.ndarray) -> np.ndarray:
    """Gram-Schmidt of the rows of ``vectors`` ([nb][ngw]) in row order.

    Implemented as a Householder QR whose R diagonal is made real and
    positive, which is the Gram-Schmidt result in exact arithmetic.
    """
    a = np.ascontiguousarray(vectors.T)          # columns = bands
    qm, rm = np.linalg.qr(a, mode="reduced")
    d = np.diagonal(rm)
    phase = d / np.abs(d)
    qm = qm * phase[None, :]
    return np.ascontiguousarray(qm.T)


def cell(nv: int):
    vol = 67.5 * nv
    length = vol ** (1.0 / 3.0)
    bmat = (2.0 * np.pi / length) * np.eye(3)
    return vol, bmat


def frequencies(wl: Workload) -> np.ndarray:
    if wl.freq == "static":
        return np.zeros(1)
    if wl.freq == "gauss-legendre-0-100eV":
        x, _ = np.polynomial.legendre.leggauss(wl.nw)
        return 50.0 * (x + 1.0)
    raise ValueError(wl.freq)


def make_system(wl: Workload, seed: int = 0, q_subset: Optional[Sequence[int]] = None,
                q0: Sequence[float] = Q0_CRYSTAL) -> dict:
    """Draw every input of ``wl``.

    Returns a dict with host numpy arrays:
      n (int), gw int32[ngw][3], nk, nv, nc, vol, bmat[3][3], omega[nw] (eV),
      cc complex128[nk][nc][ngw] (conduction at k),
      ec float64[nk][nc] (eV),
      qs: list of per-q dicts {q (crystal, [3]), ng, ge int32[ng][3],
          cv complex128[nk][nv][ngw] (valence at k+q), ev float64[nk][nv]}.
    ``q_subset`` restricts which q entries of an uneven-q batch are built
    (their draws still follow the fixed order, each q with its own stream).
    """
    rng = np.random.default_rng(seed)
    gw = gvector_list(wl.ngw)
    nb = wl.nv + wl.nc
    real = wl.flavor == "real"
    c = _draw_coeffs(rng, (wl.nk, nb), gw, real)
    xi = _draw_coeffs(rng, (wl.nk, wl.nv), gw, real)
    ev = np.sort(rng.uniform(-10.0, 0.0, size=(wl.nk, wl.nv)), axis=1)
    ec = np.sort(rng.uniform(1.0, 20.0, size=(wl.nk, wl.nc)), axis=1)

    ctype = np.float64 if real else np.complex128
    cv0 = np.empty((wl.nk, wl.nv, wl.ngw), dtype=ctype)
    cc = np.empty((wl.nk, wl.nc, wl.ngw), dtype=ctype)
    qabs = float(np.linalg.norm(q0))
    for k in range(wl.nk):
        ortho = orthonormalise(c[k])
        cc[k] = ortho[wl.nv:]
        pert = ortho[: wl.nv] + qabs * xi[k] / np.linalg.norm(xi[k], axis=1, keepdims=True)
        cv0[k] = orthonormalise(pert)
    del c, xi

    vol, bmat = cell(wl.nv)
    qs: List[dict] = []
    if wl.nq == 1:
        qs.append(dict(q=np.array(q0, dtype=np.float64), ng=wl.ng, ge=gvector_list(wl.ng), cv=cv0,
                       ev=ev.copy(), iq=0))
    else:
        lo, hi = wl.ng_range
        ngq = rng.integers(lo, hi + 1, size=wl.nq)
        qvec = rng.uniform(-0.5, 0.5, size=(wl.nq, 3))
        qvec[0] = q0
        ngq[0] = min(int(ngq[0]), wl.ngw)
        wanted = range(wl.nq) if q_subset is None else q_subset
        for iq in wanted:
            ng = int(min(ngq[iq], wl.ngw))
            if iq == 0:
                qs.append(dict(q=qvec[0].copy(), ng=ng, ge=gvector_list(ng), cv=cv0, ev=ev.copy(), iq=0))
                continue
            rq = np.random.default_rng([seed, iq])
            cq = _draw_coeffs(rq, (wl.nk, wl.nv), gw, real)
            cvq = np.stack([orthonormalise(cq[k]) for k in range(wl.nk)])
            evq = np.sort(rq.uniform(-10.0, 0.0, size=(wl.nk, wl.nv)), axis=1)
            qs.append(dict(q=qvec[iq].copy(), ng=ng, ge=gvector_list(ng), cv=cvq, ev=evq, iq=iq))
    return dict(name=wl.name, n=wl.n, gw=gw, nk=wl.nk, nv=wl.nv, nc=wl.nc, vol=vol, bmat=bmat,
                omega=frequencies(wl), cc=cc, ec=ec, qs=qs)


def uneven_q_sizes(wl: Workload, seed: int = 0) -> np.ndarray:
    """Ng_q of every q of an uneven-q workload, as make_system draws them
    (the earlier draws are replayed in chunks, nothing is kept)."""
    assert wl.nq > 1 and wl.ng_range is not None
    rng = np.random.default_rng(seed)
    ngw = wl.ngw
    for _ in range(wl.nk * (wl.nv + wl.nc)):   # C, one band at a time
        rng.standard_normal((1, ngw, 2))
    for _ in range(wl.nk * wl.nv):             # xi
        rng.standard_normal((1, ngw, 2))
    rng.uniform(-10.0, 0.0, size=(wl.nk, wl.nv))
    rng.uniform(1.0, 20.0, size=(wl.nk, wl.nc))
    lo, hi = wl.ng_range
    ngq = rng.integers(lo, hi + 1, size=wl.nq)
    return np.minimum(ngq, ngw)


def small_system(n: int, ngw: int, ng: int, nv: int, nc: int, nk: int = 1, seed: int = 0,
                 q=Q0_CRYSTAL, nw: int = 1, freq: str = "static", flavor: str = "complex") -> dict:
    """A system of arbitrary (small) size drawn by the same recipe."""
    wl = Workload("custom", n=n, ng=ng, ngw=ngw, nv=nv, nc=nc, nk=nk, nw=nw, freq=freq, flavor=flavor)
    return make_system(wl, seed, q0=q)


def digest(arrays: Sequence[np.ndarray]) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
