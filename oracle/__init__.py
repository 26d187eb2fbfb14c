"""Oracle for the RPA polarizability hot path -- TEST INFRASTRUCTURE ONLY.

A plain CPU complex128 implementation of what the GPU path computes, used
to judge it.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product
library never does, and the two share no code (the only common module is
the seeded input generator, which does none of the method's arithmetic).

The arithmetic lives in ``oracle.c`` (plain C99 loops + OpenMP); this file
only marshals numpy arrays.  Each wrapper names the passage of the paper
it follows:

* ``pair_density``  plane-wave matrix element M_vc(k,q,G) (epsilon section,
  matrix-element equation) evaluated exactly as a G-space convolution.
* ``weights``       1/(E_v,k+q - E_c,k) (static chi equation) and its
  imaginary-frequency continuation Delta/(Delta^2+omega^2), taken from the
  retarded/advanced dielectric equation at E = i omega, delta -> 0+.
* ``weights_real``  the complex weights of that equation at real E with
  broadening delta (retarded or advanced), for the full-frequency chi.
* ``ff_grid``       the real-frequency grid of the full-frequency run.
* ``bse_kx``        the Bethe-Salpeter exchange kernel (optical-properties
  section, exchange-term equation), G = 0 left out.
* ``sigma``         static self-energy matrix elements of one q: bare exchange
  (hf-x equation), screened exchange (cohsex-sx) and the Coulomb hole in its
  sum form (cohsex-ch-sum).
* ``chi``           the chi sum, compensated, any block of (G, G').
* ``vcoul``         bulk bare Coulomb 4 pi/|q+G|^2.
* ``eps``           epsilon = 1 - v chi (asymmetric Coulomb form).
* ``inverse``       Gaussian elimination with partial pivoting on [A | I]
  (ZGESV semantics), LAPACK INFO convention.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

HARTREE_EV = 27.211386245988


def build() -> str:
    """Compile oracle.c into liboracle.so with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu99", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        Lg = ctypes.c_long
        D = ctypes.c_double
        L.orc_pair_density.argtypes = [I, P, I, P, I, I, I, P, P, Lg, P, P]
        L.orc_weights.argtypes = [I, I, I, P, P, I, P, P]
        L.orc_chi.argtypes = [Lg, I, P, I, P, D, I, P, I, P, P]
        L.orc_vcoul.argtypes = [P, P, I, P, P]
        L.orc_eps.argtypes = [I, I, P, P, P]
        L.orc_inverse.argtypes = [I, P, P]
        L.orc_weights_real.argtypes = [I, I, I, P, P, I, P, D, I, P]
        L.orc_chi_cw.argtypes = [Lg, I, P, I, P, D, I, P, I, P, P]
        L.orc_ff_grid.argtypes = [D, D, D, D, I, P]
        L.orc_bse_kx.argtypes = [Lg, I, P, P, I, D, I, P, P]
        L.orc_sigma.argtypes = [I, I, I, I, P, I, P, P, D, P]
        L.orc_realify.argtypes = [I, I, I, P, P, D, P]
        for f in (L.orc_pair_density, L.orc_weights, L.orc_chi, L.orc_vcoul, L.orc_eps, L.orc_inverse,
                  L.orc_num_threads, L.orc_weights_real, L.orc_chi_cw, L.orc_ff_grid, L.orc_bse_kx, L.orc_sigma):
            f.restype = I
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def pair_density(gw: np.ndarray, ge: np.ndarray, cv: np.ndarray, cc: np.ndarray,
                 pairs: Optional[Sequence[int]] = None) -> np.ndarray:
    """M[p][G] for pair indices t = (k*nv + v)*nc + c (all pairs if None).

    cv: complex128 [nk][nv][ngw] valence at k+q; cc: [nk][nc][ngw] conduction at k.
    """
    gw = np.ascontiguousarray(gw, dtype=np.int32)
    ge = np.ascontiguousarray(ge, dtype=np.int32)
    cv = np.ascontiguousarray(cv, dtype=np.complex128)
    cc = np.ascontiguousarray(cc, dtype=np.complex128)
    nk, nv, ngw = cv.shape
    nc = cc.shape[1]
    assert cc.shape == (nk, nc, ngw) and gw.shape == (ngw, 3)
    if pairs is None:
        parr = None
        npairs = nk * nv * nc
    else:
        parr = np.ascontiguousarray(pairs, dtype=np.int64)
        npairs = parr.size
    out = np.zeros((npairs, ge.shape[0]), dtype=np.complex128)
    rc = lib().orc_pair_density(ngw, _p(gw), ge.shape[0], _p(ge), nk, nv, nc, _p(cv), _p(cc),
                                npairs, None if parr is None else _p(parr), _p(out))
    if rc != 0:
        raise RuntimeError(f"orc_pair_density failed: {rc}")
    return out


def weights(ev: np.ndarray, ec: np.ndarray, omega_ev: Sequence[float]) -> np.ndarray:
    ev = np.ascontiguousarray(ev, dtype=np.float64)
    ec = np.ascontiguousarray(ec, dtype=np.float64)
    om = np.ascontiguousarray(omega_ev, dtype=np.float64).reshape(-1)
    nk, nv = ev.shape
    nc = ec.shape[1]
    out = np.zeros((om.size, nk * nv * nc))
    rc = lib().orc_weights(nk, nv, nc, _p(ev), _p(ec), om.size, _p(om), _p(out))
    if rc != 0:
        raise ValueError(f"orc_weights failed: {rc}")
    return out


def weights_real(ev: np.ndarray, ec: np.ndarray, E_ev: Sequence[float], delta_ev: float,
                 kind: str = "retarded") -> np.ndarray:
    """Complex weights [nE][K] of the retarded (or advanced) dielectric equation at real E (eV)."""
    ev = np.ascontiguousarray(ev, dtype=np.float64)
    ec = np.ascontiguousarray(ec, dtype=np.float64)
    E = np.ascontiguousarray(E_ev, dtype=np.float64).reshape(-1)
    nk, nv = ev.shape
    nc = ec.shape[1]
    out = np.zeros((E.size, nk * nv * nc), dtype=np.complex128)
    rc = lib().orc_weights_real(nk, nv, nc, _p(ev), _p(ec), E.size, _p(E), float(delta_ev),
                                1 if kind == "retarded" else 0, _p(out))
    if rc != 0:
        raise ValueError(f"orc_weights_real failed: {rc}")
    return out


def ff_grid(dE: float, e_low: float, e_high: float, increment: float) -> np.ndarray:
    """The full-frequency real-axis grid (eV)."""
    n = lib().orc_ff_grid(float(dE), float(e_low), float(e_high), float(increment), 0, None)
    if n < 0:
        raise ValueError("bad frequency-grid parameters")
    out = np.zeros(n)
    lib().orc_ff_grid(float(dE), float(e_low), float(e_high), float(increment), n, _p(out))
    return out


def chi(M: np.ndarray, w: np.ndarray, pf: float, rows: Optional[Sequence[int]] = None,
        cols: Optional[Sequence[int]] = None) -> np.ndarray:
    """chi[w][rows][cols] = pf sum_t conj(M_t(G)) w_t M_t(G'); w real [nw][K], or complex
    (real frequency axis)."""
    M = np.ascontiguousarray(M, dtype=np.complex128)
    if np.iscomplexobj(w):
        wc = np.ascontiguousarray(np.atleast_2d(w), dtype=np.complex128)
        K, ng = M.shape
        assert wc.shape[1] == K
        r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
        c = None if cols is None else np.ascontiguousarray(cols, dtype=np.int32)
        nr = ng if r is None else r.size
        ncl = ng if c is None else c.size
        out = np.zeros((wc.shape[0], nr, ncl), dtype=np.complex128)
        rc = lib().orc_chi_cw(K, ng, _p(M), wc.shape[0], _p(wc), float(pf), nr, None if r is None else _p(r),
                              ncl, None if c is None else _p(c), _p(out))
        if rc != 0:
            raise RuntimeError(f"orc_chi_cw failed: {rc}")
        return out
    w = np.ascontiguousarray(np.atleast_2d(w), dtype=np.float64)
    K, ng = M.shape
    assert w.shape[1] == K
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    c = None if cols is None else np.ascontiguousarray(cols, dtype=np.int32)
    nr = ng if r is None else r.size
    ncl = ng if c is None else c.size
    out = np.zeros((w.shape[0], nr, ncl), dtype=np.complex128)
    rc = lib().orc_chi(K, ng, _p(M), w.shape[0], _p(w), float(pf), nr, None if r is None else _p(r),
                       ncl, None if c is None else _p(c), _p(out))
    if rc != 0:
        raise RuntimeError(f"orc_chi failed: {rc}")
    return out


def bse_kx(M: np.ndarray, v: np.ndarray, head: int, pf: float, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """Kx[t][t'] = pf sum_{G != head} conj(M_t(G)) v(G) M_t'(G): rows `rows` (all if None) x all K columns."""
    M = np.ascontiguousarray(M, dtype=np.complex128)
    v = np.ascontiguousarray(v, dtype=np.float64)
    K, ng = M.shape
    assert v.shape == (ng,)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = K if r is None else r.size
    out = np.zeros((nr, K), dtype=np.complex128)
    rc = lib().orc_bse_kx(K, ng, _p(M), _p(v), int(head), float(pf), nr, None if r is None else _p(r), _p(out))
    if rc != 0:
        raise RuntimeError(f"orc_bse_kx failed: {rc}")
    return out


SIGMA_KINDS = {"x": 0, "sx": 1, "ch": 2}


def sigma(kind: str, M: np.ndarray, v: np.ndarray, pf: float, einv: Optional[np.ndarray] = None,
          head: int = -1) -> np.ndarray:
    """Self-energy matrix [nouter][nouter] of one q from M[ninner][nouter][ng] (inner x outer pairs):
    kind "x" (bare exchange, G = head left out), "sx" (screened exchange) or "ch" (Coulomb hole, sum form)."""
    M = np.ascontiguousarray(M, dtype=np.complex128)
    v = np.ascontiguousarray(v, dtype=np.float64)
    ni, no, ng = M.shape
    e = None
    if kind != "x":
        e = np.ascontiguousarray(einv, dtype=np.complex128)
        assert e.shape == (ng, ng)
    out = np.zeros((no, no), dtype=np.complex128)
    rc = lib().orc_sigma(SIGMA_KINDS[kind], ni, no, ng, _p(M), int(head), _p(v), None if e is None else _p(e),
                         float(pf), _p(out))
    if rc != 0:
        raise ValueError(f"orc_sigma failed: {rc}")
    return out


def realify(c: np.ndarray, e: np.ndarray, tol: float):
    """Real coefficients [nk][nb][ngw] from complex ones (real flavor): Gram-Schmidt, largest remaining
    vector first, over Re and Im of each group of degenerate states (energies within tol of their
    neighbour).  Returns (r, number of groups that are not real up to a unitary)."""
    c = np.ascontiguousarray(c, dtype=np.complex128)
    e = np.ascontiguousarray(e, dtype=np.float64)
    nk, nb, ngw = c.shape
    assert e.shape == (nk, nb)
    r = np.zeros((nk, nb, ngw))
    bad = lib().orc_realify(nk, nb, ngw, _p(c), _p(e), float(tol), _p(r))
    if bad < 0:
        raise ValueError("orc_realify: bad arguments")
    return r, bad


def vcoul(bvec: np.ndarray, q: Sequence[float], ge: np.ndarray) -> np.ndarray:
    bvec = np.ascontiguousarray(bvec, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ge = np.ascontiguousarray(ge, dtype=np.int32)
    out = np.zeros(ge.shape[0])
    rc = lib().orc_vcoul(_p(bvec), _p(q), ge.shape[0], _p(ge), _p(out))
    if rc != 0:
        raise ValueError("|q+G| = 0 in vcoul")
    return out


def eps(v: np.ndarray, chi_: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    chi_ = np.ascontiguousarray(chi_, dtype=np.complex128)
    if chi_.ndim == 2:
        chi_ = chi_[None]
    nw, ng, _ = chi_.shape
    out = np.zeros_like(chi_)
    lib().orc_eps(ng, nw, _p(v), _p(chi_), _p(out))
    return out


def inverse(A: np.ndarray) -> Tuple[np.ndarray, int]:
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    out = np.zeros_like(A)
    info = lib().orc_inverse(n, _p(A), _p(out))
    if info < 0:
        raise MemoryError("orc_inverse allocation failed")
    return out, int(info)


def eps_inv(v: np.ndarray, chi_: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """epsilon^-1 for every frequency: returns (epsinv [nw][ng][ng], info [nw])."""
    e = eps(v, chi_)
    outs, infos = [], []
    for iw in range(e.shape[0]):
        x, info = inverse(e[iw])
        outs.append(x)
        infos.append(info)
    return np.stack(outs), np.array(infos, dtype=np.int32)


def prefactor(nk: int, vol: float) -> float:
    """Implicit 1/(N_k V_uc) normalisation of k/q sums (paper, GW-BSE overview)."""
    return 1.0 / (nk * vol)
