"""ctypes binding of libbgw (include/bgw.h): argument marshalling only.

Device buffers are torch tensors on a HIP device (``torch.complex128`` for
complex arrays, ``torch.float64`` for energies/Coulomb, ``torch.int32`` for
``info``); G-vector lists and frequencies are host numpy arrays.  Every call
is enqueued on ``torch.cuda.current_stream()``.  There is no fallback: if the
native library is missing or the GPU is absent, calls raise.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbgw.so")

BGW_OK = 0
BGW_ERR_ARG = -1
BGW_ERR_ALIAS = -2
BGW_ERR_SHAPE = -3
BGW_ERR_HIP = -4
BGW_ERR_NOMEM = -5
BGW_ERR_UNSUPPORTED = -6
FP64 = 0
SPLIT_BF16 = 1
AXIS_IMAG = 0
AXIS_RETARDED = 1
AXIS_ADVANCED = 2
_AXES = {"imag": AXIS_IMAG, "retarded": AXIS_RETARDED, "advanced": AXIS_ADVANCED}

# every symbol declared in include/bgw.h
EXPORTS = [
    "bgw_version", "bgw_create", "bgw_destroy", "bgw_last_error", "bgw_workspace_bytes",
    "bgw_pair_desc_check", "bgw_pair_density", "bgw_chi0", "bgw_eps_inv", "bgw_vcoul_bulk",
    "bgw_set_timing", "bgw_get_timing", "bgw_reset_timing", "bgw_pair_transform_box", "bgw_autotune",
    "bgw_tuned_config", "bgw_pair_density_workspace", "bgw_chi0_workspace", "bgw_eps_inv_workspace",
    "bgw_ff_grid", "bgw_eps_inv_noalloc", "bgw_bse_kx", "bgw_bse_kx_workspace", "bgw_sigma",
    "bgw_sigma_workspace", "bgw_pair_density_real", "bgw_chi0_real", "bgw_chi0_real_workspace", "bgw_realify",
    "bgw_realify_workspace", "bgw_eps_inv_nsd",
]

KERNELS = ["band", "pair", "weights", "herk", "finalize", "split_slice", "split_herk", "headwing", "eps_build",
           "invert", "pair_x"]


class BgwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bgw error {code}: {msg}")
        self.code = code


class PairDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("ngw", ctypes.c_int),
        ("gw", ctypes.c_void_p),
        ("ng", ctypes.c_int),
        ("ge", ctypes.c_void_p),
        ("nk", ctypes.c_int),
        ("nv", ctypes.c_int),
        ("nc", ctypes.c_int),
        ("cv", ctypes.c_void_p),
        ("cc", ctypes.c_void_p),
    ]


class ChiQ(ctypes.Structure):
    _fields_ = [
        ("ng", ctypes.c_int),
        ("nk", ctypes.c_int),
        ("nv", ctypes.c_int),
        ("nc", ctypes.c_int),
        ("M", ctypes.c_void_p),
        ("ev", ctypes.c_void_p),
        ("ec", ctypes.c_void_p),
        ("head", ctypes.c_int),
        ("prefactor", ctypes.c_double),
        ("chi", ctypes.c_void_p),
    ]


class ChiDesc(ctypes.Structure):
    _fields_ = [
        ("nq", ctypes.c_int),
        ("q", ctypes.POINTER(ChiQ)),
        ("nw", ctypes.c_int),
        ("omega", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int),
        ("accumulate", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("axis", ctypes.c_int),
        ("broadening", ctypes.c_double),
    ]


class KxDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_void_p),
        ("K", ctypes.c_longlong),
        ("ng", ctypes.c_int),
        ("head", ctypes.c_int),
        ("v", ctypes.c_void_p),
        ("prefactor", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("pad", ctypes.c_int),
        ("kx", ctypes.c_void_p),
    ]


SIGMA_X, SIGMA_SX, SIGMA_CH = 0, 1, 2
_SIGMA = {"x": SIGMA_X, "sx": SIGMA_SX, "ch": SIGMA_CH}


class SigmaDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_void_p),
        ("ninner", ctypes.c_int),
        ("nouter", ctypes.c_int),
        ("ng", ctypes.c_int),
        ("kind", ctypes.c_int),
        ("head", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("v", ctypes.c_void_p),
        ("epsinv", ctypes.c_void_p),
        ("prefactor", ctypes.c_double),
        ("accumulate", ctypes.c_int),
        ("pad", ctypes.c_int),
        ("sigma", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libbgw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"native library {LIB_PATH} is missing; run __graft_entry__.build()")
        # A process must hold one HIP runtime.  PyTorch ships its own
        # libamdhip64 and asks for it by its unversioned name, so if this
        # library were loaded first (binding the system runtime) a later
        # torch import would map a second runtime and one of the two would
        # find no device.  Loading torch first lets this library bind to
        # torch's runtime through the shared soname.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.bgw_version.restype = I
        L.bgw_create.argtypes = [ctypes.POINTER(P), I]
        L.bgw_destroy.argtypes = [P]
        L.bgw_last_error.restype = ctypes.c_char_p
        L.bgw_workspace_bytes.argtypes = [P]
        L.bgw_workspace_bytes.restype = ctypes.c_size_t
        L.bgw_pair_desc_check.argtypes = [ctypes.POINTER(PairDesc)]
        L.bgw_pair_density.argtypes = [P, ctypes.POINTER(PairDesc), P, P]
        L.bgw_chi0.argtypes = [P, ctypes.POINTER(ChiDesc), P]
        L.bgw_eps_inv.argtypes = [P, I, I, P, P, P, P, P]
        L.bgw_eps_inv_noalloc.argtypes = [P, I, I, P, P, P, P, P]
        L.bgw_eps_inv_nsd.argtypes = [P, I, I, P, P, P, P, P]
        L.bgw_bse_kx.argtypes = [P, ctypes.POINTER(KxDesc), P]
        L.bgw_sigma.argtypes = [P, ctypes.POINTER(SigmaDesc), P]
        L.bgw_pair_density_real.argtypes = [P, ctypes.POINTER(PairDesc), P, P]
        L.bgw_chi0_real.argtypes = [P, ctypes.POINTER(ChiDesc), P]
        L.bgw_chi0_real_workspace.argtypes = [P, ctypes.POINTER(ChiDesc), ctypes.POINTER(ctypes.c_size_t)]
        L.bgw_realify.argtypes = [P, I, I, I, P, P, D, P, P, P]
        L.bgw_realify_workspace.argtypes = [P, I, I, I, P, D, ctypes.POINTER(ctypes.c_size_t)]
        L.bgw_sigma_workspace.argtypes = [P, ctypes.POINTER(SigmaDesc), ctypes.POINTER(ctypes.c_size_t)]
        L.bgw_bse_kx_workspace.argtypes = [P, ctypes.POINTER(KxDesc), ctypes.POINTER(ctypes.c_size_t)]
        L.bgw_vcoul_bulk.argtypes = [P, P, I, P, P]
        L.bgw_set_timing.argtypes = [P, I]
        L.bgw_get_timing.argtypes = [P, I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
        L.bgw_reset_timing.argtypes = [P]
        L.bgw_pair_transform_box.argtypes = [ctypes.POINTER(PairDesc), ctypes.POINTER(ctypes.c_int)]
        L.bgw_autotune.argtypes = [P, ctypes.POINTER(ChiDesc), P]
        L.bgw_tuned_config.argtypes = [P, I, I, ctypes.c_longlong, ctypes.POINTER(ctypes.c_int)]
        SZ = ctypes.POINTER(ctypes.c_size_t)
        L.bgw_pair_density_workspace.argtypes = [P, ctypes.POINTER(PairDesc), SZ]
        L.bgw_chi0_workspace.argtypes = [P, ctypes.POINTER(ChiDesc), SZ]
        L.bgw_eps_inv_workspace.argtypes = [P, I, I, SZ]
        L.bgw_ff_grid.argtypes = [D, D, D, D, I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        for f in ("bgw_create", "bgw_destroy", "bgw_pair_desc_check", "bgw_pair_density", "bgw_chi0",
                  "bgw_eps_inv", "bgw_vcoul_bulk", "bgw_set_timing", "bgw_get_timing", "bgw_reset_timing",
                  "bgw_pair_transform_box", "bgw_autotune", "bgw_tuned_config", "bgw_pair_density_workspace",
                  "bgw_chi0_workspace", "bgw_eps_inv_workspace", "bgw_ff_grid", "bgw_eps_inv_noalloc", "bgw_bse_kx",
                  "bgw_bse_kx_workspace", "bgw_sigma", "bgw_sigma_workspace", "bgw_pair_density_real",
                  "bgw_chi0_real", "bgw_chi0_real_workspace", "bgw_realify", "bgw_realify_workspace", "bgw_eps_inv_nsd"):
            getattr(L, f).restype = I
        _lib = L
    return _lib


def _check(rc: int):
    if rc != BGW_OK:
        raise BgwError(rc, lib().bgw_last_error().decode())


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _dptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_pair_desc(n, gw, ge, cv=None, cc=None, nk=None, nv=None, nc=None):
    """Build a PairDesc; gw/ge host int arrays, cv/cc device tensors (or None
    for host-only validation, in which case nk/nv/nc must be given)."""
    gw = _host_i32(gw)
    ge = _host_i32(ge)
    d = PairDesc()
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    d.n = (ctypes.c_int * 3)(*nn)
    d.ngw = gw.shape[0]
    d.gw = gw.ctypes.data
    d.ng = ge.shape[0]
    d.ge = ge.ctypes.data
    if cv is not None:
        nk, nv = int(cv.shape[0]), int(cv.shape[1])
        nc = int(cc.shape[1])
    d.nk, d.nv, d.nc = int(nk), int(nv), int(nc)
    d.cv = _dptr(cv) if cv is not None else 1
    d.cc = _dptr(cc) if cc is not None else 1
    d._keep = (gw, ge)  # keep host arrays alive
    return d


def pair_desc_check(n, gw, ge, nk=1, nv=1, nc=1) -> int:
    """Host-only validation; returns the BGW code (no GPU needed)."""
    d = make_pair_desc(n, gw, ge, nk=nk, nv=nv, nc=nc)
    return int(lib().bgw_pair_desc_check(ctypes.byref(d)))


def pair_transform_box(n, gw, ge):
    """The transform box the library will use (host-only, no GPU)."""
    d = make_pair_desc(n, gw, ge, nk=1, nv=1, nc=1)
    box = (ctypes.c_int * 3)()
    _check(lib().bgw_pair_transform_box(ctypes.byref(d), box))
    return tuple(box)


def ff_grid(spacing: float, low_cutoff: float, high_cutoff: float, increment: float) -> np.ndarray:
    """Real-frequency grid (eV) of a full-frequency calculation (host only)."""
    n = ctypes.c_int()
    _check(lib().bgw_ff_grid(spacing, low_cutoff, high_cutoff, increment, 0, None, ctypes.byref(n)))
    out = np.zeros(n.value)
    _check(lib().bgw_ff_grid(spacing, low_cutoff, high_cutoff, increment, n.value,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n)))
    return out


def vcoul_bulk(bvec, q, ge) -> np.ndarray:
    bvec = np.ascontiguousarray(bvec, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ge = _host_i32(ge)
    out = np.zeros(ge.shape[0])
    _check(lib().bgw_vcoul_bulk(bvec.ctypes.data, q.ctypes.data, ge.shape[0], ge.ctypes.data, out.ctypes.data))
    return out


class Handle:
    """A bgw handle bound to one HIP device (owns the workspace)."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available: the bgw library has no CPU path")
        self.device = device
        self._h = ctypes.c_void_p()
        _check(lib().bgw_create(ctypes.byref(self._h), device))

    def close(self):
        if self._h:
            lib().bgw_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        return int(lib().bgw_workspace_bytes(self._h))

    def pair_density_workspace(self, n, gw, ge, cv, cc) -> int:
        """Workspace bytes the next pair_density call with these arguments needs."""
        d = make_pair_desc(n, gw, ge, cv, cc)
        out = ctypes.c_size_t()
        _check(lib().bgw_pair_density_workspace(self._h, ctypes.byref(d), ctypes.byref(out)))
        return int(out.value)

    def chi0_workspace(self, qs, omega, precision: int = FP64, accumulate: bool = False, chis=None, axis="imag",
                       broadening: float = 0.0) -> int:
        """Workspace bytes the chi0 call with these arguments needs."""
        d, outs, keep = self._chi_desc(qs, omega, precision, accumulate, chis, False, axis, broadening)
        out = ctypes.c_size_t()
        _check(lib().bgw_chi0_workspace(self._h, ctypes.byref(d), ctypes.byref(out)))
        del keep
        return int(out.value)

    def eps_inv_workspace(self, ng: int, nw: int) -> int:
        out = ctypes.c_size_t()
        _check(lib().bgw_eps_inv_workspace(self._h, int(ng), int(nw), ctypes.byref(out)))
        return int(out.value)

    # ---------------------------------------------------------------- timing
    def set_timing(self, enable: bool = True):
        _check(lib().bgw_set_timing(self._h, 1 if enable else 0))

    def reset_timing(self):
        _check(lib().bgw_reset_timing(self._h))

    def timing(self) -> dict:
        """{kernel name: (total ms, launches)} accumulated since the last reset."""
        out = {}
        for i, name in enumerate(KERNELS):
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            _check(lib().bgw_get_timing(self._h, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    # ---------------------------------------------------------------- pair densities
    def pair_density(self, n, gw, ge, cv, cc, M=None):
        """M[t][G] (complex128, device) for t = (k*nv + v)*nc + c."""
        import torch
        assert cv.dtype == torch.complex128 and cc.dtype == torch.complex128
        assert cv.is_contiguous() and cc.is_contiguous()
        nk, nv, ngw = cv.shape
        nc = cc.shape[1]
        assert cc.shape == (nk, nc, ngw) and len(gw) == ngw
        ng = len(ge)
        if M is None:
            M = torch.empty((nk * nv * nc, ng), dtype=torch.complex128, device=cv.device)
        assert M.shape == (nk * nv * nc, ng) and M.is_contiguous() and M.dtype == torch.complex128
        d = make_pair_desc(n, gw, ge, cv, cc)
        _check(lib().bgw_pair_density(self._h, ctypes.byref(d), _dptr(M), _stream()))
        return M

    def pair_density_real(self, n, gw, ge, cv, cc, M=None):
        """Real flavor: real coefficients (float64 [nk][nv|nc][ngw]) -> real M[t][G] (float64)."""
        import torch
        assert cv.dtype == torch.float64 and cc.dtype == torch.float64
        assert cv.is_contiguous() and cc.is_contiguous()
        nk, nv, ngw = cv.shape
        nc = cc.shape[1]
        assert cc.shape == (nk, nc, ngw) and len(gw) == ngw
        ng = len(ge)
        if M is None:
            M = torch.empty((nk * nv * nc, ng), dtype=torch.float64, device=cv.device)
        assert M.shape == (nk * nv * nc, ng) and M.is_contiguous() and M.dtype == torch.float64
        d = make_pair_desc(n, gw, ge, cv, cc)
        _check(lib().bgw_pair_density_real(self._h, ctypes.byref(d), _dptr(M), _stream()))
        return M

    # ---------------------------------------------------------------- chi0
    def _chi_desc(self, qs: Sequence[dict], omega: Sequence[float], precision: int, accumulate: bool,
                  chis: Optional[List], use_graph: bool, axis="imag", broadening: float = 0.0, real=False):
        import torch
        dt = torch.float64 if real else torch.complex128
        om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1)
        arr = (ChiQ * len(qs))()
        outs = []
        keep = [om, arr]
        for i, q in enumerate(qs):
            M = q["M"]
            ng = int(M.shape[1])
            K = int(q["nk"]) * int(q["nv"]) * int(q["nc"])
            assert M.shape[0] == K and M.dtype == dt and M.is_contiguous()
            ev = q["ev"].contiguous()
            ec = q["ec"].contiguous()
            assert ev.dtype == torch.float64 and ec.dtype == torch.float64
            assert ev.numel() == q["nk"] * q["nv"] and ec.numel() == q["nk"] * q["nc"]
            chi = None if chis is None else chis[i]
            if chi is None:
                chi = torch.empty((om.size, ng, ng), dtype=dt, device=M.device)
            assert chi.shape == (om.size, ng, ng) and chi.is_contiguous() and chi.dtype == dt
            keep += [ev, ec]
            arr[i].ng = ng
            arr[i].nk, arr[i].nv, arr[i].nc = int(q["nk"]), int(q["nv"]), int(q["nc"])
            arr[i].M = _dptr(M)
            arr[i].ev = _dptr(ev)
            arr[i].ec = _dptr(ec)
            arr[i].head = int(q.get("head", -1))
            arr[i].prefactor = float(q["prefactor"])
            arr[i].chi = _dptr(chi)
            outs.append(chi)
        d = ChiDesc()
        d.nq = len(qs)
        d.q = arr
        d.nw = om.size
        d.omega = om.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.precision = int(precision)
        d.accumulate = 1 if accumulate else 0
        d.use_graph = 1 if use_graph else 0
        d.axis = _AXES[axis] if isinstance(axis, str) else int(axis)
        d.broadening = float(broadening)
        return d, outs, keep

    def chi0(self, qs: Sequence[dict], omega: Sequence[float], precision: int = FP64, accumulate: bool = False,
             chis: Optional[List] = None, use_graph: bool = False, axis="imag", broadening: float = 0.0):
        """qs: list of dicts {M, ev, ec, nk, nv, nc, head, prefactor} (device tensors); all q and all
        frequencies form one batch.  Returns the list of chi tensors [nw][ng][ng] (complex128).
        use_graph: capture the call into a HIP graph on first use of this exact descriptor and
        replay it afterwards (the tensors' addresses are part of the descriptor).
        axis: "imag" (omega = |omega| on the imaginary axis), "retarded" or "advanced" (omega = real
        frequencies E, broadening delta in eV)."""
        d, outs, keep = self._chi_desc(qs, omega, precision, accumulate, chis, use_graph, axis, broadening)
        _check(lib().bgw_chi0(self._h, ctypes.byref(d), _stream()))
        del keep
        return outs

    def chi0_real(self, qs: Sequence[dict], omega: Sequence[float], accumulate: bool = False,
                  chis: Optional[List] = None):
        """Real flavor: qs as for chi0 with real M (float64 [K][ng]); returns real chi [nw][ng][ng]."""
        d, outs, keep = self._chi_desc(qs, omega, FP64, accumulate, chis, False, real=True)
        _check(lib().bgw_chi0_real(self._h, ctypes.byref(d), _stream()))
        del keep
        return outs

    def chi0_real_workspace(self, qs: Sequence[dict], omega: Sequence[float]) -> int:
        d, outs, keep = self._chi_desc(qs, omega, FP64, False, None, False, real=True)
        out = ctypes.c_size_t()
        _check(lib().bgw_chi0_real_workspace(self._h, ctypes.byref(d), ctypes.byref(out)))
        del keep
        return int(out.value)

    def realify(self, c, e, tol: float, r=None):
        """Real flavor: real coefficients [nk][nb][ngw] (float64, device) from complex ones (complex128,
        device) with energies e (host [nk][nb], ascending per k): Gram-Schmidt over Re and Im of each
        group of degenerate states (energies within tol of their neighbour).  Returns (r, number of
        groups that were not real up to a unitary)."""
        import torch
        assert c.dtype == torch.complex128 and c.is_contiguous() and c.dim() == 3
        nk, nb, ngw = (int(x) for x in c.shape)
        e = np.ascontiguousarray(e, dtype=np.float64)
        assert e.shape == (nk, nb)
        if r is None:
            r = torch.empty((nk, nb, ngw), dtype=torch.float64, device=c.device)
        assert r.shape == (nk, nb, ngw) and r.dtype == torch.float64 and r.is_contiguous()
        nbad = torch.empty(1, dtype=torch.int32, device=c.device)
        _check(lib().bgw_realify(self._h, nk, nb, ngw, _dptr(c), e.ctypes.data, float(tol), _dptr(r), _dptr(nbad),
                                 _stream()))
        return r, int(nbad.cpu()[0])

    def realify_workspace(self, nk: int, nb: int, ngw: int, e, tol: float) -> int:
        e = np.ascontiguousarray(e, dtype=np.float64)
        out = ctypes.c_size_t()
        _check(lib().bgw_realify_workspace(self._h, nk, nb, ngw, e.ctypes.data, float(tol), ctypes.byref(out)))
        return int(out.value)

    def autotune(self, qs: Sequence[dict], omega: Sequence[float], precision: int = FP64,
                 chis: Optional[List] = None):
        """Time the chi-sum candidates for every size class in qs and keep the fastest
        (overwrites chis[i][0] of the timed q)."""
        d, outs, keep = self._chi_desc(qs, omega, precision, False, chis, False)
        _check(lib().bgw_autotune(self._h, ctypes.byref(d), _stream()))
        del keep
        return outs

    def tuned_config(self, precision: int, ng: int, K: int) -> dict:
        cfg = (ctypes.c_int * 4)()
        _check(lib().bgw_tuned_config(self._h, int(precision), int(ng), int(K), cfg))
        return {"tile": cfg[0], "items_per_cu": cfg[1], "split_nsplit": cfg[2], "tuned": bool(cfg[3])}

    # ---------------------------------------------------------------- eps^-1
    def eps_inv(self, vcoul, chi, epsinv=None, info=None, nsd=False):
        """epsilon^-1 for every frequency; returns (epsinv, info) device tensors.  nsd: chi is Hermitian
        negative semidefinite (zero or imaginary frequency), inverted without row interchanges
        (bgw_eps_inv_nsd; info -2 / -3 when that does not hold)."""
        import torch
        if chi.dim() == 2:
            chi = chi.unsqueeze(0)
        nw, ng, _ = chi.shape
        assert chi.dtype == torch.complex128 and chi.is_contiguous()
        assert vcoul.dtype == torch.float64 and vcoul.numel() == ng
        if epsinv is None:
            epsinv = torch.empty_like(chi)
        if info is None:
            info = torch.empty(nw, dtype=torch.int32, device=chi.device)
        fn = lib().bgw_eps_inv_nsd if nsd else lib().bgw_eps_inv
        _check(fn(self._h, ng, nw, _dptr(vcoul.contiguous()), _dptr(chi), _dptr(epsinv), _dptr(info), _stream()))
        return epsinv, info

    # ---------------------------------------------------------------- BSE exchange kernel
    def _kx_desc(self, M, v, head, prefactor, precision, kx):
        import torch
        K, ng = M.shape
        assert M.dtype == torch.complex128 and M.is_contiguous()
        assert v.dtype == torch.float64 and v.numel() == ng and v.is_contiguous()
        assert kx.shape == (K, K) and kx.dtype == torch.complex128 and kx.is_contiguous()
        return KxDesc(M=_dptr(M), K=K, ng=ng, head=int(head), v=_dptr(v), prefactor=float(prefactor),
                      precision=int(precision), pad=0, kx=_dptr(kx))

    def bse_kx(self, M, v, head=0, prefactor=1.0, precision=FP64, kx=None):
        """Kx[t][t'] = prefactor sum_{G != head} conj(M_t(G)) v(G) M_t'(G) (device complex128 [K][K])."""
        import torch
        if kx is None:
            kx = torch.empty((M.shape[0], M.shape[0]), dtype=torch.complex128, device=M.device)
        d = self._kx_desc(M, v, head, prefactor, precision, kx)
        _check(lib().bgw_bse_kx(self._h, ctypes.byref(d), _stream()))
        return kx

    def bse_kx_workspace(self, M, v, head=0, prefactor=1.0, precision=FP64, kx=None) -> int:
        import torch
        if kx is None:
            kx = torch.empty((1, 1), dtype=torch.complex128, device=M.device).expand(M.shape[0], M.shape[0])
            d = KxDesc(M=_dptr(M), K=M.shape[0], ng=M.shape[1], head=int(head), v=_dptr(v),
                       prefactor=float(prefactor), precision=int(precision), pad=0, kx=_dptr(kx))
        else:
            d = self._kx_desc(M, v, head, prefactor, precision, kx)
        out = ctypes.c_size_t()
        _check(lib().bgw_bse_kx_workspace(self._h, ctypes.byref(d), ctypes.byref(out)))
        return int(out.value)

    # ---------------------------------------------------------------- static self-energy
    def _sigma_desc(self, kind, M, v, epsinv, head, prefactor, precision, accumulate, sigma):
        import torch
        ni, no, ng = M.shape
        assert M.dtype == torch.complex128 and M.is_contiguous()
        assert v.dtype == torch.float64 and v.numel() == ng and v.is_contiguous()
        if epsinv is not None:
            assert epsinv.shape == (ng, ng) and epsinv.dtype == torch.complex128 and epsinv.is_contiguous()
        assert sigma.shape == (no, no) and sigma.dtype == torch.complex128 and sigma.is_contiguous()
        return SigmaDesc(M=_dptr(M), ninner=ni, nouter=no, ng=ng, kind=_SIGMA[kind], head=int(head),
                         precision=int(precision), v=_dptr(v), epsinv=_dptr(epsinv), prefactor=float(prefactor),
                         accumulate=1 if accumulate else 0, pad=0, sigma=_dptr(sigma))

    def sigma(self, kind, M, v, prefactor, epsinv=None, head=-1, precision=FP64, accumulate=False, sigma=None):
        """Self-energy matrix [nouter][nouter] of one q from M[ninner][nouter][ng]: kind "x", "sx" or "ch"."""
        import torch
        if sigma is None:
            sigma = torch.zeros((M.shape[1], M.shape[1]), dtype=torch.complex128, device=M.device)
        d = self._sigma_desc(kind, M, v, epsinv, head, prefactor, precision, accumulate, sigma)
        _check(lib().bgw_sigma(self._h, ctypes.byref(d), _stream()))
        return sigma

    def sigma_workspace(self, kind, M, v, prefactor, epsinv=None, head=-1, precision=FP64, sigma=None) -> int:
        import torch
        if sigma is None:
            sigma = torch.zeros((M.shape[1], M.shape[1]), dtype=torch.complex128, device=M.device)
        d = self._sigma_desc(kind, M, v, epsinv, head, prefactor, precision, False, sigma)
        out = ctypes.c_size_t()
        _check(lib().bgw_sigma_workspace(self._h, ctypes.byref(d), ctypes.byref(out)))
        return int(out.value)

    def eps_inv_noalloc(self, vcoul, chi, epsinv, info):
        """bgw_eps_inv_noalloc: epsilon^-1 into caller-owned epsinv and info, with the
        library's fixed device scratch (no allocation by the library)."""
        import torch
        nw, ng, _ = chi.shape
        assert chi.dtype == torch.complex128 and chi.is_contiguous()
        assert epsinv.shape == chi.shape and epsinv.dtype == chi.dtype and epsinv.is_contiguous()
        assert vcoul.dtype == torch.float64 and vcoul.numel() == ng and vcoul.is_contiguous()
        assert info.dtype == torch.int32 and info.numel() == nw
        _check(lib().bgw_eps_inv_noalloc(self._h, ng, nw, _dptr(vcoul), _dptr(chi), _dptr(epsinv), _dptr(info),
                                         _stream()))
        return epsinv, info
