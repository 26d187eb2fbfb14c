"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol the header declares, and host-side validation returns the documented
codes.  No compute call reaches the GPU here."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1111_4429_amd import bgw, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "bgw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bgw_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_header_symbol():
    L = bgw.lib()
    syms = header_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(bgw.EXPORTS) == syms
    assert L.bgw_version() >= 100


def test_library_has_no_oracle_dependency():
    """The product library must not link or embed the oracle."""
    data = open(bgw.LIB_PATH, "rb").read()
    assert b"orc_" not in data and b"liboracle" not in data


def test_pair_desc_validation_codes():
    gw = synth.gvector_list(300)   # max |m| = 4
    ge = synth.gvector_list(300)
    assert bgw.pair_desc_check(16, gw, ge) == bgw.BGW_OK
    # alias: need n > 2*4 + 4 = 12
    assert bgw.pair_desc_check(12, gw, ge) == bgw.BGW_ERR_ALIAS
    assert bgw.pair_desc_check((16, 16, 12), gw, ge) == bgw.BGW_ERR_ALIAS
    # unsupported grid lengths
    assert bgw.pair_desc_check(20, gw, ge) == bgw.BGW_ERR_UNSUPPORTED
    assert bgw.pair_desc_check(2048, gw, ge) == bgw.BGW_ERR_UNSUPPORTED
    assert bgw.pair_desc_check((0, 16, 16), gw, ge) == bgw.BGW_ERR_ARG
    # duplicate G and out-of-range component
    dup = np.concatenate([ge[:10], ge[3:4]])
    assert bgw.pair_desc_check(16, gw, dup) == bgw.BGW_ERR_SHAPE
    bad = gw.copy()
    bad[5] = (8, 0, 0)  # outside [-8, 8)
    assert bgw.pair_desc_check(16, bad, ge) == bgw.BGW_ERR_SHAPE
    ok = gw.copy()
    ok[5] = (-8, 0, 0)
    assert bgw.pair_desc_check(32, ok, ge) == bgw.BGW_OK
    # sizes
    assert bgw.pair_desc_check(16, gw, ge, nk=0) == bgw.BGW_ERR_ARG
    assert bgw.pair_desc_check(16, gw, ge, nv=-1) == bgw.BGW_ERR_ARG
    big = synth.gvector_list(12289)
    assert bgw.pair_desc_check(128, big, big) == bgw.BGW_ERR_UNSUPPORTED
    assert "12288" in bgw.lib().bgw_last_error().decode()
    # the message names the failing check
    dup = gw.copy()
    dup[7] = dup[3]
    assert bgw.pair_desc_check(16, dup, ge) == bgw.BGW_ERR_SHAPE
    assert "duplicate" in bgw.lib().bgw_last_error().decode()


def test_transform_box_is_minimal_alias_free():
    """The library transforms on the smallest 2^a 3^b box with
    b_i > 2 max|gw_i| + max|ge_i| (at most the caller's grid)."""
    for name, expect in (("tiny-static-16", 16), ("silicon-like-48", 24), ("supercell-96", 48),
                         ("imag-freq-64", 32)):
        wl = synth.WORKLOADS[name]
        gw, ge = synth.gvector_list(wl.ngw), synth.gvector_list(wl.ng)
        box = bgw.pair_transform_box(wl.n, gw, ge)
        assert box == (expect,) * 3, (name, box)
        need = 2 * np.abs(gw).max(axis=0) + np.abs(ge).max(axis=0)
        assert all(b > m for b, m in zip(box, need))


def test_null_arguments_rejected_without_gpu():
    L = bgw.lib()
    assert L.bgw_pair_desc_check(None) == bgw.BGW_ERR_ARG
    gw = synth.gvector_list(27)
    d = bgw.make_pair_desc(8, gw, gw, nk=1, nv=1, nc=1)
    # valid descriptor, null handle / output: argument error before any GPU work
    assert L.bgw_pair_density(None, ctypes.byref(d), None, None) == bgw.BGW_ERR_ARG
    assert L.bgw_chi0(None, None, None) == bgw.BGW_ERR_ARG
    assert L.bgw_eps_inv(None, 10, 1, None, None, None, None, None) == bgw.BGW_ERR_ARG
    assert L.bgw_eps_inv_nsd(None, 10, 1, None, None, None, None, None) == bgw.BGW_ERR_ARG
    assert L.bgw_eps_inv_nsd(None, 0, 1, 1, 1, 1, 1, None) == bgw.BGW_ERR_ARG
    assert L.bgw_destroy(None) == bgw.BGW_OK
    h = ctypes.c_void_p()
    assert L.bgw_create(None, 0) == bgw.BGW_ERR_ARG


def test_chi_descriptor_validation_without_gpu():
    L = bgw.lib()
    q = (bgw.ChiQ * 1)()
    q[0].ng, q[0].nk, q[0].nv, q[0].nc = 10, 1, 1, 1
    q[0].M = q[0].ev = q[0].ec = q[0].chi = 1
    q[0].head = 0
    om = (ctypes.c_double * 2)(0.0, -1.0)
    d = bgw.ChiDesc()
    d.nq, d.q, d.nw, d.omega, d.precision = 1, q, 2, om, 0
    assert L.bgw_chi0(None, ctypes.byref(d), None) == bgw.BGW_ERR_ARG  # omega < 0
    om[1] = 1.0
    d.precision = 7
    assert L.bgw_chi0(None, ctypes.byref(d), None) == bgw.BGW_ERR_ARG  # precision
    d.precision = 0
    q[0].head = 10
    assert L.bgw_chi0(None, ctypes.byref(d), None) == bgw.BGW_ERR_ARG  # head out of range


def test_vcoul_bulk_matches_oracle():
    s = synth.make_system(synth.WORKLOADS["tiny-static-16"])
    q = s["qs"][0]
    v = bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"])
    assert np.array_equal(v, oracle.vcoul(s["bmat"], q["q"], q["ge"])) or np.allclose(
        v, oracle.vcoul(s["bmat"], q["q"], q["ge"]), rtol=1e-15)
    with pytest.raises(bgw.BgwError) as e:
        bgw.vcoul_bulk(s["bmat"], np.zeros(3), q["ge"])
    assert e.value.code == bgw.BGW_ERR_SHAPE


def test_vcoul_bulk_non_cubic_cell():
    """The library's Coulomb helper on a skewed reciprocal basis, against the
    hand-computed values (q = (0.1, 0.2, -0.3); G = (1, -2, 3) gives
    |q+G|^2 = 37.1396 and G = 0 gives 0.4996 with rows of B as b_i)."""
    B = np.array([[1.0, 0.2, 0.0], [0.1, 1.5, 0.3], [0.0, -0.4, 2.0]])
    ge = np.array([[1, -2, 3], [0, 0, 0]], dtype=np.int32)
    v = bgw.vcoul_bulk(B, np.array([0.1, 0.2, -0.3]), ge)
    assert abs(v[0] - 4 * np.pi / 37.1396) <= 1e-14 * v[0]
    assert abs(v[1] - 4 * np.pi / 0.4996) <= 1e-14 * v[1]


def test_generator_is_deterministic():
    a = synth.make_system(synth.WORKLOADS["tiny-static-16"], seed=0)
    b = synth.make_system(synth.WORKLOADS["tiny-static-16"], seed=0)
    c = synth.make_system(synth.WORKLOADS["tiny-static-16"], seed=1)
    da = synth.digest([a["cc"], a["qs"][0]["cv"], a["ec"], a["qs"][0]["ev"]])
    db = synth.digest([b["cc"], b["qs"][0]["cv"], b["ec"], b["qs"][0]["ev"]])
    dc = synth.digest([c["cc"], c["qs"][0]["cv"], c["ec"], c["qs"][0]["ev"]])
    assert da == db != dc
    g = a["gw"]
    assert tuple(g[0]) == (0, 0, 0)
    mm = (g.astype(int) ** 2).sum(1)
    assert np.all(np.diff(mm) >= 0)
    e = a["ec"]
    assert np.all(np.diff(e, axis=1) >= 0) and e.min() >= 1 and e.max() <= 20


def test_next_row_entry_points_validate_without_gpu():
    """The self-energy, exchange-kernel and real-flavor entry points check their
    descriptors (then the handle) on the host and return the documented codes."""
    L = bgw.lib()
    # self-energy: a valid bare-exchange descriptor, then one field wrong at a time
    s = bgw.SigmaDesc()
    s.M = s.v = s.sigma = 1
    s.ninner, s.nouter, s.ng, s.kind, s.head, s.precision, s.prefactor = 2, 3, 10, bgw.SIGMA_X, 0, bgw.FP64, 1.0
    assert L.bgw_sigma(None, ctypes.byref(s), None) == bgw.BGW_ERR_ARG  # null handle
    s.kind = 5
    assert L.bgw_sigma(None, ctypes.byref(s), None) == bgw.BGW_ERR_ARG  # unknown kind
    s.kind, s.head = bgw.SIGMA_X, 10
    assert L.bgw_sigma(None, ctypes.byref(s), None) == bgw.BGW_ERR_ARG  # head out of range
    s.head, s.kind, s.epsinv = -1, bgw.SIGMA_SX, None
    assert L.bgw_sigma(None, ctypes.byref(s), None) == bgw.BGW_ERR_ARG  # screened kinds need eps^-1
    s.epsinv, s.precision = 1, bgw.SPLIT_BF16
    assert L.bgw_sigma(None, ctypes.byref(s), None) == bgw.BGW_ERR_UNSUPPORTED  # SX is FP64 only
    s.precision, s.ng = bgw.FP64, 13000
    assert L.bgw_sigma(None, ctypes.byref(s), None) == bgw.BGW_ERR_UNSUPPORTED  # ng above 12288
    # exchange kernel
    k = bgw.KxDesc()
    k.M = k.v = k.kx = 1
    k.K, k.ng, k.head, k.prefactor, k.precision = 4, 10, 0, 1.0, bgw.FP64
    assert L.bgw_bse_kx(None, ctypes.byref(k), None) == bgw.BGW_ERR_ARG  # null handle
    k.head = 10
    assert L.bgw_bse_kx(None, ctypes.byref(k), None) == bgw.BGW_ERR_ARG  # head out of range
    k.head, k.precision = -1, 7
    assert L.bgw_bse_kx(None, ctypes.byref(k), None) == bgw.BGW_ERR_ARG  # unknown precision
    k.precision, k.K = bgw.FP64, 0
    assert L.bgw_bse_kx(None, ctypes.byref(k), None) == bgw.BGW_ERR_UNSUPPORTED  # no pairs
    # real flavor: FP64, imaginary axis, no graph capture
    q = (bgw.ChiQ * 1)()
    q[0].ng, q[0].nk, q[0].nv, q[0].nc = 10, 1, 1, 1
    q[0].M = q[0].ev = q[0].ec = q[0].chi = 1
    q[0].head, q[0].prefactor = 0, 1.0
    om = (ctypes.c_double * 1)(0.0)
    d = bgw.ChiDesc()
    d.nq, d.q, d.nw, d.omega, d.precision = 1, q, 1, om, bgw.FP64
    assert L.bgw_chi0_real(None, ctypes.byref(d), None) == bgw.BGW_ERR_ARG  # null handle
    d.precision = bgw.SPLIT_BF16
    assert L.bgw_chi0_real(None, ctypes.byref(d), None) == bgw.BGW_ERR_UNSUPPORTED
    d.precision, d.axis, d.broadening = bgw.FP64, bgw.AXIS_RETARDED, 0.5
    assert L.bgw_chi0_real(None, ctypes.byref(d), None) == bgw.BGW_ERR_UNSUPPORTED
    d.axis, d.use_graph = bgw.AXIS_IMAG, 1
    assert L.bgw_chi0_real(None, ctypes.byref(d), None) == bgw.BGW_ERR_UNSUPPORTED
    gw = synth.gvector_list(27)
    pd = bgw.make_pair_desc(8, gw, gw, nk=1, nv=1, nc=1)
    assert L.bgw_pair_density_real(None, ctypes.byref(pd), None, None) == bgw.BGW_ERR_ARG
    # real coefficients from complex ones: energies, then group size, then the handle
    e = np.zeros((2, 40))
    e[0] = np.arange(40.0)
    e[1, :33] = 0.0
    e[1, 33:] = np.arange(1.0, 8.0)
    ep = e.ctypes.data
    assert L.bgw_realify(None, 2, 40, 50, 1, ep, 1e-6, 1, 1, None) == bgw.BGW_ERR_UNSUPPORTED  # group of 33
    e[1, 32] = 0.5
    assert L.bgw_realify(None, 2, 40, 50, 1, ep, 1e-6, 1, 1, None) == bgw.BGW_ERR_ARG  # null handle
    e[1, 32] = -0.5
    assert L.bgw_realify(None, 2, 40, 50, 1, ep, 1e-6, 1, 1, None) == bgw.BGW_ERR_ARG  # energies descend
    assert b"ascend" in L.bgw_last_error()
    e[1, 32] = 0.5
    assert L.bgw_realify(None, 2, 40, 50, 1, ep, -1.0, 1, 1, None) == bgw.BGW_ERR_ARG  # negative tol
    assert L.bgw_realify(None, 0, 40, 50, 1, ep, 1e-6, 1, 1, None) == bgw.BGW_ERR_ARG  # no k
    nbytes = ctypes.c_size_t()
    assert L.bgw_realify_workspace(None, 2, 40, 50, ep, 1e-6, ctypes.byref(nbytes)) == bgw.BGW_ERR_ARG


def test_bench_refuses_several_gpus():
    """One GPU only: --gpus above 1 ends with a message and a nonzero status."""
    import json
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_large_grids_transform_on_the_small_box(monkeypatch):
    """A caller grid above 128 is accepted while the alias-free box fits the
    transform kernels (at most 128 per axis); the box does not depend on the
    grid; a sphere whose box needs more, or the full-grid mode on such a grid,
    is refused."""
    gw = synth.gvector_list(300)
    ge = synth.gvector_list(300)
    assert bgw.pair_desc_check(256, gw, ge) == bgw.BGW_OK
    assert bgw.pair_desc_check((192, 256, 1024), gw, ge) == bgw.BGW_OK
    assert bgw.pair_transform_box(256, gw, ge) == bgw.pair_transform_box(16, gw, ge)
    far = np.array([[0, 0, 0], [43, 0, 0]], dtype=np.int32)  # 2*43 + 43 + 1 = 130 points needed along x
    assert bgw.pair_desc_check(256, far, far) == bgw.BGW_ERR_UNSUPPORTED
    assert "128" in bgw.lib().bgw_last_error().decode()
    monkeypatch.setenv("BGW_FFT_BOX", "full")
    assert bgw.pair_desc_check(256, gw, ge) == bgw.BGW_ERR_UNSUPPORTED
    assert bgw.pair_desc_check(64, gw, ge) == bgw.BGW_OK
