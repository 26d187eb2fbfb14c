#!/usr/bin/env python3
"""Benchmark of the chi0 / eps^-1 hot path on one MI355X.

One step = one pass of the whole path over the workload's q points: pair
densities by FFT for every q -> energy weights + chi-sum for all q and all
frequencies in one batched call -> epsilon and its inverse per q.  The
default workload is imaginary-frequency chi0 (64^3 grid, Ng = 4000,
K = 512,000 pairs, 32 frequencies, split-BF16 chi-sum, FP64 eps^-1): the
largest configuration whose steps fit a run of a few minutes on one GPU.
The other workloads run in their own precision; the uneven-q one streams
its 64 q through the GPU in batches whose pair densities fit
--m-budget-gb, one chi0 call per batch (--graph replays each batch's
captured graph, --autotune tunes every size class first).
Inputs are generated once (seeded, synthetic) and are resident in HBM before
the timed region; W untimed warm-up steps, then exactly K timed steps
bracketed by torch.cuda.synchronize().

Prints ONE JSON line.  `value` is the chi-sum algorithmic rate of the whole
step: sum over q of 4 Ng^2 K Nw flops / step time (TFLOP/s, FP64-equivalent).
Per-kernel times come from HIP events the library records on the launch
stream during the timed steps; the roofline entry is for the kernel that
dominates the step.  `cpu_baseline` times the oracle on a bounded sample of
the same workload and extrapolates linearly in pairs (and in Ng^3 for the
inversion when Ng is large).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2516.6
SPLIT_PRODUCTS = 10  # BF16 slice products per FP64-equivalent product in the split form


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="imag-freq-64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-pairs", type=int, default=6400,
                    help="pairs of q0 the oracle baseline computes (0: every pair, end to end)")
    ap.add_argument("--split-reps", type=int, default=2)
    ap.add_argument("--split-omegas", type=int, default=4,
                    help="frequencies of the split-vs-FP64 comparison (evenly spread subset; 0 = all)")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-full-grid", action="store_true")
    ap.add_argument("--q-subset", default="all",
                    help="uneven-q workloads: all, comma-separated q indices, or spreadN (N q spanning the Ng range)")
    ap.add_argument("--m-budget-gb", type=float, default=96.0,
                    help="device memory for the pair densities of one q batch; the q are streamed in batches")
    ap.add_argument("--autotune", action="store_true", help="run the autotuner on every q batch before the warm-up")
    ap.add_argument("--precision", choices=["fp64", "split"], default=None,
                    help="chi-sum precision of the step (default: the workload's)")
    ap.add_argument("--graph", action="store_true", help="chi0 through HIP-graph replay")
    ap.add_argument("--eps-path", choices=["nsd", "pivoted"], default="nsd",
                    help="epsilon^-1 without row interchanges (chi Hermitian negative semidefinite, as at zero and "
                         "imaginary frequency) or with partial pivoting")
    ap.add_argument("--no-graph-compare", action="store_true", help="skip the graph-vs-eager comparison")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (PMC byte-counter calibration)")
    return ap.parse_args()


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, src_files):
    """HBM bytes per launch measured by rocprofv3 PMC runs, if the committed
    record was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_digest") != source_digest(src_files):
        return None
    return rec


def cpu_baseline(s, pairs_sample: int, chi_flops_step: float):
    """The oracle on a bounded sample: M by convolution for a sample of pairs
    of the first q, chi of those pairs over all Ng x Ng entries and all
    frequencies, one inversion; extrapolated linearly in pairs and q (and in
    Ng^3 for inversions of Ng > 2000, timed on a 1500 x 1500 block)."""
    import oracle

    q = s["qs"][0]
    K = s["nk"] * s["nv"] * s["nc"]
    ng = q["ng"]
    nw = len(s["omega"])
    # keep the oracle's chi sample near 2e11 flops; pairs_sample <= 0: every pair (end to end)
    full = pairs_sample <= 0
    pairs_sample = K if full else int(max(16, min(pairs_sample, K, 2e11 / (8.0 * ng * ng * nw))))
    rng = np.random.default_rng(123)
    pairs = np.sort(rng.choice(K, size=pairs_sample, replace=False))
    t0 = time.perf_counter()
    Ms = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"], pairs=pairs)
    t_m = time.perf_counter() - t0
    w_all = oracle.weights(q["ev"], s["ec"], s["omega"])
    w = w_all[:, pairs]
    pf = 1.0 / (s["nk"] * s["vol"])
    t0 = time.perf_counter()
    chi_s = oracle.chi(Ms, w, pf)
    t_c = time.perf_counter() - t0
    v = oracle.vcoul(s["bmat"], q["q"], q["ge"])
    ni = min(ng, 1500) if ng > 2000 else ng
    t0 = time.perf_counter()
    oracle.eps_inv(v[:ni], np.ascontiguousarray(chi_s[:1, :ni, :ni]))
    t_i = (time.perf_counter() - t0) * (ng / ni) ** 3 * nw
    scale = K / pairs_sample
    nq = len(s["qs"])
    sum_ng2 = sum(float(x["ng"]) ** 2 for x in s["qs"])
    sum_ng3 = sum(float(x["ng"]) ** 3 for x in s["qs"])
    t_step = t_m * scale * nq + t_c * scale * sum_ng2 / (ng * ng) + t_i * sum_ng3 / ng ** 3
    return {
        "value": chi_flops_step / t_step / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": ("end to end: " if full and nq == 1 and ni == ng else "") + (
                   f"oracle on {pairs_sample} of {K} pairs of q0: M by convolution ({t_m:.2f} s) and chi over all "
                   f"{ng}x{ng} entries and {nw} frequencies ({t_c:.2f} s), extrapolated x{scale:.0f} and over "
                   f"{nq} q by Ng^2; inversions {t_i:.2f} s for q0"
                   + (f" (timed at {ni}x{ni}, scaled by Ng^3)" if ni != ng else "")
                   + f"; extrapolated step {t_step:.1f} s"),
        "cpu": _cpu_model(),
    }


def full_grid_pairs(torch, bgw, n, s, q, cv, cc, M, fft_bytes_nominal, reps=2):
    """Pair densities on the caller's full FFT grid (BGW_FFT_BOX=full) instead of
    the minimal alias-free box, for comparison: same M, more work."""
    os.environ["BGW_FFT_BOX"] = "full"
    try:
        h2 = bgw.Handle(0)
        ref = M.clone()
        h2.pair_density(n, s["gw"], q["ge"], cv, cc, M=M)
        torch.cuda.synchronize()
        diff = float(torch.linalg.vector_norm(M - ref) / torch.linalg.vector_norm(ref))
        h2.reset_timing()
        h2.set_timing(True)
        for _ in range(reps):
            h2.pair_density(n, s["gw"], q["ge"], cv, cc, M=M)
        torch.cuda.synchronize()
        tm = h2.timing()
        h2.close()
    finally:
        del os.environ["BGW_FFT_BOX"]
    band = tm["band"][0] / reps
    pair = (tm["pair"][0] + tm["pair_x"][0]) / reps
    return {"grid": f"{n}^3", "band_ms": band, "pair_fft_ms": pair,
            "pair_fft_GBs_algorithmic": fft_bytes_nominal / (pair * 1e-3) / 1e9,
            "rel_diff_vs_minimal_box": diff}


def split_vs_fp64(torch, h, bgw, ents, omega, chis64, reps):
    """Split-BF16 vs FP64 chi-sum over the same resident M (whole batched chi0
    calls, HIP events on the launch stream), with the relative Frobenius error
    of every split (q, omega) result against the FP64 one (worst reported)."""
    chissp = [torch.empty_like(c) for c in chis64]
    res = {}
    for name, prec, bufs in (("fp64", bgw.FP64, chis64), ("split", bgw.SPLIT_BF16, chissp)):
        h.chi0(ents, omega, precision=prec, chis=bufs)  # warm-up
        torch.cuda.synchronize()
        h.reset_timing()
        h.set_timing(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            h.chi0(ents, omega, precision=prec, chis=bufs)
        e1.record()
        torch.cuda.synchronize()
        h.set_timing(False)
        res[name] = (e0.elapsed_time(e1) / reps, h.timing())
    err = head_err = 0.0
    for c64, csp in zip(chis64, chissp):
        for iw in range(c64.shape[0]):
            a, b = csp[iw], c64[iw]
            err = max(err, float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)))
            head_err = max(head_err, float(torch.linalg.vector_norm(a[0] - b[0]) / torch.linalg.vector_norm(b[0])))
    nw = len(omega)
    flops = 0.0
    for e in ents:
        ng = int(e["M"].shape[1])
        K = int(e["M"].shape[0])
        flops += 4.0 * ng * ng * K * nw
    issued = SPLIT_PRODUCTS * flops  # BF16 MFMA flops of the split form (ten slice products)
    tsp = res["split"][1]
    herk_ms = tsp["split_herk"][0] / reps
    t64 = res["fp64"][0]
    tspl = res["split"][0]
    return {
        "fp64_chi_ms": t64,
        "split_chi_ms": tspl,
        "speedup": t64 / tspl,
        "rel_err_vs_fp64": err,
        "head_row_rel_err": head_err,
        "bar": 1e-9,
        "meets_bar": err <= 1e-9,
        "split_slice_ms": tsp["split_slice"][0] / reps,
        "split_herk_ms": herk_ms,
        "split_headwing_ms": tsp["headwing"][0] / reps,
        "split_finalize_ms": tsp["finalize"][0] / reps,
        "fp64_herk_ms": res["fp64"][1]["herk"][0] / reps,
        "split_chi_TFLOPs_fp64_equiv": flops / (tspl * 1e-3) / 1e12,
        "fp64_chi_TFLOPs": flops / (t64 * 1e-3) / 1e12,
        "split_herk_bf16_TFLOPs": issued / (herk_ms * 1e-3) / 1e12,
        "split_herk_frac_bf16_peak": issued / (herk_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
    }


def graph_vs_eager(torch, h, bgw, ents, omega, chis, precision, reps=3):
    """The same chi0 call launched directly and replayed from its HIP graph."""
    out = {}
    for name, g in (("eager_ms", False), ("graph_ms", True)):
        h.chi0(ents, omega, precision=precision, chis=chis, use_graph=g)  # warm-up / capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            h.chi0(ents, omega, precision=precision, chis=chis, use_graph=g)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) * 1e3 / reps
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_kx(args, wl):
    """Bethe-Salpeter exchange kernel: one step = pair densities of the K pairs
    -> Kx = pf sum_{G != 0} conj(M_t(G)) v(G) M_t'(G) (4 K^2 Ng flops, FP64 or
    split precision), timed like the chi0 steps; the split form against FP64."""
    import torch

    from paper_1111_4429_amd import bgw, synth

    dev = torch.device("cuda:0")
    print(f"[bench] generating {wl.name}", file=sys.stderr, flush=True)
    s = synth.make_system(wl)
    q = s["qs"][0]
    n, K, ng = s["n"], wl.npairs, q["ng"]
    pf = 1.0 / (s["nk"] * s["vol"])
    precision = bgw.SPLIT_BF16 if args.precision == "split" else bgw.FP64
    h = bgw.Handle(0)
    cc = torch.from_numpy(s["cc"]).to(dev)
    cv = torch.from_numpy(q["cv"]).to(dev)
    v = torch.from_numpy(bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"])).to(dev)
    M = torch.empty((K, ng), dtype=torch.complex128, device=dev)
    kx = torch.empty((K, K), dtype=torch.complex128, device=dev)

    def step(prec):
        h.pair_density(n, s["gw"], q["ge"], cv, cc, M=M)
        h.bse_kx(M, v, head=0, prefactor=pf, precision=prec, kx=kx)

    for _ in range(args.warmup):
        step(precision)
    torch.cuda.synchronize()
    h.reset_timing()
    h.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(precision)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    h.set_timing(False)
    tm = h.timing()
    ms_step = elapsed * 1e3 / args.steps
    flops = 4.0 * K * K * ng
    per_step = {k: tm[k][0] / args.steps for k in tm if tm[k][1]}
    launches = {k: tm[k][1] / args.steps for k in tm if tm[k][1]}
    key = "herk" if precision == bgw.FP64 else "split_herk"
    if precision == bgw.FP64:
        name, work, peak = "k_herk_f64 (Kx, 4 K^2 Ng)", flops, FP64_PEAK_TFLOPS
    else:
        name, work, peak = "k_chi_split (Kx, BF16 MFMA, 10 x 4 K^2 Ng)", SPLIT_PRODUCTS * flops, BF16_PEAK_TFLOPS
    nl = launches.get(key, 1)
    avg = per_step[key] / nl
    kx_tr = load_traffic(f"herk_{wl.name}", ["paper_1111_4429_amd/csrc/chi.hip", "paper_1111_4429_amd/csrc/common.h"])
    kx_traffic = kx_tr["bytes_per_launch"] if (kx_tr is not None and precision == bgw.FP64) else None
    ach = work / nl / (avg * 1e-3) / 1e12
    kx_ms = sum(per_step.get(k, 0) for k in ("weights", "herk", "finalize", "split_slice", "split_herk"))
    out = {
        "metric": "chi-sum TFLOP/s + pair-FFT GB/s; split vs FP64 speedup at rel err <=1e-9",
        "value": flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == bgw.FP64 else "bf16-split/f32-acc/f64-recombined",
        "data": "synthetic (seeded generator: orthonormal plane-wave coefficients, uniform band energies)",
        "config": {"workload": wl.name, "quantity": "Bethe-Salpeter exchange kernel Kx", "grid": f"{n}^3",
                   "ng": ng, "nv": wl.nv, "nc": wl.nc, "nk": wl.nk, "npairs": K,
                   "precision": "fp64" if precision == bgw.FP64 else "split"},
        "stages": {"pair_density_ms": per_step.get("band", 0) + per_step.get("pair", 0) + per_step.get("pair_x", 0),
                   "kx_ms": kx_ms, "kx_TFLOPs": flops / (kx_ms * 1e-3) / 1e12},
        "roofline": {"kernel": name, "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": kx_traffic, "algorithmic_per_launch": work / nl, "avg_launch_ms": avg,
                     "launches_per_step": nl},
        "split": None,
        "cpu_baseline": None,
    }
    if not args.no_split:
        res = {}
        k64 = None
        for nm, prec in (("fp64", bgw.FP64), ("split", bgw.SPLIT_BF16)):
            step(prec)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.split_reps):
                h.bse_kx(M, v, head=0, prefactor=pf, precision=prec, kx=kx)
            e1.record()
            torch.cuda.synchronize()
            res[nm] = e0.elapsed_time(e1) / args.split_reps
            if nm == "fp64":
                k64 = kx.clone()
        err = float(torch.linalg.vector_norm(kx - k64) / torch.linalg.vector_norm(k64))
        out["split"] = {"fp64_kx_ms": res["fp64"], "split_kx_ms": res["split"], "speedup": res["fp64"] / res["split"],
                        "rel_err_vs_fp64": err, "bar": 1e-9, "meets_bar": err <= 1e-9}
        del k64
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        import oracle

        Mh = M.cpu().numpy()
        rows = np.arange(0, K, max(1, K // 32))[:32]
        t0 = time.perf_counter()
        oracle.bse_kx(Mh, v.cpu().numpy(), 0, pf, rows=rows)
        t_kx = (time.perf_counter() - t0) * K / len(rows)
        rng = np.random.default_rng(123)
        pairs = np.sort(rng.choice(K, size=64, replace=False))
        t0 = time.perf_counter()
        oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"], pairs=pairs)
        t_m = (time.perf_counter() - t0) * K / len(pairs)
        out["cpu_baseline"] = {"value": flops / (t_kx + t_m) / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"oracle Kx rows {len(rows)} of {K} ({t_kx * len(rows) / K:.2f} s) and M by "
                                         f"convolution for 64 of {K} pairs, extrapolated linearly in rows and pairs: "
                                         f"{t_kx + t_m:.1f} s per step", "cpu": _cpu_model()}
    h.close()
    del M, kx, cv, cc, v
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def bench_sigma(args, wl, nouter=64):
    """Static self-energy of one q: one step = pair densities of all inner x
    outer states -> bare exchange (occupied inner states) -> screened exchange
    (occupied) -> Coulomb hole (all inner states), with a given eps^-1 (a
    generic dense stand-in: the step times the self-energy contractions)."""
    import torch

    from paper_1111_4429_amd import bgw, synth

    dev = torch.device("cuda:0")
    print(f"[bench] generating {wl.name}", file=sys.stderr, flush=True)
    s = synth.make_system(wl)
    q = s["qs"][0]
    n, ng, nocc = s["n"], q["ng"], wl.nv
    ninner = wl.nv + wl.nc
    pf = 1.0 / (s["nk"] * s["vol"])
    h = bgw.Handle(0)
    inner = torch.from_numpy(np.ascontiguousarray(np.concatenate([q["cv"], s["cc"]], axis=1))).to(dev)
    outer = torch.from_numpy(np.ascontiguousarray(s["cc"][:, :nouter])).to(dev)
    v = torch.from_numpy(bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"])).to(dev)
    rng = np.random.default_rng(0)
    W = torch.from_numpy(np.eye(ng) + 0.01 * (rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng)))).to(dev)
    Mflat = torch.empty((ninner * nouter, ng), dtype=torch.complex128, device=dev)
    M = Mflat.view(ninner, nouter, ng)
    occ = M[:nocc]
    sig = {k: torch.empty((nouter, nouter), dtype=torch.complex128, device=dev) for k in ("x", "sx", "ch")}

    def step():
        h.pair_density(n, s["gw"], q["ge"], inner, outer, M=Mflat)
        h.sigma("x", occ, v, pf, head=0, sigma=sig["x"])
        h.sigma("sx", occ, v, pf, epsinv=W, sigma=sig["sx"])
        h.sigma("ch", M, v, pf, epsinv=W, sigma=sig["ch"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    # CH alone, events on the launch stream: the dominant product W M
    e0.record()
    for _ in range(args.steps):
        h.sigma("ch", M, v, pf, epsinv=W, sigma=sig["ch"])
    e1.record()
    torch.cuda.synchronize()
    ch_ms = e0.elapsed_time(e1) / args.steps
    f_x = 4.0 * nouter * nouter * nocc * ng
    # HBM bytes of one Coulomb-hole call (all its kernels) from the committed PMC record
    ch_tr = load_traffic(f"sigma-ch_{wl.name}", ["paper_1111_4429_amd/csrc/chi.hip", "paper_1111_4429_amd/csrc/common.h"])
    f_w = lambda ni: 8.0 * ng * ng * ni * nouter + 8.0 * nouter * nouter * ni * ng
    flops = f_x + f_w(nocc) + f_w(ninner)
    out = {
        "metric": "chi-sum TFLOP/s + pair-FFT GB/s; split vs FP64 speedup at rel err <=1e-9",
        "value": flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator: orthonormal plane-wave coefficients, uniform band energies; "
                "eps^-1 a seeded dense stand-in)",
        "config": {"workload": wl.name, "quantity": "static self-energy (X, SX, CH sum form) of one q",
                   "grid": f"{n}^3", "ng": ng, "ninner": ninner, "nocc": nocc, "nouter": nouter},
        "stages": {"coulomb_hole_ms": ch_ms, "coulomb_hole_TFLOPs": f_w(ninner) / (ch_ms * 1e-3) / 1e12},
        "roofline": {"kernel": "k_gemm_phq (W M and the (i, G) contraction of the Coulomb hole)", "bound": "mfma",
                     "achieved": f_w(ninner) / (ch_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": f_w(ninner) / (ch_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "traffic": None if ch_tr is None else ch_tr["bytes_per_launch"],
                     "algorithmic_per_launch": f_w(ninner), "avg_launch_ms": ch_ms, "launches_per_step": 1,
                     "note": "per bgw_sigma call of the Coulomb hole (its two products, regrouping and finalize)"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        import oracle

        Mh, vh, Wh = M.cpu().numpy(), v.cpu().numpy(), W.cpu().numpy()
        sel = list(range(0, nouter, nouter // 4))[:4]
        t0 = time.perf_counter()
        oracle.sigma("ch", Mh[:, sel], vh, pf, einv=Wh)
        t_s = time.perf_counter() - t0
        t_ch = t_s * nouter / len(sel)  # the oracle's cost is linear in the outer states (ninner Ng^2 each)
        out["cpu_baseline"] = {"value": f_w(ninner) / t_ch / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"oracle Coulomb hole on {len(sel)} of {nouter} outer states "
                                         f"({t_s:.1f} s), extrapolated linearly in the outer states: "
                                         f"{t_ch:.0f} s per call", "cpu": _cpu_model()}
    h.close()
    del M, Mflat, occ, W, inner, outer, v, sig
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def bench_real(args, wl):
    """Real flavor (real coefficients): one step = real pair densities of every
    pair -> real symmetric chi-sum (FP64 MFMA, Ng^2 K flops per frequency: the
    half of the real product that symmetry leaves).  The complex FP64 chi-sum
    of the same M is timed beside it: both give the same chi."""
    import torch

    from paper_1111_4429_amd import bgw, synth

    dev = torch.device("cuda:0")
    print(f"[bench] generating {wl.name}", file=sys.stderr, flush=True)
    s = synth.make_system(wl)
    q = s["qs"][0]
    n, nk, nv, nc, ng = s["n"], s["nk"], s["nv"], s["nc"], q["ng"]
    K = nk * nv * nc
    omega = s["omega"]
    nw = len(omega)
    pf = 1.0 / (nk * s["vol"])
    h = bgw.Handle(0)
    cv = torch.from_numpy(q["cv"]).to(dev)
    cc = torch.from_numpy(s["cc"]).to(dev)
    ev = torch.from_numpy(q["ev"]).to(dev)
    ec = torch.from_numpy(s["ec"]).to(dev)
    M = torch.empty((K, ng), dtype=torch.float64, device=dev)
    chi = torch.empty((nw, ng, ng), dtype=torch.float64, device=dev)
    ent = dict(M=M, ev=ev, ec=ec, nk=nk, nv=nv, nc=nc, head=0, prefactor=pf)

    def step():
        h.pair_density_real(n, s["gw"], q["ge"], cv, cc, M=M)
        h.chi0_real([ent], omega, chis=[chi])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.reset_timing()
    h.set_timing(True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    h.set_timing(False)
    tm = h.timing()
    per_step = {k: tm[k][0] / args.steps for k in tm if tm[k][1]}
    launches = {k: tm[k][1] / args.steps for k in tm if tm[k][1]}
    flops = float(ng) * ng * K * nw
    sy_tr = load_traffic(f"syrk_{wl.name}", ["paper_1111_4429_amd/csrc/real.hip", "paper_1111_4429_amd/csrc/common.h"])
    chi_ms = sum(per_step.get(k, 0) for k in ("weights", "herk", "finalize"))
    syrk_ms = per_step["herk"] / launches["herk"]
    # the complex FP64 chi-sum of the same (real) M, cast to complex
    Mc = M.to(torch.complex128)
    chic = torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev)
    centry = [dict(ent, M=Mc)]
    h.chi0(centry, omega, chis=[chic])
    torch.cuda.synchronize()
    h.reset_timing()
    h.set_timing(True)
    for _ in range(args.steps):
        h.chi0(centry, omega, chis=[chic])
    torch.cuda.synchronize()
    h.set_timing(False)
    tc = h.timing()
    cplx_ms = sum(tc[k][0] for k in ("weights", "herk", "finalize") if tc[k][1]) / args.steps
    agree = float(torch.linalg.vector_norm(chi - chic.real) / torch.linalg.vector_norm(chic.real))
    del Mc, chic
    out = {
        "metric": "chi-sum TFLOP/s + pair-FFT GB/s; split vs FP64 speedup at rel err <=1e-9",
        "value": flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator: real orthonormal plane-wave coefficients, uniform band energies)",
        "config": {"workload": wl.name, "flavor": "real", "grid": f"{n}^3", "ng": ng, "nv": nv, "nc": nc,
                   "nk": nk, "npairs": K, "nw": nw,
                   "flops": "Ng^2 K per frequency (real symmetric rank-K update)"},
        "stages": {"pair_density_ms": per_step.get("band", 0) + per_step.get("pair", 0) + per_step.get("pair_x", 0),
                   "chi_ms": chi_ms, "syrk_ms": per_step["herk"],
                   "chi_sum_TFLOPs": flops / (chi_ms * 1e-3) / 1e12,
                   "complex_fp64_chi_ms_same_M": cplx_ms,
                   "real_vs_complex_chi_speedup": cplx_ms / chi_ms,
                   "real_vs_complex_chi_rel_diff": agree},
        "roofline": {"kernel": "k_syrk_f64 (real symmetric rank-K update)", "bound": "mfma",
                     "achieved": flops / launches["herk"] / (syrk_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s",
                     "frac": flops / launches["herk"] / (syrk_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "traffic": None if sy_tr is None else sy_tr["bytes_per_launch"],
                     "algorithmic_per_launch": flops / launches["herk"], "avg_launch_ms": syrk_ms,
                     "launches_per_step": launches["herk"]},
        "kernel_share": {k: per_step[k] / ms_step for k in per_step},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        import oracle

        sample = int(max(16, min(args.cpu_sample_pairs, K, 2e11 / (8.0 * ng * ng * nw))))
        pairs = np.sort(np.random.default_rng(123).choice(K, size=sample, replace=False))
        t0 = time.perf_counter()
        Ms = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"], pairs=pairs)
        t_m = time.perf_counter() - t0
        w = oracle.weights(q["ev"], s["ec"], omega)[:, pairs]
        t0 = time.perf_counter()
        oracle.chi(Ms, w, pf)
        t_c = time.perf_counter() - t0
        t_step = (t_m + t_c) * K / sample
        out["cpu_baseline"] = {"value": flops / t_step / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"oracle on {sample} of {K} pairs: M by convolution ({t_m:.2f} s) and chi "
                                         f"over all {ng}x{ng} entries ({t_c:.2f} s), extrapolated x{K / sample:.0f}: "
                                         f"{t_step:.0f} s per step", "cpu": _cpu_model()}
    h.close()
    del M, chi, cv, cc, ev, ec, ent
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


# Real-axis workload: the paper's full-frequency grid (uniform 0.5 eV up to
# 10 eV, then a spacing growing by 0.5 eV per point up to 40 eV: 30
# frequencies) and a broadening of 0.1 eV.
REALAXIS_GRID = (0.5, 10.0, 40.0, 0.5)
REALAXIS_DELTA = 0.1


def bench_realaxis(args, wl):
    """Real frequency axis: one step = pair densities of every pair -> the
    retarded chi^r(E) for every E of the grid (two Hermitian sums per E, of
    Re w and Im w) -> epsilon^-1(E) by elimination with partial pivoting
    (chi^r is not Hermitian).  value = FP64-equivalent chi flops (2 x 4 Ng^2 K
    per frequency) / step time."""
    import torch

    from paper_1111_4429_amd import bgw, synth

    dev = torch.device("cuda:0")
    print(f"[bench] generating {wl.name}", file=sys.stderr, flush=True)
    s = synth.make_system(wl)
    q = s["qs"][0]
    n, nk, nv, nc, ng = s["n"], s["nk"], s["nv"], s["nc"], q["ng"]
    K = nk * nv * nc
    E = bgw.ff_grid(*REALAXIS_GRID)
    nE = len(E)
    delta = REALAXIS_DELTA
    precision = bgw.FP64 if (args.precision or wl.precision) == "fp64" else bgw.SPLIT_BF16
    pf = 1.0 / (nk * s["vol"])
    h = bgw.Handle(0)
    cv = torch.from_numpy(q["cv"]).to(dev)
    cc = torch.from_numpy(s["cc"]).to(dev)
    ev = torch.from_numpy(q["ev"]).to(dev)
    ec = torch.from_numpy(s["ec"]).to(dev)
    v = torch.from_numpy(bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"])).to(dev)
    M = torch.empty((K, ng), dtype=torch.complex128, device=dev)
    chi = torch.empty((nE, ng, ng), dtype=torch.complex128, device=dev)
    einv = torch.empty_like(chi)
    info = torch.empty(nE, dtype=torch.int32, device=dev)
    ent = dict(M=M, ev=ev, ec=ec, nk=nk, nv=nv, nc=nc, head=0, prefactor=pf)

    def step():
        h.pair_density(n, s["gw"], q["ge"], cv, cc, M=M)
        h.chi0([ent], E, precision=precision, chis=[chi], axis="retarded", broadening=delta)
        h.eps_inv(v, chi, epsinv=einv, info=info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.reset_timing()
    h.set_timing(True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    h.set_timing(False)
    assert int(info.abs().max()) == 0
    tm = h.timing()
    per_step = {k: tm[k][0] / args.steps for k in tm if tm[k][1]}
    launches = {k: tm[k][1] / args.steps for k in tm if tm[k][1]}
    flops = 2.0 * 4.0 * ng * ng * K * nE
    gemm = "split_herk" if precision == bgw.SPLIT_BF16 else "herk"
    chi_ms = sum(per_step.get(k, 0) for k in ("weights", "herk", "finalize", "split_slice", "split_herk", "headwing"))
    nl = launches[gemm]
    g_ms = per_step[gemm] / nl
    work = SPLIT_PRODUCTS * flops if gemm == "split_herk" else flops
    peak = BF16_PEAK_TFLOPS if gemm == "split_herk" else FP64_PEAK_TFLOPS
    ach = work / nl / (g_ms * 1e-3) / 1e12
    src = "split.hip" if gemm == "split_herk" else "chi.hip"
    tr = load_traffic(f"{gemm}_{wl.name}", [f"paper_1111_4429_amd/csrc/{src}", "paper_1111_4429_amd/csrc/common.h"])
    # split against FP64 on four frequencies of the grid (both timed), and their difference
    pick = [0, nE // 3, 2 * nE // 3, nE - 1]
    cmp = {}
    if precision == bgw.SPLIT_BF16:
        E4 = E[pick]
        c64 = torch.empty((4, ng, ng), dtype=torch.complex128, device=dev)
        csp = torch.empty_like(c64)
        times = {}
        for name, prec, out in (("fp64", bgw.FP64, c64), ("split", bgw.SPLIT_BF16, csp)):
            h.chi0([ent], E4, precision=prec, chis=[out], axis="retarded", broadening=delta)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.split_reps):
                h.chi0([ent], E4, precision=prec, chis=[out], axis="retarded", broadening=delta)
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) * 1e3 / args.split_reps
        err = float(torch.linalg.vector_norm(csp - c64) / torch.linalg.vector_norm(c64))
        cmp = {"frequencies_eV": [float(x) for x in E4], "fp64_chi_ms": times["fp64"], "split_chi_ms": times["split"],
               "speedup": times["fp64"] / times["split"], "rel_err_vs_fp64": err, "bar": 1e-9, "meets_bar": err <= 1e-9}
        del c64, csp
    out = {
        "metric": "chi-sum TFLOP/s + pair-FFT GB/s; split vs FP64 speedup at rel err <=1e-9",
        "value": flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-split/f32-acc/f64-recombined" if gemm == "split_herk" else "f64",
        "data": "synthetic (seeded generator: orthonormal plane-wave coefficients, uniform band energies)",
        "config": {"workload": wl.name, "axis": "retarded", "grid": f"{n}^3", "ng": ng, "nv": nv, "nc": nc, "nk": nk,
                   "npairs": K, "nE": nE, "E_grid": list(REALAXIS_GRID), "broadening_eV": delta,
                   "precision": "split" if gemm == "split_herk" else "fp64",
                   "flops": "2 x 4 Ng^2 K per frequency (Hermitian sums of Re w and Im w)"},
        "stages": {"pair_density_ms": per_step.get("band", 0) + per_step.get("pair", 0) + per_step.get("pair_x", 0),
                   "chi_ms": chi_ms, "chi_sum_TFLOPs": flops / (chi_ms * 1e-3) / 1e12,
                   "eps_inv_ms": per_step.get("eps_build", 0) + per_step.get("invert", 0),
                   "eps_inv_TFLOPs": 8.0 * ng ** 3 * nE / (per_step.get("invert", float("nan")) * 1e-3) / 1e12,
                   "eps_inv_path": "pivoted"},
        "split": cmp or None,
        "roofline": {"kernel": "k_chi_split (BF16 MFMA, 10 x 4 Ng^2 K per weight vector)" if gemm == "split_herk"
                     else "k_herk_f64", "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": None if tr is None else tr["bytes_per_launch"],
                     "algorithmic_per_launch": work / nl, "avg_launch_ms": g_ms, "launches_per_step": nl},
        "kernel_share": {k: per_step[k] / ms_step for k in per_step},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        import oracle

        sample = int(max(16, min(args.cpu_sample_pairs, K, 2e11 / (16.0 * ng * ng * nE))))
        pairs = np.sort(np.random.default_rng(123).choice(K, size=sample, replace=False))
        t0 = time.perf_counter()
        Ms = oracle.pair_density(s["gw"], q["ge"], q["cv"], s["cc"], pairs=pairs)
        t_m = time.perf_counter() - t0
        w = oracle.weights_real(q["ev"], s["ec"], E, delta, "retarded")[:, pairs]
        t0 = time.perf_counter()
        chi_s = oracle.chi(Ms, w, pf)
        t_c = time.perf_counter() - t0
        vo = oracle.vcoul(s["bmat"], q["q"], q["ge"])
        t0 = time.perf_counter()
        oracle.eps_inv(vo, np.ascontiguousarray(chi_s[:1]))
        t_i = (time.perf_counter() - t0) * nE
        t_step = (t_m + t_c) * K / sample + t_i
        out["cpu_baseline"] = {"value": flops / t_step / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"oracle on {sample} of {K} pairs: M by convolution ({t_m:.2f} s) and chi^r "
                                         f"with complex weights over all {ng}x{ng} entries and {nE} frequencies "
                                         f"({t_c:.2f} s), extrapolated x{K / sample:.0f}; one inversion x {nE} "
                                         f"({t_i:.1f} s); {t_step:.0f} s per step", "cpu": _cpu_model()}
    h.close()
    del M, chi, einv, cv, cc, ev, ec, ent
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)

    import torch

    from paper_1111_4429_amd import bgw, synth

    assert torch.cuda.is_available(), "bench needs a HIP device"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # 4 GiB read + 4 GiB written by one copy kernel, 3 times
        nbytes = 4 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}))
        return
    wl = synth.WORKLOADS[args.workload]
    if wl.name.startswith("bse-kx"):
        bench_kx(args, wl)
        return
    if wl.name.startswith("sigma"):
        bench_sigma(args, wl)
        return
    if wl.flavor == "real":
        bench_real(args, wl)
        return
    if wl.name.startswith("realaxis"):
        bench_realaxis(args, wl)
        return
    q_subset = None
    if wl.nq > 1 and args.q_subset != "all":
        if args.q_subset.startswith("spread"):
            cnt = int(args.q_subset[len("spread"):] or 4)
            sizes = synth.uneven_q_sizes(wl)
            order = np.argsort(sizes, kind="stable")
            q_subset = sorted({int(order[round(i * (len(order) - 1) / max(1, cnt - 1))]) for i in range(cnt)})
        else:
            q_subset = [int(x) for x in args.q_subset.split(",")]
    print(f"[bench] generating {wl.name}" + (f" q {q_subset}" if q_subset else ""), file=sys.stderr, flush=True)
    s = synth.make_system(wl, q_subset=q_subset)
    prec_name = args.precision or wl.precision
    precision = bgw.FP64 if prec_name == "fp64" else bgw.SPLIT_BF16
    n, nk, nv, nc = s["n"], s["nk"], s["nv"], s["nc"]
    K = nk * nv * nc
    N = n ** 3
    nw = len(s["omega"])
    pf = 1.0 / (nk * s["vol"])
    omega = s["omega"]

    h = bgw.Handle(0)
    cc = torch.from_numpy(s["cc"]).to(dev)
    ec = torch.from_numpy(s["ec"]).to(dev)
    Q = []
    for q in s["qs"]:
        ng = q["ng"]
        Q.append(dict(q=q, ng=ng, cv=torch.from_numpy(q["cv"]).to(dev), ev=torch.from_numpy(q["ev"]).to(dev),
                      v=torch.from_numpy(bgw.vcoul_bulk(s["bmat"], q["q"], q["ge"])).to(dev),
                      chi=torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev),
                      einv=torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev),
                      info=torch.empty(nw, dtype=torch.int32, device=dev)))
    # q batches whose pair densities fit the M budget (one batch unless the q must be streamed);
    # each batch's M live in one pool, reused by the next batch
    budget = int(args.m_budget_gb * (1 << 30))
    batches, cur, cur_b = [], [], 0
    for i, x in enumerate(Q):
        b = K * x["ng"] * 16
        if cur and cur_b + b > budget:
            batches.append(cur)
            cur, cur_b = [], 0
        cur.append(i)
        cur_b += b
    batches.append(cur)
    pool_elems = max(sum(K * Q[i]["ng"] for i in bt) for bt in batches)
    pool = torch.empty(pool_elems, dtype=torch.complex128, device=dev)
    for bt in batches:
        off = 0
        for i in bt:
            Q[i]["M"] = pool[off:off + K * Q[i]["ng"]].view(K, Q[i]["ng"])
            off += K * Q[i]["ng"]
    bents = [[dict(M=Q[i]["M"], ev=Q[i]["ev"], ec=ec, nk=nk, nv=nv, nc=nc, head=0, prefactor=pf) for i in bt]
             for bt in batches]
    bchis = [[Q[i]["chi"] for i in bt] for bt in batches]
    ents, chis = bents[0], bchis[0]  # the first batch serves the split and graph comparisons
    if len(batches) > 1:
        print(f"[bench] {len(Q)} q streamed in {len(batches)} batches", file=sys.stderr, flush=True)

    def step(graph):
        for bt, be, bc in zip(batches, bents, bchis):
            for i in bt:
                x = Q[i]
                h.pair_density(n, s["gw"], x["q"]["ge"], x["cv"], cc, M=x["M"])
            h.chi0(be, omega, precision=precision, chis=bc, use_graph=graph)
            for i in bt:
                x = Q[i]
                h.eps_inv(x["v"], x["chi"], epsinv=x["einv"], info=x["info"], nsd=args.eps_path == "nsd")

    if args.autotune:
        print("[bench] autotune", file=sys.stderr, flush=True)
        for bt, be in zip(batches, bents):
            for i in bt:
                h.pair_density(n, s["gw"], Q[i]["q"]["ge"], Q[i]["cv"], cc, M=Q[i]["M"])
            h.autotune(be, omega, precision=precision)
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step(args.graph)
    torch.cuda.synchronize()
    if args.graph:
        # the timed steps replay graphs (no per-kernel events inside them): one eager
        # step first gives the per-kernel durations of the roofline entry
        h.reset_timing()
        h.set_timing(True)
        step(False)
        torch.cuda.synchronize()
        h.set_timing(False)
        tm = h.timing()
        tm_steps = 1
    h.reset_timing()
    h.set_timing(not args.graph)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(args.graph)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    h.set_timing(False)
    if not args.graph:
        tm = h.timing()
        tm_steps = args.steps
    for x in Q:
        assert int(x["info"].cpu().max()) == 0 and int(x["info"].cpu().min()) == 0

    ms_step = elapsed * 1e3 / args.steps
    q0 = Q[0]["q"]
    box = bgw.pair_transform_box(n, s["gw"], q0["ge"])
    boxes = [bgw.pair_transform_box(n, s["gw"], x["q"]["ge"]) for x in Q]
    ngs = [x["ng"] for x in Q]
    chi_flops = sum(4.0 * g * g * K * nw for g in ngs)
    # algorithmic bytes of the pair transform on the box actually transformed
    fft_bytes = sum(K * 16.0 * (b[0] * b[1] * b[2] + g) for b, g in zip(boxes, ngs))
    fft_bytes_nominal = sum(K * 16.0 * (N + g) for g in ngs)
    lu_flops = sum(8.0 * g ** 3 * nw for g in ngs)

    per_step = {k: tm[k][0] / tm_steps for k in tm if tm[k][1]}
    launches = {k: tm[k][1] / tm_steps for k in tm if tm[k][1]}
    pair_t = per_step.get("pair", 0) + per_step.get("pair_x", 0)
    herk_key = "herk" if precision == bgw.FP64 else "split_herk"
    chi_ms = sum(per_step.get(k, 0) for k in ("weights", "herk", "finalize", "split_slice", "split_herk",
                                               "headwing"))
    stages = {
        "pair_density_ms": per_step.get("band", 0) + pair_t,
        "band_ms": per_step.get("band", 0),
        "pair_fft_ms": per_step.get("pair", 0),
        "pair_x_ms": per_step.get("pair_x", 0),
        "chi_ms": chi_ms,
        "herk_ms": per_step.get(herk_key, 0),
        "eps_inv_ms": per_step.get("eps_build", 0) + per_step.get("invert", 0),
        "chi_sum_TFLOPs": chi_flops / (chi_ms * 1e-3) / 1e12,
        "pair_fft_GBs_algorithmic": fft_bytes / (pair_t * 1e-3) / 1e9,
        "pair_fft_nominal_TFLOPs": sum(5.0 * b[0] * b[1] * b[2] * np.log2(b[0] * b[1] * b[2]) * K for b in boxes)
        / (pair_t * 1e-3) / 1e12,
        "eps_inv_TFLOPs": lu_flops / (per_step.get("invert", float("nan")) * 1e-3) / 1e12,
        "eps_inv_path": args.eps_path,
    }
    ptr = load_traffic(f"pair_{wl.name}", ["paper_1111_4429_amd/csrc/fft2.hip", "paper_1111_4429_amd/csrc/common.h"])
    if ptr is not None and len(Q) == 1 and pair_t > 0:
        # HBM bytes of one pair-density call counted by rocprofv3 (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
        stages["pair_fft_GBs_counters"] = ptr["pair_bytes_per_step"] / (pair_t * 1e-3) / 1e9
        stages["pair_fft_counters_source"] = ptr["profile"]
    if precision == bgw.FP64:
        stages["chi_sum_frac_fp64_peak"] = chi_flops / (per_step["herk"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
    kernel_share = {k: per_step[k] / ms_step for k in per_step}
    # algorithmic work per step of each timed kernel group
    t_bytes = 0.0
    for x, b in zip(Q, boxes):
        rey = int(np.abs(x["q"]["ge"][:, 1]).max())
        rez = int(np.abs(x["q"]["ge"][:, 2]).max())
        t_bytes += K * 16.0 * b[0] * (2 * rey + 1) * (2 * rez + 1)
    box_bytes = sum(16.0 * b[0] * b[1] * b[2] for b in boxes)
    split_bf16 = SPLIT_PRODUCTS * chi_flops  # BF16 MFMA flops of the split form: ten products of 4 Ng^2 K
    work = {
        "pair": ("k_pair_yz (product + z/y FFT)", "hbm", K * box_bytes + t_bytes, "GB/s", HBM_PEAK_GBS),
        "pair_x": ("k_pair_x (x transform + sphere gather)", "hbm", t_bytes + K * 16.0 * sum(ngs), "GB/s",
                   HBM_PEAK_GBS),
        "band": ("k_band_to_real3", "hbm", (nk * (nv + nc)) * box_bytes, "GB/s", HBM_PEAK_GBS),
        "herk": ("k_herk_f64", "mfma", chi_flops, "TFLOP/s", FP64_PEAK_TFLOPS),
        "split_herk": ("k_chi_split (BF16 MFMA, 10 x 4 Ng^2 K per frequency)", "mfma", split_bf16, "TFLOP/s",
                       BF16_PEAK_TFLOPS),
        "invert": ("Gauss-Jordan inversion (k_gje_* or k_nsd_*)", "mfma", lu_flops, "TFLOP/s", FP64_PEAK_TFLOPS),
    }
    dominant = max(work, key=lambda k: per_step.get(k, 0))
    name, bound, per_step_work, unit, peak = work[dominant]
    nl = launches.get(dominant, 1)
    avg_ms = per_step[dominant] / nl
    per_launch = per_step_work / nl
    ach = per_launch / (avg_ms * 1e-3) / (1e9 if unit == "GB/s" else 1e12)
    src = {"pair": ["paper_1111_4429_amd/csrc/fft2.hip", "paper_1111_4429_amd/csrc/common.h"],
           "pair_x": ["paper_1111_4429_amd/csrc/fft2.hip", "paper_1111_4429_amd/csrc/common.h"],
           "band": ["paper_1111_4429_amd/csrc/fft2.hip", "paper_1111_4429_amd/csrc/common.h"],
           "herk": ["paper_1111_4429_amd/csrc/chi.hip", "paper_1111_4429_amd/csrc/common.h"],
           "split_herk": ["paper_1111_4429_amd/csrc/split.hip", "paper_1111_4429_amd/csrc/common.h"],
           "invert": ["paper_1111_4429_amd/csrc/eps.hip", "paper_1111_4429_amd/csrc/common.h"]}[dominant]
    tr = load_traffic(f"{dominant}_{wl.name}", src)
    roof = {"kernel": name, "bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "traffic": None if tr is None else tr["bytes_per_launch"],
            "algorithmic_per_launch": per_launch, "avg_launch_ms": avg_ms, "launches_per_step": nl}
    if tr is not None:
        roof["traffic_source"] = tr.get("profile")

    out = {
        "metric": "chi-sum TFLOP/s + pair-FFT GB/s; split vs FP64 speedup at rel err <=1e-9",
        "value": chi_flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == bgw.FP64 else "bf16-split/f32-acc/f64-recombined",
        "data": "synthetic (seeded generator: orthonormal plane-wave coefficients, uniform band energies)",
        "config": {"workload": wl.name, "grid": f"{n}^3", "transform_box": "x".join(map(str, box)),
                   "ng": ngs[0] if len(ngs) == 1 else ngs, "ngw": len(s["gw"]), "nv": nv, "nc": nc, "nk": nk,
                   "npairs": K, "nw": nw, "nq": len(Q), "precision": prec_name,
                   "q": [list(map(float, x["q"]["q"])) for x in Q] if len(Q) > 1 else list(map(float, q0["q"])),
                   "q_index": [int(x["q"]["iq"]) for x in Q] if len(Q) > 1 else 0, "graph": bool(args.graph)},
        "stages": stages,
        "kernel_share": kernel_share,
        "roofline": roof,
        "split": None,
        "cpu_baseline": None,
    }
    if not args.no_full_grid and len(Q) == 1 and tuple(box) != (n, n, n):
        x = Q[0]
        out["full_grid_pair_density"] = full_grid_pairs(torch, bgw, n, s, x["q"], x["cv"], cc, x["M"],
                                                        fft_bytes_nominal)
    if not args.no_split:
        print("[bench] split vs fp64", file=sys.stderr, flush=True)
        sub = omega
        if 0 < args.split_omegas < nw:
            sub = omega[np.unique(np.round(np.linspace(0, nw - 1, args.split_omegas)).astype(int))]
        out["split"] = split_vs_fp64(torch, h, bgw, ents, sub,
                                     [torch.empty((len(sub),) + tuple(c.shape[1:]), dtype=c.dtype, device=c.device)
                                      for c in chis], args.split_reps)
        out["split"]["omegas"] = [float(x) for x in sub]
    if (len(Q) > 1 or nw > 1) and not args.no_graph_compare:
        print("[bench] graph vs eager", file=sys.stderr, flush=True)
        out["batch_graph"] = graph_vs_eager(torch, h, bgw, ents, omega, chis, precision,
                                            reps=1 if chi_ms > 1000.0 else 3)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_sample_pairs, chi_flops)
    h.close()
    # release the device memory before the interpreter's own teardown
    x = None
    del Q, bents, bchis, ents, chis, pool, cc, ec
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
