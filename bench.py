#!/usr/bin/env python
"""Benchmark of the ParO hot path on one MI355X.

A step is one ParO outer iteration (Algorithm 1: 160 independent shifted
source problems solved by 20 Teter-preconditioned CG steps each, H applied
to the 160 solutions, Rayleigh-Ritz, residuals and the next shift) on the
34,265-plane-wave cell: a = 20 bohr cubic, E_cut = 20 Ha, 96^3 FFT grid,
32 Gaussian pseudo-atoms with s + 3p Kleinman-Bylander projectors (128),
N = 128 orbitals plus 32 buffer orbitals, FP64 (complex128) throughout.
Inputs are seeded synthetic cells (see synth/), resident in HBM before
the timed region.

Prints one JSON line.  value = ParO outer iterations per second in plain
FP64; also H-psi band-applies per second, the live HIP-event timing of the
dominant kernel against its roofline, the time to a 1e-8 Ha eigenvalue error
from the random trial block, and the CPU oracle's rate on the host cores.
"mixed" holds the same measurements for the batched mixed-precision path
(FP32 source problems, FP64 H U and Rayleigh-Ritz).  Also: the time to
1e-8 Ha of MParO I (Algorithm 2) with 10 PCG steps, in FP64 and mixed; the
density of the 160-band block; the uneven 24-cell batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "ParO iters/s & Hψ applies/s, plain FP64 vs batched mixed, at 1e-8 Ha eig err"
# HBM bytes per plane-kernel launch from the committed counter summary; it
# counts only while the kernel sources hash to the value recorded there.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_plane_96_c1_hbm_traffic.txt")
DENSITY_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_plane_density_96_c1_hbm_traffic.txt")
F32_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_plane_96_f32_c1_hbm_traffic.txt")
# the sources of the 96-point plane and density kernels (the traffic summaries
# hold their SHA-256; a summary taken on other sources reads as null)
PLANE_SOURCES = ["paper_1702_04045_amd/csrc/apply.hip", "paper_1702_04045_amd/csrc/fft_device.h"]
COPY_BYTES = 1 << 30         # bytes read (and written) by the calibration copy
PEAK_FP64_VALU = 78.6e12     # MI355X FP64 vector, flop/s
PEAK_FP32_VALU = 157.3e12    # MI355X FP32 vector, flop/s
PEAK_HBM = 8.0e12            # bytes/s
PEAK_BF16_MFMA = 2.5e15      # MI355X dense BF16 matrix cores, flop/s
# stride of the event-timed plane launches in the timed outer iterations:
# each event pair orders the stream (about 5.6 us of idle per pair), so only
# every fourth launch is bracketed
PLANE_SAMPLE = 4
# the plane-stage schedules at 96 points (paro_plan_set_schedule)
PLANE_SCHEDULES = {0: "two bands' columns in LDS", 1: "four lanes per line",
                   2: "compressed columns, two work-groups per CU"}


def fft_flops(n):
    return 5.0 * n * np.log2(n)


def plane_flops(N, ncol):
    """Algorithmic flops of one z-plane of one band: inverse and forward
    transforms along n2 for the ncol populated n1 columns and along n1 for
    all N rows (5 N log2 N each), plus the real potential multiply (2 per
    complex point)."""
    return (2 * ncol + 2 * N) * fft_flops(N) + 2.0 * N * N


def density_plane_flops(N, ncol):
    """Algorithmic flops of one z-plane of one band in the density: inverse
    transforms along n2 for the ncol populated columns and along n1 for all
    N rows, then w |psi|^2 accumulated (4 per point)."""
    return (ncol + N) * fft_flops(N) + 4.0 * N * N


def kato_temple_bound(eps, res, n):
    """Certified bound on max_i<n |eps_i - lambda_i| from Ritz values eps
    (ascending) and residual norms res = |H psi_i - eps_i psi_i|.

    Ritz values are upper bounds, lambda_i <= eps_i.  The Kato-Temple
    inequality gives eps_i - lambda_i <= res_i^2 / (b_i - eps_i) when no
    eigenvalue other than lambda_i lies in (a_i, b_i); b_i = eps_{i+1} -
    res_{i+1} bounds lambda_{i+1} from below and a_i = eps_{i-1} + res_{i-1}
    bounds lambda_{i-1} from above, so the gap taken is min(b_i - eps_i,
    eps_i - a_i).  Where that gap is not positive only the residual bound
    |eps_i - lambda_i| <= res_i remains."""
    out = 0.0
    for i in range(n):
        gap = np.inf
        if i + 1 < len(eps):
            gap = min(gap, (eps[i + 1] - res[i + 1]) - eps[i])
        if i > 0:
            gap = min(gap, eps[i] - (eps[i - 1] + res[i - 1]))
        b = res[i] if not gap > 0 else min(res[i], res[i] ** 2 / gap)
        out = max(out, b)
    return out


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def hpsi_work(N, nst, ncol, ng, nproj, bands_per_launch):
    """Algorithmic work of one band-apply of H (FP64).

    Local part (sphere -> sticks -> planes and back): inverse and forward
    3-D transforms pruned to the data that is not identically zero --
    5 N log2 N flops per line over nst z-sticks, ncol populated n2 columns
    per plane and N rows per plane -- plus the real potential multiply
    (2 flops per grid point) and the kinetic epilogue (4 flops per plane
    wave).  Bytes: psi read and H psi written (32 n_g), plus the potential
    (8 N^3) shared by the bands_per_launch bands of a launch.  Nonlocal
    part: P = B^H psi and B (D P), 2 x 8 n_g n_proj flops on the matrix cores."""
    lines = nst + N * ncol + N * N
    local = 2 * lines * fft_flops(N) + 2.0 * N ** 3 + 4.0 * ng
    nl = 16.0 * ng * nproj
    byts = 32.0 * ng + 8.0 * N ** 3 / bands_per_launch
    return local, nl, byts


def plane_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in PLANE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch from a counter summary, or None when the summary
    is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("plane_sources_sha256") != plane_sources_sha256():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device copy of COPY_BYTES, for scaling the FETCH_SIZE and
    WRITE_SIZE counters to bytes."""
    import torch
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": 3}))


def traffic_pass(seed):
    """Only the FP64 and FP32 H applies and the density calls of the 160-band
    block on the 34,265-plane-wave cell (no Rayleigh-Ritz): the run the plane
    kernels' HBM counters are read from."""
    import torch
    import paper_1702_04045_amd as P
    dev = torch.device("cuda:0")
    spec = synth.WORKLOADS["c1"]
    cell = synth.make_cell(spec, seed)
    v = synth.vloc_on_grid(cell["cell"], cell["grid"], cell["positions"], cell["depths"], cell["widths"])
    pl = P.Plan(cell["cell"], cell["ecut"], v, cell["projectors"], device=dev)
    x = torch.from_numpy(synth.trial_block(pl.ng, spec.n_carried, seed)).to(dev)
    w = torch.ones(spec.n_carried, dtype=torch.float64, device=dev)
    x32 = x.to(torch.complex64)
    for _ in range(3):
        pl.apply_h(x)
    for _ in range(3):
        pl.apply_h_f32(x32)
    for _ in range(3):
        pl.density(x, w)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_pass": {"bands": spec.n_carried, "applies": 3, "fp32_applies": 3, "density_calls": 3}}))


def cpu_baseline(spec, cell, v, x_trial, sample_bands=64):
    """The CPU oracle's outer-iteration time, extrapolated from a bounded sample."""
    import oracle
    h = oracle.Hamiltonian(cell["cell"], cell["ecut"], v, cell["projectors"])
    nb = spec.n_carried
    nbs = min(sample_bands, nb)
    threads = min(oracle.num_threads(), nbs)
    sig = h.shift_bound()
    xs = x_trial[:nbs]
    t0 = time.perf_counter()
    hx = h.apply(xs)
    t_apply = time.perf_counter() - t0
    eps = np.einsum("bg,bg->b", xs.conj(), hx).real / np.einsum("bg,bg->b", xs.conj(), xs).real
    t0 = time.perf_counter()
    h.pcg(xs, hx, eps, np.full(nbs, sig), spec.n_cg)
    t_pcg = time.perf_counter() - t0
    # Rayleigh-Ritz on the full 160-band block (the cost does not depend on the vectors)
    t0 = time.perf_counter()
    W = np.concatenate([hx, hx[np.arange(nb - nbs) % nbs]], axis=0)
    oracle.rayleigh_ritz(x_trial, W, nb)
    t_rr = time.perf_counter() - t0
    t_outer = (t_pcg + t_apply) * (nb / nbs) + t_rr
    return {"value": 1.0 / t_outer, "unit": "ParO outer iterations/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "compiler_flags": " ".join(["gcc", *oracle.CFLAGS]),
            "sample": (f"PCG ({spec.n_cg} steps) and one H apply on {nbs} of {nb} bands, scaled x{nb / nbs:g}, "
                       f"plus Rayleigh-Ritz on all {nb} bands; measured {t_pcg + t_apply + t_rr:.1f} s"),
            "seconds_per_outer_iteration": t_outer}


def batched_cells(args, P, torch, n_outer=5, n_cg=10, n_streams=8, reps=3):
    """The uneven 24-cell workload: n_outer ParO outer iterations (adaptive
    shift, initial Rayleigh-Ritz) of every cell from its trial block, once
    cell after cell with paro_iterate and once with paro_iterate_batch over
    n_streams streams, in FP64 and in mixed precision; best of reps, wall
    time between device synchronisations."""
    specs = synth.batch_specs(args.seed)
    plans, xs = [], []
    for i, sp in enumerate(specs):
        c = synth.make_cell(sp, i)
        v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
        pl = P.Plan(c["cell"], c["ecut"], v, c["projectors"])
        plans.append(pl)
        xs.append(torch.from_numpy(synth.trial_block(pl.ng, sp.n_bands, i)).cuda())
    sig = [pl.shift_lower_bound() for pl in plans]
    streams = [torch.cuda.Stream() for _ in range(n_streams)]

    prec = [P.PREC_FP64]

    def sequential():
        for pl, x, s in zip(plans, xs, sig):
            pl.iterate(x.clone(), n_outer, n_cg, s, shift_mode=P.SHIFT_ADAPTIVE, stats=False, precision=prec[0])

    def batch():
        P.iterate_batch(plans, [x.clone() for x in xs], n_outer, n_cg, sig, shift_mode=P.SHIFT_ADAPTIVE,
                        streams=streams, precision=prec[0])

    def best(f):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return min(ts)

    t_seq, t_bat = best(sequential), best(batch)
    prec[0] = P.PREC_MIXED
    m_seq, m_bat = best(sequential), best(batch)
    # fixed shift (no host decisions): the batch eager and as a captured graph, continuing
    # from the initial Rayleigh-Ritz; every repetition does the same work
    init = P.iterate_batch(plans, [x.clone() for x in xs], 0, n_cg, sig, initial_rr=True)
    st_e = [[o[k].clone() for o in init] for k in ("psi", "hpsi", "eps")]
    st_g = [[o[k].clone() for o in init] for k in ("psi", "hpsi", "eps")]

    def eager_fixed():
        P.iterate_batch(plans, st_e[0], n_outer, n_cg, sig, initial_rr=False, hpsis=st_e[1], epss=st_e[2])

    graph = P.capture_batch(plans, st_g[0], st_g[1], st_g[2], n_outer, n_cg, sig)
    f_eager, f_graph = best(eager_fixed), best(graph.replay)
    del graph
    # the plane stage's schedule and bands per work-group tuned per cell, then the same runs
    t0 = time.perf_counter()
    tuned = [pl.autotune(x.shape[0], force=True) for pl, x in zip(plans, xs)]
    t_tune = time.perf_counter() - t0
    prec[0] = P.PREC_FP64
    a_seq, a_bat = best(sequential), best(batch)
    prec[0] = P.PREC_MIXED
    am_seq, am_bat = best(sequential), best(batch)
    choices = {}
    for sp, r in zip(specs, tuned):
        key = f"{sp.grid}: schedule {r['schedule'][0]}/{r['schedule'][1]}, bands {r['bands'][0]}/{r['bands'][1]}"
        choices[key] = choices.get(key, 0) + 1
    applies = sum(x.shape[0] for x in xs) * (n_cg + 1) * n_outer
    return {"cells": len(specs), "grids": sorted({sp.grid for sp in specs}),
            "bands": [sp.n_bands for sp in specs], "plane_waves": [pl.ng for pl in plans],
            "projectors": [pl.n_proj for pl in plans], "outer_iterations_per_cell": n_outer, "pcg_steps": n_cg,
            "streams": n_streams, "seconds": t_bat, "cell_iterations_per_s": len(specs) * n_outer / t_bat,
            "band_applies_per_s": applies / t_bat, "sequential_seconds": t_seq,
            "speedup_vs_sequential": t_seq / t_bat, "dtype": "f64",
            "mixed": {"seconds": m_bat, "cell_iterations_per_s": len(specs) * n_outer / m_bat,
                      "sequential_seconds": m_seq, "speedup_vs_sequential": m_seq / m_bat,
                      "speedup_vs_fp64_batch": t_bat / m_bat,
                      "dtype": "f32 source problems, f64 H U and Rayleigh-Ritz"},
            "fixed_shift_graph": {"eager_seconds": f_eager, "graph_replay_seconds": f_graph,
                                  "speedup": f_eager / f_graph,
                                  "note": "fixed shift, no initial Rayleigh-Ritz: the batch captured once and replayed"},
            "autotuned": {"tune_seconds": t_tune, "seconds": a_bat, "sequential_seconds": a_seq,
                          "speedup_vs_sequential": a_seq / a_bat, "speedup_vs_untuned_batch": t_bat / a_bat,
                          "mixed_seconds": am_bat, "mixed_sequential_seconds": am_seq,
                          "mixed_speedup_vs_untuned_batch": m_bat / am_bat,
                          "cell_iterations_per_s": len(specs) * n_outer / a_bat,
                          "choices (grid: FP64/FP32)": choices,
                          "note": "paro_plan_autotune per cell: plane-stage line schedule and bands per work-group"}}


def at_scale(args, P, torch, steps=3, tta=False, tta_seconds=600.0):
    """The 161k-plane-wave cell (a = 30 bohr, E_cut = 25 Ha, 160^3 grid, 128
    atoms with 512 projectors, 512 + 128 bands, 20 PCG steps, adaptive shift):
    outer iterations per second in FP64 and in mixed precision, timed with
    events after one warm-up iteration from the initial Rayleigh-Ritz; the
    timed paro_apply_h / paro_apply_h_f32 on the 640-band block.  With tta,
    both precisions run from the trial block until the certified bound on the
    512 lowest eigenvalues is 1e-8 Ha, and the two sets of eigenvalues are
    compared band by band."""
    spec = synth.WORKLOADS["c3"]
    dev = torch.device("cuda:0")
    cell = synth.make_cell(spec, args.seed)
    v = synth.vloc_on_grid(cell["cell"], cell["grid"], cell["positions"], cell["depths"], cell["widths"])
    pl = P.Plan(cell["cell"], cell["ecut"], v, cell["projectors"], device=dev)
    nb, nconv, ncg = spec.n_carried, spec.n_bands, spec.n_cg
    x0 = torch.from_numpy(synth.trial_block(pl.ng, nb, args.seed)).to(dev)
    sig = pl.shift_lower_bound()
    kw = dict(shift_mode=P.SHIFT_ADAPTIVE, n_conv=nconv)
    out = {"workload": spec.name, "n_g": pl.ng, "grid": list(pl.grid), "bands": nb, "bands_converged": nconv,
           "projectors": pl.n_proj, "pcg_steps": ncg}
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    precs = (("fp64", P.PREC_FP64), ("mixed", P.PREC_MIXED), ("mixed_bf16", P.PREC_MIXED_BF16))
    for name, prec in precs:
        psi = x0.clone()
        st = pl.iterate(psi, 1, ncg, sig, initial_rr=True, stats=False, precision=prec, **kw)
        h, e = st["hpsi"], st["eps"]
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        pl.iterate(psi, steps, ncg, sig, hpsi=h, eps=e, initial_rr=False, stats=False, precision=prec, **kw)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[name] = {"outer_iterations_per_s": 1000.0 / ms, "ms_per_step": ms, "status_flags": pl.status()}
    x32 = x0.to(torch.complex64)
    bf = lambda blk, out=None: pl.apply_h_f32(blk, out=out, bf16=True)  # noqa: E731
    for name, f, blk in (("fp64", pl.apply_h, x0), ("mixed", pl.apply_h_f32, x32), ("mixed_bf16", bf, x32)):
        o = f(blk)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(3):
            f(blk, out=o)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 3 * 1e3 / nb
        local, nlf, byts = hpsi_work(pl.grid[0], pl.n_sticks, 2 * pl.nmax[0] + 1, pl.ng, pl.n_proj, 64)
        peak = PEAK_FP64_VALU if name == "fp64" else PEAK_FP32_VALU
        # split-BF16: three BF16 matrix-core products per product
        t_nl = 3 * nlf / PEAK_BF16_MFMA if name == "mixed_bf16" else nlf / peak
        t_roof = max(byts / (1 if name == "fp64" else 2) / PEAK_HBM, local / peak) * 1e6 + t_nl * 1e6
        out[name]["hpsi_us_per_band_apply"] = us
        out[name]["hpsi_roofline_frac"] = t_roof / us
        out[name]["hpsi_t_roof_us"] = t_roof
    for name in ("mixed", "mixed_bf16"):
        out[name]["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out[name]["ms_per_step"]
    if tta:
        final = {}
        for name, prec in precs:
            psi = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pl.iterate(psi, 0, ncg, sig, initial_rr=True, stats=True, precision=prec, **kw)
            h, e = r["hpsi"], r["eps"]
            its, bound, row = 0, np.inf, None
            while time.perf_counter() - t0 < tta_seconds:
                r = pl.iterate(psi, 10, ncg, sig, hpsi=h, eps=e, initial_rr=False, stats=True, precision=prec, **kw)
                its += r["n_done"]
                row = r["stats"][-1].cpu().numpy()
                bound = kato_temple_bound(row[:nb], row[nb:2 * nb], nconv)
                print(json.dumps({"c3_tta_progress": name, "outer_iterations": its, "bound": bound}), flush=True)
                if bound <= 1e-8:
                    break
            torch.cuda.synchronize()
            out[name]["time_to_1e-8"] = {"outer_iterations": its, "seconds": time.perf_counter() - t0,
                                         "eig_err_bound": bound, "reached": bool(bound <= 1e-8)}
            final[name] = row
        for name in ("mixed", "mixed_bf16"):
            de = np.abs(final[name][:nconv] - final["fp64"][:nconv])
            out[name + "_vs_fp64_eigenvalues"] = {
                "max_abs_diff_ha": float(de.max()), "median_abs_diff_ha": float(np.median(de)),
                "per_band_bound_ha": "Kato-Temple bound of each run <= 1e-8 (time_to_1e-8.eig_err_bound); "
                                     "|diff| <= sum of the two bounds"}
    return out


def adjoint_leg(args, P, torch, K=8):
    """The gradient of the band energy after K truncated outer iterations
    (N = 128 bands of the 34k-plane-wave cell, 20 PCG steps, fixed shift):
    the time of paro_truncated_gradient (forward with checkpoints, backward)
    against the forward alone (paro_iterate)."""
    spec = synth.WORKLOADS["c1"]
    cell = synth.make_cell(spec, args.seed)
    v = synth.vloc_on_grid(cell["cell"], cell["grid"], cell["positions"], cell["depths"], cell["widths"])
    pl = P.Plan(cell["cell"], cell["ecut"], v, cell["projectors"])
    nb = spec.n_bands
    x = torch.from_numpy(synth.trial_block(pl.ng, nb, args.seed)).cuda()
    sig = pl.shift_lower_bound()
    pl.truncated_gradient(x, 1, spec.n_cg, sig)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, dv, dr = pl.truncated_gradient(x, K, spec.n_cg, sig)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    t0 = time.perf_counter()
    pl.iterate(x.clone(), K, spec.n_cg, sig, stats=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    return {"workload": spec.name, "bands": nb, "outer_iterations": K, "pcg_steps": spec.n_cg,
            "seconds_per_gradient": t_grad, "seconds_forward_only": t_fwd, "gradient_over_forward": t_grad / t_fwd,
            "outputs": "dE/dV on the 96^3 grid, dE/dR for 128 projector centres"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-1e-8 run")
    ap.add_argument("--tta-seconds", type=float, default=60.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the 24-cell batched run")
    ap.add_argument("--no-c3", action="store_true", help="skip the 161k-plane-wave (160^3) leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the truncated-iteration gradient timing")
    ap.add_argument("--c3-tta", action="store_true",
                    help="only run the 161k-plane-wave leg with the time to 1e-8 Ha in both precisions and exit")
    ap.add_argument("--batch-only", action="store_true", help="only run the 24-cell batched leg and exit")
    ap.add_argument("--c3-only", action="store_true",
                    help="only run the 161k-plane-wave leg (3 timed outer iterations per precision) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--traffic-pass", action="store_true",
                    help="only run FP64 and FP32 H applies and density calls on the benchmark cell (HBM counters) "
                         "and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.traffic_pass:
        traffic_pass(args.seed)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the band-sharded multi-GPU "
              "layout is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1702_04045_amd as P
    from paper_1702_04045_amd import _lib as L
    if args.batch_only:
        print(json.dumps({"batched_cells": batched_cells(args, P, torch)}))
        return
    if args.c3_tta or args.c3_only:
        print(json.dumps({"at_scale": at_scale(args, P, torch, tta=args.c3_tta, tta_seconds=args.tta_seconds)}))
        return

    dev = torch.device("cuda:0")
    spec = synth.WORKLOADS["c1"]
    cell = synth.make_cell(spec, args.seed)
    v = synth.vloc_on_grid(cell["cell"], cell["grid"], cell["positions"], cell["depths"], cell["widths"])
    pl = P.Plan(cell["cell"], cell["ecut"], v, cell["projectors"], device=dev)
    nb, nconv, ncg = spec.n_carried, spec.n_bands, spec.n_cg
    x_np = synth.trial_block(pl.ng, nb, args.seed)
    x0 = torch.from_numpy(x_np).to(dev)
    sigma_lb = pl.shift_lower_bound()
    kw = dict(shift_mode=P.SHIFT_ADAPTIVE, n_conv=nconv)

    # the timing events, created before the warm-up: the library keeps them
    # for every later profile, so starting one leaves the GPU no idle time
    lib = P.load()
    L.check(lib.paro_profile_start_sampled(L.K_PLANE, 1 << 12, 1), "paro_profile_start_sampled")
    L.check(lib.paro_profile_stop(None, None), "paro_profile_stop")
    # initial Rayleigh-Ritz (Algorithm 1, step 1) and warm-up iterations (untimed)
    psi = x0.clone()
    st = pl.iterate(psi, 0, ncg, sigma_lb, initial_rr=True, stats=False, **kw)
    hpsi, eps = st["hpsi"], st["eps"]
    if args.warmup:
        pl.iterate(psi, args.warmup, ncg, sigma_lb, hpsi=hpsi, eps=eps, initial_rr=False, stats=False, **kw)
    torch.cuda.synchronize()
    start = (psi.clone(), hpsi.clone(), eps.clone())
    N = pl.grid[0]
    ncol = 2 * pl.nmax[0] + 1

    def launches_per_apply(precision):
        """Plane-stage launches of one apply: the bands go in chunks of 64
        (FP64 sticks) or 160 (FP32 sticks)."""
        chunk = 64 if precision == P.PREC_FP64 else 160
        return (nb + chunk - 1) // chunk

    def flops_launch(precision):
        return plane_flops(N, ncol) * (nb * pl.grid[2]) / launches_per_apply(precision)

    def timed(precision):
        """K outer iterations from the warmed-up state; HIP events around every
        PLANE_SAMPLE-th plane-stage launch."""
        import ctypes as C
        p, h, e = (t.clone() for t in start)
        if precision != P.PREC_FP64 and args.warmup:
            pl.iterate(p.clone(), 1, ncg, sigma_lb, hpsi=h.clone(), eps=e.clone(), initial_rr=False, stats=False,
                       precision=precision, **kw)
        torch.cuda.synchronize()
        # every PLANE_SAMPLE-th plane launch bracketed by events (coprime to the
        # three launches of an apply, so every chunk size is sampled)
        L.check(lib.paro_profile_start_sampled(L.K_PLANE, 1 << 12, PLANE_SAMPLE), "paro_profile_start_sampled")
        stream = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        pl.iterate(p, args.steps, ncg, sigma_lb, hpsi=h, eps=e, initial_rr=False, stats=True, precision=precision,
                   **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        nl, tot = C.c_int32(), C.c_double()
        L.check(lib.paro_profile_stop(C.byref(nl), C.byref(tot)), "paro_profile_stop")
        ms_step = e0.elapsed_time(e1) / max(args.steps, 1)
        # plane launches per step: n_cg + 1 applies in FP64, or n_cg in FP32 and one in FP64
        n_prec = launches_per_apply(precision) * (ncg if precision != P.PREC_FP64 else ncg + 1) * args.steps
        return ms_step, wall, nl.value, tot.value, n_prec

    def tta(precision, variant=P.VARIANT_PARO, n_cg=None):
        """Time to a 1e-8 Ha eigenvalue error from the trial block (separate run)."""
        if args.no_tta:
            return None
        n_cg = n_cg or ncg
        psi2 = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pl.iterate(psi2, 0, n_cg, sigma_lb, initial_rr=True, stats=True, precision=precision, variant=variant,
                       **kw)
        h2, e2 = r["hpsi"], r["eps"]
        its, bound, chunk = 0, np.inf, 10
        while time.perf_counter() - t0 < args.tta_seconds and its < 2000:
            r = pl.iterate(psi2, chunk, n_cg, sigma_lb, hpsi=h2, eps=e2, initial_rr=False, stats=True,
                           precision=precision, variant=variant, **kw)
            its += r["n_done"]
            row = r["stats"][-1].cpu().numpy()
            bound = kato_temple_bound(row[:nb], row[nb:2 * nb], nconv)
            if bound <= 1e-8:
                break
        torch.cuda.synchronize()
        names = {P.VARIANT_PARO: "ParO (Algorithm 1)", P.VARIANT_MPARO1: "MParO I (Algorithm 2)",
                 P.VARIANT_MPARO2: "MParO II (Algorithm 3)"}
        return {"outer_iterations": its, "seconds": time.perf_counter() - t0, "eig_err_bound": bound,
                "reached": bool(bound <= 1e-8), "checked_every": chunk, "pcg_steps": n_cg,
                "variant": names[variant] + ", adaptive shift"}

    def roofline_of(ms_step, nl, tot, precision, n_launches, every):
        """nl of the n_launches plane launches (one in every `every`) timed,
        tot ms in all."""
        avg_ms = tot / max(nl, 1)
        peak = PEAK_FP32_VALU if precision == P.PREC_MIXED else PEAK_FP64_VALU
        fl = flops_launch(precision)
        achieved = fl / (avg_ms * 1e-3)
        esize = 8 if precision == P.PREC_MIXED else 16
        bytes_launch = (2 * float(esize) * pl.n_sticks * pl.grid[2] * (nb / launches_per_apply(precision))
                        + esize / 2 * N ** 3)
        sch = pl.get_schedule(precision)
        name = (f"k_plane<96, {'float2' if precision == P.PREC_MIXED else 'double2'}, {sch['schedule']}>"
                f" (z-plane stage: n2/n1 FFTs, V multiply; {PLANE_SCHEDULES[sch['schedule']]},"
                f" {sch['bands']} bands per work-group)")
        return {"kernel": name, "bound": "alu",
                "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(TRAFFIC_FILE if precision == P.PREC_FP64 else F32_TRAFFIC_FILE),
                "algorithmic_bytes_per_launch": bytes_launch,
                "hbm_frac_algorithmic": bytes_launch / (avg_ms * 1e-3) / PEAK_HBM,
                "launches_timed": int(nl), "launches_sampled_every": every, "avg_launch_ms": avg_ms,
                "flops_per_launch": fl, "bands_per_launch": nb / launches_per_apply(precision),
                "share_of_step": avg_ms * n_launches / max(args.steps, 1) / ms_step}

    def hpsi_timed(block, reps=10):
        """paro_apply_h on the whole 160-band block, HIP events on the plan's
        stream around reps calls; the K1-K5 chain against its roofline."""
        out = torch.empty_like(block)
        pl.apply_h(block, out=out)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            pl.apply_h(block, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_call = e0.elapsed_time(e1) / reps
        us_band = ms_call * 1e3 / nb
        local, nlf, byts = hpsi_work(N, pl.n_sticks, ncol, pl.ng, pl.n_proj, nb / launches_per_apply(P.PREC_FP64))
        t_hbm = byts / PEAK_HBM * 1e6
        t_local = local / PEAK_FP64_VALU * 1e6
        t_nl = nlf / PEAK_FP64_VALU * 1e6
        t_roof = max(t_hbm, t_local) + t_nl
        return {"bands": nb, "ms_per_call": ms_call, "us_per_band_apply": us_band,
                "band_applies_per_s": 1e6 / us_band,
                "roofline": {"chain": "k_stick_inv + k_plane + k_stick_fwd (local) + k_gemm_hn_part + "
                                      "k_gemm_hn_reduce + k_gemm_nn (nonlocal)",
                             "bound": "fp64 (local transforms on the vector units at the HBM ridge; "
                                      "projector products on the matrix cores)",
                             "local_flops_per_band": local, "nonlocal_flops_per_band": nlf,
                             "bytes_per_band": byts, "t_hbm_us": t_hbm, "t_local_flops_us": t_local,
                             "t_nonlocal_us": t_nl, "t_roof_us": t_roof, "t_measured_us": us_band,
                             "frac": t_roof / us_band}}

    # FP64: every plane launch is the FP64 kernel
    ms_step, wall, nl, tot, n64 = timed(P.PREC_FP64)
    iters_s = 1000.0 / ms_step
    applies_s = iters_s * nb * (ncg + 1)
    status = pl.status()
    roofline = roofline_of(ms_step, nl, tot, P.PREC_FP64, n64, PLANE_SAMPLE)
    hpsi = hpsi_timed(psi)
    tta64 = tta(P.PREC_FP64)

    # mixed: the whole step is timed; its FP32 plane kernel is timed alone below
    ms_m, wall_m, _, _, n32 = timed(P.PREC_MIXED)
    iters_m = 1000.0 / ms_m
    mixed = {"value": iters_m, "unit": "ParO outer iterations/s", "ms_per_step": ms_m, "wall_s_timed": wall_m,
             "hpsi_applies_per_s": iters_m * nb * (ncg + 1), "dtype": "f32 source problems, f64 H U and RR",
             "speedup_vs_fp64": ms_step / ms_m, "status_flags": pl.status(),
             "time_to_1e-8": tta(P.PREC_MIXED)}
    # FP32 plane kernel alone (the mixed step's dominant kernel), HIP events over 10 FP32 applies
    import ctypes as C
    x32 = x0.to(torch.complex64)
    # untimed applies first: the GPU clocks back up after the host-side pause
    for _ in range(10):
        pl.apply_h_f32(x32)
    L.check(lib.paro_profile_start(L.K_PLANE, 1 << 12), "paro_profile_start")
    for _ in range(10):
        pl.apply_h_f32(x32)
    nlf, totf = C.c_int32(), C.c_double()
    L.check(lib.paro_profile_stop(C.byref(nlf), C.byref(totf)), "paro_profile_stop")
    mixed["roofline"] = roofline_of(ms_m, nlf.value, totf.value, P.PREC_MIXED, n32, 1)
    # the same with split-BF16 projector products in the FP32 source problems
    ms_b, wall_b, _, _, _ = timed(P.PREC_MIXED_BF16)
    mixed["bf16_projector_products"] = {
        "value": 1000.0 / ms_b, "unit": "ParO outer iterations/s", "ms_per_step": ms_b, "wall_s_timed": wall_b,
        "speedup_vs_fp64": ms_step / ms_b, "status_flags": pl.status(),
        "dtype": "f32 source problems with bf16x3 projector products, f64 H U and RR",
        "time_to_1e-8": tta(P.PREC_MIXED_BF16)}

    # density of the whole block (the Hellmann-Feynman gradient of the band
    # energy): the full call timed with events on the plan's stream, its
    # plane kernel with the library's per-launch events
    rho = pl.density(psi)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    L.check(lib.paro_profile_start(L.K_DENSITY, 1 << 12), "paro_profile_start")
    e0.record()
    for _ in range(10):
        pl.density(psi, out=rho)
    e1.record()
    torch.cuda.synchronize()
    nld, totd = C.c_int32(), C.c_double()
    L.check(lib.paro_profile_stop(C.byref(nld), C.byref(totd)), "paro_profile_stop")
    ms_dens = e0.elapsed_time(e1) / 10
    avg_d = totd.value / max(nld.value, 1)
    # per-launch means over the 64-band chunks of one call: sticks read once,
    # one partial grid written per group of 8 bands
    chunks = [min(64, nb - c0) for c0 in range(0, nb, 64)]
    fl_d = density_plane_flops(N, ncol) * pl.grid[2] * np.mean(chunks)
    bytes_d = float(np.mean([16.0 * pl.n_sticks * pl.grid[2] * cb + 8.0 * (-(-cb // 8)) * N ** 3
                             for cb in chunks]))
    # projector gradient of the same block (two matrix-core products with
    # the 128 projectors and G-weighted projectors, 4 x 8 N_G N_p flops per band)
    pl.projector_gradient(psi)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        pl.projector_gradient(psi)
    e1.record()
    torch.cuda.synchronize()
    ms_pg = e0.elapsed_time(e1) / 10
    fl_pg = 4 * 8.0 * pl.ng * pl.n_proj * nb
    density = {"bands": nb, "ms_per_call": ms_dens, "calls_per_s": 1000.0 / ms_dens,
               "projector_gradient": {"ms_per_call": ms_pg, "tflops": fl_pg / (ms_pg * 1e-3) / 1e12,
                                      "frac_fp64_matrix_peak": fl_pg / (ms_pg * 1e-3) / PEAK_FP64_VALU},
               "roofline": {"kernel": "k_plane_density<96> (z-plane stage: inverse n2/n1 FFTs, w |psi|^2)",
                            "bound": "alu", "achieved": fl_d / (avg_d * 1e-3) / 1e12,
                            "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                            "frac": fl_d / (avg_d * 1e-3) / PEAK_FP64_VALU,
                            "traffic": measured_traffic(DENSITY_TRAFFIC_FILE),
                            "algorithmic_bytes_per_launch": bytes_d,
                            "hbm_frac_algorithmic": bytes_d / (avg_d * 1e-3) / PEAK_HBM,
                            "launches_timed": int(nld.value), "avg_launch_ms": avg_d,
                            "flops_per_launch": fl_d, "share_of_call": totd.value / 10 / ms_dens}}

    # the paper's best variant with shorter source solves: MParO I converges
    # in about half the outer iterations of ParO, and 10 PCG steps per source
    # problem reach 1e-8 Ha in as few outer iterations as 20
    fastest = None if args.no_tta else {
        "fp64": tta(P.PREC_FP64, P.VARIANT_MPARO1, 10), "mixed": tta(P.PREC_MIXED, P.VARIANT_MPARO1, 10)}

    batched = None if args.no_batch else batched_cells(args, P, torch)
    scale = None if args.no_c3 else at_scale(args, P, torch)
    adjoint = None if args.no_adjoint else adjoint_leg(args, P, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, cell, v, x_np)

    rec = {"metric": METRIC, "value": iters_s, "unit": "ParO outer iterations/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": spec.name, "n_g": pl.ng, "grid": list(pl.grid), "bands": nb,
                      "bands_converged": nconv, "projectors": pl.n_proj, "pcg_steps": ncg,
                      "variant": "ParO (Algorithm 1)", "shift": "adaptive", "parallelism": "single GPU"},
           "hpsi_applies_per_s": applies_s, "hpsi_applies_per_s_note": "outer iterations/s x 160 bands x 21 "
           "applies (20 PCG + H U); hpsi_timed is paro_apply_h alone", "hpsi_timed": hpsi,
           "wall_s_timed": wall, "status_flags": status,
           "roofline": roofline, "time_to_1e-8": tta64, "mixed": mixed,
           "time_to_1e-8_mparo1_10pcg": fastest, "density": density, "batched_cells": batched,
           "mixed_at_scale": scale, "truncated_gradient": adjoint, "cpu_baseline": cpu}
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
