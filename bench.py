"""Benchmark: spherical harmonic transform pairs (alm2map + map2alm) per second.

Default workload (gl4095s2): 16 simultaneous spin-2 transforms (E/B <-> Q/U)
at lmax = mmax = 4095 on a Gauss-Legendre grid of 4096 rings x 8191 pixels,
a_lm ~ N(0, C_l) with C_l = 1/(l+1)^2 (seeded synthetic data), FP64.  The same
pairs are timed in the precision form (FP64 recursion, FP32 matrix-core
products with FP64 carry) and its speed-up and errors are reported next to the
FP64 number.

One step = one alm2map + map2alm pair of all transforms, inputs resident in
HBM, run through the stage entry points so that per-kernel times can be taken
with HIP events on the launch stream inside the timed region.  The staged
Legendre synthesis and FFT analysis also zero the phase entries of
polar-skipped terms (about 0.7 ms each at gl4095s2), which sht_execute does
not run: the reported rate slightly understates the full transforms.  The CPU
baseline times the oracle on a bounded sample of the same workload on the host
cores.

Other workloads (--workload): hp1024 (HEALPix N_side 1024, lmax 2047, one
scalar transform), gl127 (GL 128 x 255, lmax 127, one scalar transform),
hp2048 (HEALPix N_side 2048, lmax 4095, 8 maps: loss 0.5 ||alm2map(a) - d||^2
and its backward through the adjoint synthesis), mixed (64 scalar transforms,
16 each at lmax 255/511/1023/2047 on matching GL grids, as one batch).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32_mfma": 157.3e12, "hbm": 8.0e12}
METRIC = "alm2map+map2alm pairs/sec at lmax=4095; FP32-MFMA vs FP64 speedup at 1e-6"

# HBM traffic of the dominant kernel, summarised from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE) of this benchmark; only used while the
# kernel sources hash to what they were when the counters were taken.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "legendre_anal_gl4095s2_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1303_4945_amd", "csrc", f)
                  for f in ("legendre.hip", "sht_internal.h")] + \
                 [os.path.join(ROOT, "paper_1303_4945_amd", "build.py")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gl4095s2",
                    choices=["gl4095s2", "hp1024", "gl127", "hp2048", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-j1", action="store_true", help="skip the 16 x (J = 1) comparison")
    ap.add_argument("--cpu-items", type=int, default=0,
                    help="sampled rings and m values of the CPU baseline (default: the thread count)")
    ap.add_argument("--cpu-ntrans", type=int, default=2)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, run a plain device copy of this many MiB three "
                         "times (calibrates the HBM byte counters of a --pmc profile)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(x, ref):
    d = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / (d if d > 0 else 1.0))


def per_degree_rel(x, ref, lmax):
    """max over l >= 2 of sqrt(sum_m |x - ref|^2 / sum_m |ref|^2), and the l."""
    import sht_inputs as si
    ls, _ = si.lm_arrays(lmax, lmax)
    d2 = np.sum((x - ref) ** 2, axis=(0, 1, 3))
    r2 = np.sum(ref ** 2, axis=(0, 1, 3))
    num = np.bincount(ls, weights=d2, minlength=lmax + 1)
    den = np.bincount(ls, weights=r2, minlength=lmax + 1)
    pd = np.where(den > 0, np.sqrt(num / np.where(den > 0, den, 1.0)), 0.0)
    pd[:2] = 0.0
    return float(pd.max()), int(np.argmax(pd))


def pair_errors(a, back):
    """Errors of a synthesis-analysis pair as Sect. 5 defines them: the relative rms
    error over all stored coefficients and the largest absolute error of one."""
    d = (back - a).ravel()
    rms = math.sqrt(float(np.dot(d, d)) / float(np.dot(a.ravel(), a.ravel())))
    d = d.reshape(a.shape)
    mx = float(np.sqrt(np.max(d[..., 0] ** 2 + d[..., 1] ** 2)))
    return {"eps_rms": rms, "eps_max": mx}


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic():
    """Bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is absent or the kernel changed since."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"<!-- traffic (\{.*?\}) -->", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != kernel_sources_hash():
        return None
    return rec


def copy_probe(mib):
    """A plain streaming kernel of known size: reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    return {"nproc": os.cpu_count(), "omp_threads": threads, "cpu_model": model}


STAGES = ["legendre_synth", "ring_synth", "ring_anal", "legendre_anal"]


def time_pairs(plan, alm, steps, warmup):
    """Run warmup + timed steps through the stage entry points (the kernels
    sht_execute launches, plus the fill of polar-skipped phase entries after
    the Legendre synthesis and the FFT analysis), recording HIP events between
    stages on the stream the library launches on (torch's current stream)."""
    import torch

    def one(evs=None):
        if evs:
            evs[0].record()
        F = plan.legendre_synth(alm)
        if evs:
            evs[1].record()
        mp = plan.ring_synth(F)
        if evs:
            evs[2].record()
        G = plan.ring_anal(mp, weights=True)
        if evs:
            evs[3].record()
        out = plan.legendre_anal(G)
        if evs:
            evs[4].record()
        return mp, out

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        mp, out = one(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = {n: [] for n in STAGES}
    for k in range(steps):
        for i, n in enumerate(STAGES):
            ktimes[n].append(ev[k][i].elapsed_time(ev[k][i + 1]))
    return (t1 - t0) * 1e3 / steps, {n: float(np.mean(v)) for n, v in ktimes.items()}, mp, out


def fused_pairs(plan, alm, steps, warmup):
    """Whole transform pairs through sht_execute (alm2map, then map2alm of its
    map) into preallocated outputs: ms per pair, and the last map and a_lm."""
    import torch
    mp = torch.empty(plan.map_shape, dtype=torch.float64, device=alm.device)
    back = torch.empty(plan.alm_shape, dtype=torch.float64, device=alm.device)
    for _ in range(warmup):
        plan.alm2map(alm, out=mp)
        plan.map2alm(mp, out=back)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.alm2map(alm, out=mp)
        plan.map2alm(mp, out=back)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, mp, back


def legendre_fracs(plan, kms):
    """Per Legendre kernel: achieved FLOP/s and the fraction of the time floor
    flops_fp64 / 78.6 TFLOP/s + flops_mfma / 157.3 TFLOP/s."""
    import paper_1303_4945_amd as sht
    out = {}
    for name, d in (("legendre_synth", sht.ALM2MAP), ("legendre_anal", sht.MAP2ALM)):
        f64, fmm, _ = plan.flops(d)
        t = kms[name] * 1e-3
        floor = f64 / PEAK["fp64"] + fmm / PEAK["fp32_mfma"]
        out[name] = {"tflops": (f64 + fmm) / t / 1e12, "floor_ms": floor * 1e3, "frac": floor / t}
    return out


def fft_hbm(plan, kms):
    """Ring FFT kernels against HBM: algorithmic bytes per launch (maps read or
    written once, phases written or read once) over the event time."""
    ph = 16.0 * plan.ntrans * plan.ncomp * plan.nrings * (plan.mmax + 1)
    mp = 8.0 * plan.ntrans * plan.ncomp * plan.npix
    out = {}
    for name in ("ring_synth", "ring_anal"):
        t = kms[name] * 1e-3
        out[name] = {"bytes_per_launch": ph + mp, "gbps": (ph + mp) / t / 1e9,
                     "frac": (ph + mp) / t / PEAK["hbm"]}
    return out


def cpu_baseline(g, lmax, spin, a, nitems, ntrans_s, G64map, G64alm, G32map, G32alm):
    """Oracle on a bounded sample: synthesis of `nitems` rings and analysis of
    `nitems` m values for the first `ntrans_s` transforms; scaled to whole
    pairs.  OpenMP runs over the sampled rings resp. m values, one per thread."""
    import oracle
    oracle.build(force=False)
    hi = host_info()
    rings = np.linspace(0, g.nrings - 1, nitems).round().astype(int)
    ms = np.linspace(0, lmax, nitems).round().astype(int)
    sub = np.ascontiguousarray(a[:ntrans_s])
    t0 = time.perf_counter()
    ref_map = oracle.synthesis(g, lmax, lmax, spin, sub, rings=rings)
    t1 = time.perf_counter()
    # analysis input: the GPU FP64 map of the same transforms (any map will do
    # for timing; using it also gives a sampled parity check of map2alm)
    ref_alm = oracle.analysis(g, lmax, lmax, spin, G64map[:ntrans_s], ms=ms)
    t2 = time.perf_counter()
    ts, ta = t1 - t0, t2 - t1
    used = min(hi["omp_threads"], nitems)
    ntr = a.shape[0]
    t_pair = (ts / nitems * g.nrings + ta / nitems * (lmax + 1)) * (ntr / ntrans_s)
    pix = np.concatenate([np.arange(g.ofs[y], g.ofs[y] + g.nphi[y]) for y in rings])
    lsel = np.concatenate([np.arange(m * (2 * lmax + 1 - m) // 2 + m,
                                     m * (2 * lmax + 1 - m) // 2 + lmax + 1) for m in ms])
    acc = {
        "fp64_map_sampled_rel_err": rel_err(G64map[:ntrans_s][..., pix], ref_map[..., pix]),
        "fp64_alm_sampled_rel_err": rel_err(G64alm[:ntrans_s][:, :, lsel], ref_alm[:, :, lsel]),
    }
    if G32map is not None:
        acc["fp32_map_sampled_rel_err"] = rel_err(G32map[:ntrans_s][..., pix], ref_map[..., pix])
        acc["fp32_alm_sampled_rel_err"] = rel_err(G32alm[:ntrans_s][:, :, lsel], ref_alm[:, :, lsel])
    res = {"value": ntr / t_pair, "unit": "pairs/s", "cores": used, "kind": "oracle",
           "nproc": hi["nproc"], "cpu_model": hi["cpu_model"],
           "sample": (f"synthesis of {nitems} of {g.nrings} rings and analysis of {nitems} of "
                      f"{lmax + 1} m for {ntrans_s} of {ntr} transforms "
                      f"({ts:.1f} s + {ta:.1f} s wall on {used} threads), scaled to whole pairs")}
    return res, acc


def base_record(args, value, ms, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype,
            "data": "synthetic (seeded power-law a_lm, C_l = 1/(l+1)^2)", "config": config}


def roofline_record(plan, kms, name):
    """FP64 plans: the MFMA path is bound by the FP64 matrix cores, the vector
    path by the FP64 vector ALUs (256 CUs x 4 SIMDs x 16 lanes x 2 flop per FMA
    x 2.4 GHz = 78.6 TFLOP/s); both peaks are the same figure."""
    import paper_1303_4945_amd as sht
    f64, fmm, _ = plan.flops(sht.ALM2MAP if name == "legendre_synth" else sht.MAP2ALM)
    achieved = (f64 + fmm) / (kms[name] * 1e-3)
    bound = "alu" if plan.tuning()["valu"] else "mfma"
    return {"bound": bound, "kernel": f"{name} (fp64)", "achieved": achieved / 1e12,
            "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK["fp64"],
            "traffic": None, "flops_per_launch": f64 + fmm}


def run_gl4095s2(args):
    import torch

    import sht_inputs as si
    import paper_1303_4945_amd as sht

    lmax, spin, ntrans = 4095, 2, 16
    t = time.perf_counter()
    g = si.gauss_geometry(4096, 8191)
    a = si.random_alm(lmax, lmax, ntrans, spin)
    log(f"inputs ready in {time.perf_counter() - t:.1f} s")
    geom = sht.Geometry.from_inputs(g)
    alm = torch.from_numpy(a).to("cuda:0")

    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    t = time.perf_counter()
    p64 = sht.Plan(geom, lmax, spin=spin, ntrans=ntrans, precision="fp64")
    log(f"fp64 plan in {time.perf_counter() - t:.2f} s")
    # value: whole pairs through sht_execute; stage times: the staged entry points
    ms64, map64, alm64 = fused_pairs(p64, alm, args.steps, args.warmup)
    ms64_staged, k64, _, _ = time_pairs(p64, alm, args.steps, 1)
    log(f"fp64: {ms64:.1f} ms/pair-step (staged {ms64_staged:.1f})  kernels {k64}")
    map64_h = map64.cpu().numpy()
    alm64_h = alm64.cpu().numpy()
    del map64, alm64
    map32_h = alm32_h = None
    if not args.no_fp32:
        p32 = sht.Plan(geom, lmax, spin=spin, ntrans=ntrans, precision="fp32_mfma")
        ms32, map32, alm32 = fused_pairs(p32, alm, args.steps, args.warmup)
        ms32_staged, k32, _, _ = time_pairs(p32, alm, args.steps, 1)
        log(f"fp32: {ms32:.1f} ms/pair-step (staged {ms32_staged:.1f})  kernels {k32}")
        map32_h = map32.cpu().numpy()
        alm32_h = alm32.cpu().numpy()
        fr32 = legendre_fracs(p32, k32)
        del map32, alm32, p32
    j1 = None
    if not args.no_j1:
        # Sect. 5.2.4 / Fig. 10 analogue: 16 simultaneous transforms (lambda
        # computed once per triple) against 16 single transforms
        p1 = sht.Plan(geom, lmax, spin=spin, ntrans=1, precision="fp64")
        a1 = alm[:1].contiguous()
        ms1, _, _ = fused_pairs(p1, a1, max(1, args.steps - 1), 1)
        _, k1, _, _ = time_pairs(p1, a1, max(1, args.steps - 1), 1)
        leg1 = k1["legendre_synth"] + k1["legendre_anal"]
        leg16 = k64["legendre_synth"] + k64["legendre_anal"]
        j1 = {"j16_pair_ms": ms64, "j1_pair_ms_x16": 16 * ms1, "pair_speedup": 16 * ms1 / ms64,
              "j16_legendre_ms": leg16, "j1_legendre_ms_x16": 16 * leg1, "legendre_speedup": 16 * leg1 / leg16,
              "j1_legendre_kernels": "vector units" if p1.tuning()["valu"] else "matrix cores",
              "j1_legendre_synth_ms": k1["legendre_synth"], "j1_legendre_anal_ms": k1["legendre_anal"]}
        del p1
    torch.cuda.empty_cache()

    dom = max(("legendre_synth", "legendre_anal"), key=lambda n: k64[n])
    ncomp = 2
    leg_bytes = 16.0 * ntrans * ncomp * (g.nrings * (lmax + 1) + (lmax + 1) * (lmax + 2) // 2)
    tr = profiled_traffic()
    config = {"workload": "gl4095s2: Gauss-Legendre 4096 rings x 8191 px, lmax=mmax=4095, "
                          "spin 2 E/B<->Q/U, 16 simultaneous transforms",
              "lmax": lmax, "spin": spin, "ntrans": ntrans, "nrings": 4096, "nphi": 8191}
    out = base_record(args, ntrans / (ms64 * 1e-3), ms64, "f64", config)
    out["ms_per_step_staged"] = ms64_staged
    out["kernels_ms"] = {"fp64": k64}
    out["roofline"] = roofline_record(p64, k64, dom)
    out["roofline"]["traffic"] = tr["bytes_per_launch"] if tr and tr.get("kernel") == dom else None
    out["roofline"]["algorithmic_bytes_per_launch"] = leg_bytes
    out["legendre_fp64"] = legendre_fracs(p64, k64)
    out["ring_fft_hbm"] = fft_hbm(p64, k64)
    if j1:
        out["simultaneous_transforms"] = j1
    # the pair's own round trip (exact quadrature on this grid)
    out["sht_pair_errors"] = {"fp64": pair_errors(a, alm64_h),
                              "inputs": "the timed pair's power-law a_lm, C_l = 1/(l+1)^2"}
    if not args.no_fp32:
        out["sht_pair_errors"]["fp32_mfma"] = pair_errors(a, alm32_h)
        out["kernels_ms"]["fp32_mfma"] = k32
        pd, pl = per_degree_rel(alm32_h, alm64_h, lmax)
        out["fp32_mfma"] = {"value": ntrans / (ms32 * 1e-3), "unit": "pairs/s", "ms_per_step": ms32,
                            "speedup_vs_fp64": ms64 / ms32,
                            "legendre": fr32,
                            "max_rel_err_map_vs_fp64": rel_err(map32_h, map64_h),
                            "max_rel_err_alm_vs_fp64": rel_err(alm32_h, alm64_h),
                            "max_per_degree_rel_err_alm_vs_fp64": pd, "at_degree": pl}
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        nitems = args.cpu_items or max(8, host_info()["omp_threads"])
        cb, acc = cpu_baseline(g, lmax, spin, a, nitems, args.cpu_ntrans, map64_h, alm64_h, map32_h, alm32_h)
        log(f"cpu baseline in {time.perf_counter() - t:.1f} s")
        out["cpu_baseline"] = cb
        out["accuracy_vs_oracle"] = acc
    return out


def run_single(args, name):
    """hp1024 / gl127: one scalar FP64 transform pair (alm2map, then map2alm of
    its map) through sht_execute; stage times from the staged entry points."""
    import torch

    import sht_inputs as si
    import paper_1303_4945_amd as sht
    if name == "hp1024":
        lmax, g = 2047, si.healpix_geometry(1024)
        desc = "hp1024: HEALPix N_side 1024 (4095 rings, 12,582,912 px), lmax=mmax=2047, 1 scalar transform"
    else:
        lmax, g = 127, si.gauss_geometry(128, 255)
        desc = "gl127: Gauss-Legendre 128 rings x 255 px, lmax=mmax=127, 1 scalar transform"
    a = si.random_alm(lmax, lmax, 1, 0, spectrum="powerlaw" if name == "hp1024" else "unit", tag=7)
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=0, ntrans=1)
    alm = torch.from_numpy(a).to("cuda:0")
    # timed: whole transforms through sht_execute (alm2map, then map2alm of its
    # map) into preallocated outputs; a small transform needs many steps
    steps = max(args.steps, 200) if name == "gl127" else args.steps
    mp = torch.empty(p.map_shape, dtype=torch.float64, device="cuda:0")
    back = torch.empty(p.alm_shape, dtype=torch.float64, device="cuda:0")
    for _ in range(max(args.warmup, 2)):
        p.alm2map(alm, out=mp)
        p.map2alm(mp, out=back)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.alm2map(alm, out=mp)
        p.map2alm(mp, out=back)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # stage times (HIP events between the staged entry points)
    _, k, _, _ = time_pairs(p, alm, max(args.steps, 5), 2)
    log(f"{name}: {ms:.3f} ms/pair  kernels {k}")
    out = base_record(args, 1.0 / (ms * 1e-3), ms, "f64",
                      {"workload": desc, "lmax": lmax, "spin": 0, "ntrans": 1, "nrings": g.nrings})
    out["steps"] = steps
    out["metric"] = "alm2map+map2alm pairs/sec"
    out["kernels_ms"] = {"fp64": k}
    dom = max(("legendre_synth", "legendre_anal"), key=lambda n: k[n])
    out["roofline"] = roofline_record(p, k, dom)
    out["legendre_fp64"] = legendre_fracs(p, k)
    out["ring_fft_hbm"] = fft_hbm(p, k)
    return out


def run_hp2048(args):
    """Differentiation form: loss = 0.5 ||alm2map(a) - d||^2 and its gradient
    through the hand-written adjoint synthesis, 8 maps at N_side 2048."""
    import torch

    import sht_inputs as si
    import paper_1303_4945_amd as sht
    from paper_1303_4945_amd import autograd as sag
    lmax = 4095
    g = si.healpix_geometry(2048)
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=0, ntrans=8)
    a_true = torch.from_numpy(si.random_alm(lmax, lmax, 8, 0, tag=81)).cuda()
    d = p.alm2map(a_true) + torch.from_numpy(si.random_map(g, 8, 1, sigma=0.1, tag=82)).cuda()
    a = (a_true + torch.from_numpy(si.random_alm(lmax, lmax, 8, 0, tag=83)).cuda()).requires_grad_(True)

    def step():
        a.grad = None
        loss = 0.5 * torch.sum((sag.alm2map(a, p) - d) ** 2)
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # stage times of the forward and the backward kernels
    _, k, _, _ = time_pairs(p, a.detach(), 2, 1)
    log(f"hp2048 loss+backward: {ms:.1f} ms/step  kernels {k}")
    out = base_record(args, 8.0 / (ms * 1e-3), ms, "f64",
                      {"workload": "hp2048: HEALPix N_side 2048 (8191 rings, 50,331,648 px), lmax=4095, "
                                   "8 scalar maps, loss 0.5||alm2map(a)-d||^2 + backward (adjoint synthesis)",
                       "lmax": lmax, "spin": 0, "ntrans": 8})
    out["metric"] = "loss+gradient evaluations (forward + adjoint) per second, per map"
    out["kernels_ms"] = {"fp64_pair_stages": k}
    dom = max(("legendre_synth", "legendre_anal"), key=lambda n: k[n])
    out["roofline"] = roofline_record(p, k, dom)
    out["legendre_fp64"] = legendre_fracs(p, k)
    out["ring_fft_hbm"] = fft_hbm(p, k)
    return out


def run_mixed(args):
    """Batching form: 64 scalar transforms (16 each at lmax 255/511/1023/2047,
    GL grids of lmax+1 rings x 2lmax+1 px) as one batch on a non-default stream
    (captured into a HIP graph), against the four plans run one after another;
    each schedule of the batch (queue order; per-plan chains on one stream or
    concurrent streams, or the persistent synthesis over all plans) is timed,
    the fastest is the reported value.  The staged batch Legendre steps are
    timed with events for the roofline of the persistent analysis kernel."""
    import torch

    import sht_inputs as si
    import paper_1303_4945_amd as sht
    lmaxes = [255, 511, 1023, 2047]
    plans, alms = [], []
    for k, lmax in enumerate(lmaxes):
        g = si.gauss_geometry(lmax + 1, 2 * lmax + 1, 0.1 * k)
        plans.append(sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=0, ntrans=16))
        alms.append(torch.from_numpy(si.random_alm(lmax, lmax, 16, 0, tag=100 + k)).cuda())
    t = time.perf_counter()
    for p in plans:
        p.autotune(2.0)
    log(f"autotuned in {time.perf_counter() - t:.1f} s: {[p.tuning() for p in plans]}")
    b = sht.Batch(plans)
    s = torch.cuda.Stream()
    maps = [torch.empty(p.map_shape, dtype=torch.float64, device="cuda") for p in plans]
    back = [torch.empty(p.alm_shape, dtype=torch.float64, device="cuda") for p in plans]
    ph = [torch.empty(p.phase_shape, dtype=torch.float64, device="cuda") for p in plans]

    def batch_step():
        b.alm2map(alms, outs=maps, stream=s)
        b.map2alm(maps, outs=back, stream=s)

    def plans_step():
        for p, a, mp, ab in zip(plans, alms, maps, back):
            p.alm2map(a, out=mp, stream=s)
            p.map2alm(mp, out=ab, stream=s)

    def timed(fn, steps):
        for _ in range(max(args.warmup, 2)):
            fn()
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    res = {}
    with torch.cuda.stream(s):
        res["plans_one_by_one"] = timed(plans_step, args.steps)
        # the persistent synthesis (schedule 2) runs only when every plan is on
        # the matrix-core kernels with one synthesis shape
        tun = [p.tuning() for p in plans]
        eligible = all(t["valu"] == 0 for t in tun) and len({t["synth_ncb"] for t in tun}) == 1
        sched = {"serial": 0, "concurrent": 1}
        if eligible:
            sched["persistent_synthesis"] = 2
        for conc in sched:
            for order in (sht.QUEUE_COST, sht.QUEUE_MPAIRS):
                b.configure(order, sched[conc])
                name = f"batch_{'cost' if order == sht.QUEUE_COST else 'mpairs'}_{conc}"
                res[name] = timed(batch_step, args.steps)
        best = min((k for k in res if k.startswith("batch")), key=lambda k: res[k])

        def use_best():
            b.configure(sht.QUEUE_MPAIRS if "mpairs" in best else sht.QUEUE_COST,
                        next(v for k, v in sched.items() if best.endswith(k)))

        # the persistent synthesis against the per-plan chains with every plan on
        # one matrix-core synthesis shape (the autotuned choice restored after)
        common = {}
        for p in plans:
            p.set_tuning(valu=0, synth_ncb=1)
        for conc, v in (("concurrent", 1), ("persistent_synthesis", 2)):
            b.configure(sht.QUEUE_COST, v)
            common[f"batch_cost_{conc}"] = timed(batch_step, args.steps)
            common[f"legendre_synth_{conc}"] = timed(lambda: b.legendre(sht.ALM2MAP, alms, ph, stream=s), args.steps)
        for p, t in zip(plans, tun):
            p.set_tuning(**t)
        use_best()
        ms = timed(batch_step, args.steps)
        # staged Legendre steps of the batch (events on the launch stream)
        leg = {"legendre_synth": timed(lambda: b.legendre(sht.ALM2MAP, alms, ph, stream=s), args.steps)}
        b.legendre(sht.ALM2MAP, alms, ph, stream=s)
        leg["legendre_anal"] = timed(lambda: b.legendre(sht.MAP2ALM, ph, back, stream=s), args.steps)
    log(f"mixed: {res}; chosen {best}: {ms:.2f} ms/pair-step; staged Legendre {leg}; one matrix-core "
        f"shape, per-plan chains vs persistent synthesis: {common}")
    f64 = sum(p.flops(sht.MAP2ALM)[0] for p in plans)
    out = base_record(args, 64.0 / (ms * 1e-3), ms, "f64",
                      {"workload": "mixed: 64 scalar transforms, 16 each at lmax 255/511/1023/2047 on "
                                   "GL grids (lmax+1 rings x 2lmax+1 px), one batch, HIP graph",
                       "lmaxes": lmaxes, "ntrans_each": 16, "schedule": best})
    out["metric"] = "alm2map+map2alm pairs/sec (mixed batch)"
    out["schedules_ms"] = res
    out["persistent_synthesis_vs_chains_ms"] = {"tuning": "every plan matrix-core, synth_ncb 1", **common}
    out["batch_speedup_vs_plans"] = res["plans_one_by_one"] / ms
    out["kernels_ms"] = {"batch_legendre": leg}
    achieved = f64 / (leg["legendre_anal"] * 1e-3)
    valu = any(p.tuning()["valu"] for p in plans)
    out["roofline"] = {"bound": "alu" if valu else "mfma",
                       "kernel": "batch legendre_anal (fp64, " + ("per-plan launches)" if valu else "persistent)"),
                       "achieved": achieved / 1e12, "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                       "frac": achieved / PEAK["fp64"], "traffic": None, "flops_per_launch": f64}
    out["tuning"] = [p.tuning() for p in plans]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not a build", file=sys.stderr)
        sys.exit(2)
    if args.workload == "gl4095s2":
        out = run_gl4095s2(args)
    elif args.workload in ("hp1024", "gl127"):
        out = run_single(args, args.workload)
    elif args.workload == "hp2048":
        out = run_hp2048(args)
    else:
        out = run_mixed(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
