#!/usr/bin/env python3
"""Throughput of the FDAS hot path on one MI355X.

Workload (the SKA-shaped single trial): 2^23 float32 samples of seeded white
noise plus 4 injected accelerated pulsars with 8 harmonics each; 201 templates
(z in [-200, 200], step 2); 8192-bin overlap-save segments; harmonic sums over
1/2/4/8/16 harmonics; 6-sigma threshold.  One step = one trial through the
whole path (real DFT, normalisation, segment DFTs, template multiply, inverse
DFTs, powers, harmonic sums, peaks, candidates to the host) with the series
already resident in device memory.

Prints one JSON line: the plain per-trial rate as ``value``, plus the batched
rate, a short served burst (host series in, PCIe included) with p50/p99
latency, the roofline of the dominant kernel (the fused multiply / inverse
DFT / power kernel, timed with HIP events on its own stream during the timed
steps) and the FP64 CPU oracle timed on a bounded sample of the same trial.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 1 << 23
ZMAX, DZ, SEG = 200.0, 2.0, 8192
NHARM, SIGMA = 16, 6.0
METRIC = "DM trials/sec (2^23 samp, z∈[-200,200]) plain vs served/batched; p50/p99 latency"
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "correlate_ska_trial_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1511_07343_amd", "csrc", f) for f in ("kernels.hip", "fft_wg.hpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def correlate_flops(nseg: int, nz: int, S: int, L: int) -> float:
    """Algorithmic flops of one fused-correlation launch: per (segment,
    template) an S-point complex inverse DFT (5 S log2 S), the complex multiply
    (6 S) and the powers of the L kept bins (3 L)."""
    lg = S.bit_length() - 1
    return float(nseg) * nz * (5.0 * S * lg + 6.0 * S + 3.0 * L)


def correlate_bytes(nseg: int, nz: int, S: int, nb: int) -> float:
    """Algorithmic HBM bytes of one fused-correlation launch: the plane written
    once (4 nz Nb), the segment spectra (8 nseg S) and the bank (8 nz S) read once."""
    return 4.0 * nz * nb + 8.0 * nseg * S + 8.0 * nz * S


def read_traffic():
    """HBM bytes per correlation launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    for line in open(PROFILE_TRAFFIC):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(trial, bins: int):
    """Time the FP64 oracle on a bounded sample of one trial: the real DFT and
    normalisation of the whole series, then the direct correlation, harmonic
    sums and peaks over all templates for `bins` consecutive frequency bins,
    scaled to the whole spectrum."""
    import numpy as np

    import oracle as O

    omp = os.environ.get("OMP_NUM_THREADS")
    cores = len(os.sched_getaffinity(0))
    if omp:
        cores = min(cores, int(omp))
    t0 = time.perf_counter()
    Xh = O.normalise(O.real_spectrum(trial.x), 1024)
    t_spec = time.perf_counter() - t0
    taps, zs, h = O.template_taps(ZMAX, DZ)
    nb = N // 2
    k0 = nb // 3
    seg = Xh[k0 - h: k0 + bins + h]
    t0 = time.perf_counter()
    P = O.correlate(seg, taps)[:, h: h + bins]
    t_corr = time.perf_counter() - t0
    izc = (zs.shape[0] - 1) // 2
    thr = O.thresholds(SIGMA, O.harmonic_list(NHARM))
    t0 = time.perf_counter()
    for nh in O.harmonic_list(NHARM):
        S = P if nh == 1 else O.harmonic_sum(P, nh, izc)
        O.find_peaks(S, thr[nh])
    t_hs = time.perf_counter() - t0
    scale = nb / bins
    t_trial = t_spec + scale * (t_corr + t_hs)
    return {
        "value": 1.0 / t_trial, "unit": "DM trials/s", "cores": cores, "kind": "oracle",
        "sample": (f"one 2^23-sample trial: FP64 real DFT + normalisation of the whole series "
                   f"({t_spec:.2f} s), then direct correlation ({t_corr:.2f} s), harmonic sums and peaks "
                   f"({t_hs:.2f} s) for all 201 templates over {bins} of {nb} bins, scaled x{scale:.0f}; "
                   f"{t_spec + t_corr + t_hs:.1f} s measured, {t_trial:.0f} s per trial extrapolated"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8, help="trials per batched launch")
    ap.add_argument("--served", type=int, default=24, help="requests in the served burst (0 = skip)")
    ap.add_argument("--cpu-bins", type=int, default=1 << 17, help="oracle sample width in bins (0 = skip)")
    ap.add_argument("--plain-only", action="store_true", help="only the plain per-trial loop (profiling)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build runs the search on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1511_07343_amd as fdas
    import synth

    fdas.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating inputs")
    trials = [synth.ska_trial(N, seed=2)] + [synth.ska_trial(N, seed=1000 + i, npulsars=i % 4) for i in range(3)]
    xs = [torch.from_numpy(t.x).to(dev) for t in trials]
    bank = fdas.make_templates(ZMAX, DZ)
    plan = fdas.Plan(bank, N, SEG, nharm_max=NHARM, sigma=SIGMA)
    nz, h = bank.nz, bank.h
    L = SEG - 2 * h
    nb = N // 2
    nseg = -(-nb // L)
    torch.cuda.synchronize()

    out = fdas.pinned_candidates(1 << 22)  # page-locked record buffer, reused every step
    log(f"warmup {args.warmup}")
    for i in range(args.warmup):
        plan.search(xs[i % len(xs)], out=out)
    torch.cuda.synchronize()
    plan.enable_timing(True)
    lat = []
    log(f"timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        plan.search(xs[i % len(xs)], out=out)
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, ntimed = plan.stage_times()
    plan.enable_timing(False)
    ms_step = 1e3 * (t1 - t0) / args.steps
    value = args.steps / (t1 - t0)
    corr_ms = stages["correlate"] / max(ntimed, 1)
    flops = correlate_flops(nseg, nz, SEG, L)
    achieved = flops / (corr_ms * 1e-3) / 1e12
    traffic = read_traffic()
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "DM trials/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "SKA-shaped single trial: 2^23 float32 samples, 4 pulsars x 8 harmonics, "
                               "201 templates z in [-200,200] step 2, 8192-bin segments, 1/2/4/8/16 "
                               "harmonic sums, 6 sigma; series resident in HBM",
                   "nsamp": N, "templates": nz, "segment": SEG, "halfwidth": h, "segments": nseg,
                   "path": "plain (fdas_search per trial)"},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 4),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 4)},
        "stages_ms": {k: round(v / max(ntimed, 1), 4) for k, v in stages.items()},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": traffic, "kernel": "k_correlate (fused multiply, inverse DFT, power)",
                     "algorithmic_flops": flops, "launch_ms": round(corr_ms, 4),
                     "hbm_GBs": round(correlate_bytes(nseg, nz, SEG, nb) / (corr_ms * 1e-3) / 1e9, 1)},
    }

    if not args.plain_only and args.batch > 0:
        log("autotune (segment length, templates per block) for the batched path")
        seg_b, tpb_b, tune_ms = fdas.autotune(bank, N, nharm_max=NHARM, sigma=SIGMA)
        log(f"batched: {args.batch} trials per call, segment {seg_b}, {tpb_b} templates per block")
        planb = fdas.Plan(bank, N, seg_b, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb_b)
        bx = [xs[i % len(xs)] for i in range(args.batch)]
        bcap = 1 << 20
        bout = fdas.pinned_candidates(bcap * len(bx))
        planb.search_batch(bx, caps=[bcap] * len(bx), out=bout)
        torch.cuda.synchronize()
        reps = 3
        tb0 = time.perf_counter()
        for _ in range(reps):
            planb.search_batch(bx, caps=[bcap] * len(bx), out=bout)
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb0
        planb.close()
        out["batched"] = {"value": round(reps * len(bx) / tb, 3), "unit": "DM trials/s",
                          "trials_per_call": len(bx), "ms_per_trial": round(1e3 * tb / (reps * len(bx)), 4),
                          "autotuned": {"segment": seg_b, "templates_per_block": tpb_b,
                                        "segment_dft_plus_correlate_ms": round(tune_ms, 4)}}
    plan.close()

    if not args.plain_only and args.served > 0:
        log(f"served burst: {args.served} requests")
        rng = np.random.default_rng(4)
        lens = rng.choice([1 << 21, 1 << 22, 1 << 23], size=args.served, p=[0.2, 0.3, 0.5])
        host = {n: synth.make_series(int(n), seed=40000 + int(n).bit_length()).x for n in set(lens.tolist())}
        srv = fdas.Server(bank, SEG, N, max_slots=4, nharm_max=NHARM, sigma=SIGMA)
        srv.submit(host[N], tag=999999)  # warm the buffers of the longest length
        srv.poll(timeout_ms=120000)
        ts0 = time.perf_counter()
        for i, n in enumerate(lens):
            srv.submit(host[int(n)], tag=i)
        lats = []
        for _ in range(args.served):
            r = srv.poll(timeout_ms=120000)
            lats.append(r[3])
        ts = time.perf_counter() - ts0
        srv.close()
        out["served"] = {"value": round(args.served / ts, 3), "unit": "DM trials/s",
                         "requests": args.served, "mix": "20/30/50 % of 2^21/2^22/2^23 samples",
                         "arrival": "all submitted at once (saturated); host series, PCIe copy included",
                         "latency_ms": {"p50": round(1e3 * float(np.percentile(lats, 50)), 2),
                                        "p99": round(1e3 * float(np.percentile(lats, 99)), 2)}}

    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nbytes

    bank.close()
    if not args.plain_only and args.cpu_bins > 0:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(trials[0], args.cpu_bins)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
