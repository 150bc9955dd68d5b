#!/usr/bin/env python3
"""Throughput of the FDAS hot path on one MI355X.

Workload (the SKA-shaped single trial): 2^23 float32 samples of seeded white
noise plus 4 injected accelerated pulsars with 8 harmonics each; 201 templates
(z in [-200, 200], step 2); 8192-bin overlap-save segments; harmonic sums over
1/2/4/8/16 harmonics; 6-sigma threshold.  One step = one trial through the
whole path: the series copied from page-locked host memory (fdas_search_host;
the next step's copy overlaps this step's search), real DFT, normalisation,
segment DFTs, template multiply, inverse DFTs, powers, harmonic sums, peaks,
sorted candidates to page-locked host memory.

Prints one JSON line: that plain per-trial rate as ``value`` (and, as
``plain_resident``, the same loop with the series already in HBM), then
  plain_autotuned  the same loop with the segment length and templates per
             block the autotuner picks (fdas_autotune: 1024- to 8192-point
             segments) instead of the named 8192;
  batched    64 distinct trials of 2^23 samples (0-3 pulsars each) through
             fdas_search_batch (graph-captured launches, autotuned segment
             length and templates per block; the persistent form at its own
             tuned shape, 4096 or 8192 points), series resident in HBM, and
             again with the series copied from page-locked host memory
             (PCIe included; the next call's copies overlap the current
             call);
  served     the 6000-request trace (20/30/50 % of 2^21/2^22/2^23 samples,
             Poisson arrivals filling 530 s, 5 % with a pulsar) replayed
             through the continuous-batching server (autotuned shape) from host memory (PCIe
             included): saturated (a bounded number in flight) for
             throughput, and the first requests at their arrival times,
             compressed 10x, for p50/p99 latency;
  small      the 2^17-sample, 101-template single-tone configuration: per-call
             latency (launch-bound);
  refine     Fourier interpolation and candidate refinement: the 256 most
             significant records of the trial refined by fdas_refine, and
             the small configuration with every candidate refined;
  template_sweep  the plain rate at 51, 101, 201 and 401 templates;
  interbin   the plain rate with the half-bin plane (2 Nb columns);
  time_domain  the time-domain resampling search on the same trials (201
             acceleration trials, one long DFT each);
  dedisperse the de-dispersion front end: 256 DM trials of a 64-channel
             8-bit filterbank into 2^23-sample series;
  precision  16 trials of 2^22 samples, 801 templates (z in [-400, 400],
             step 1): FP32 FFT correlation against the BF16 and FP16
             matrix-core correlators, with power error and candidate
             agreement against the FP64 oracle on a band of bins;
the roofline of the dominant kernel (the fused multiply / inverse DFT / power
kernel, timed with HIP events on its own stream over 20 searches of the same
trial, which also give ``stages_ms``: the events add gaps between the stages'
kernels, so the plain loops time the path without them); the
whole path against the HBM roof (``path_roofline``: the bytes the method must
move per trial, series in, spectrum out and back, plane out and back, times
the trial rate, over 8 TB/s) for the plain, batched and served rates; and the
FP64 CPU oracle timed on a bounded sample of the same trial.
"""
from __future__ import annotations

import argparse
import gc
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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1511_07343_amd", "csrc", f)
                  for f in ("kernels.hip", "fft_wg.hpp", "device_common.hpp")]


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
    """Algorithmic HBM bytes of one fused-correlation launch: the plane and its
    2-bin block codes written once (4 nz Nb + nz Nb / 2), the segment spectra
    (8 nseg S) and the bank (8 nz S) read once."""
    return 4.0 * nz * nb + 0.5 * nz * nb + 8.0 * nseg * S + 8.0 * nz * S


def path_bytes(nsamp: int, nz: int) -> float:
    """Algorithmic HBM bytes of one whole search: the series read (4 N), the
    spectrum written and read once (2 x 8 Nb), the f-fdot plane written once
    and read once by the harmonic sums (2 x 4 nz Nb).  Bank and candidates are
    negligible."""
    nb = nsamp // 2
    return 4.0 * nsamp + 16.0 * nb + 8.0 * nz * nb


def path_roofline(bytes_per_trial: float, trials_per_s: float) -> dict:
    """Whole-path throughput as a fraction of the HBM roof."""
    ach = bytes_per_trial * trials_per_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_trial": round(bytes_per_trial)}


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


def _gen(spec):
    """Worker: one synthetic series (kind, args) -> float32 array."""
    import synth
    kind, a = spec
    if kind == "batch":
        return synth._trial_with_random_pulsars(1 << 23, 1000 + a, None).x
    if kind == "ring":
        n, seed, pulsar = a
        return synth._trial_with_random_pulsars(n, seed, 1 if pulsar else 0).x
    raise ValueError(kind)


def generate(specs, workers: int = 16):
    """Series for `specs`, generated in a process pool (before any GPU use)."""
    import multiprocessing as mp
    workers = max(1, min(workers, len(os.sched_getaffinity(0)), len(specs)))
    if workers == 1:
        return [_gen(sp) for sp in specs]
    pool = mp.get_context("fork").Pool(workers)
    try:
        return pool.map(_gen, specs)
    finally:
        # close and join (not terminate) so that no worker outlives the call
        pool.close()
        pool.join()


RING = 8            # distinct host series per length class in the served replay
HOST_COPIES = 4     # page-locked copies of the trial cycled by the headline loop
STAGE_STEPS = 20    # searches of the trial timed stage by stage with HIP events
C4_LENGTHS = (1 << 21, 1 << 22, 1 << 23)


def bench_batched(fdas, bank, xs, per_call: int, tuned, tuned_p, host=None):
    """64 distinct trials through fdas_search_batch, per_call trials per call,
    the series resident in HBM, in both launch forms: the default (per-trial
    graphs on two streams) and the persistent kernel (one launch per call of
    up to 64 trials); with `host` (the same series in host memory) also the
    default form with the series first copied from page-locked host memory
    (PCIe included): calls of per_call / 2 trials, each call's copies
    overlapping the previous call's search on a second stream."""
    import numpy as np
    import torch
    seg_b, tpb_b, tune_ms = tuned
    seg_p, tpb_p, tune_p = tuned_p
    log(f"batched: {len(xs)} trials, {per_call} per call, segment {seg_b}, {tpb_b} templates per block "
        f"(persistent form: {seg_p}, {tpb_p})")
    bcap = 1 << 19
    bout = fdas.pinned_candidates(bcap * per_call)
    # the persistent kernel first, at the shape tuned over its own segment lengths
    plans = fdas.Plan(bank, N, seg_p, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb_p,
                      batch_launch="persistent")
    ref = [c.copy() for c in plans.search_batch(xs[:per_call], caps=[bcap] * per_call, out=bout)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(0, len(xs), per_call):
        chunk = xs[i:i + per_call]
        plans.search_batch(chunk, caps=[bcap] * len(chunk), out=bout)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    plans.close()
    persistent = {"value": round(len(xs) / ts, 3), "unit": "DM trials/s", "ms_per_trial": round(1e3 * ts / len(xs), 4),
                  "segment": seg_p, "templates_per_block": tpb_p,
                  "segment_dft_plus_correlate_ms": round(tune_p, 4),
                  "launch": "one persistent-kernel launch per call of up to 64 trials "
                            "(fdas_opts.batch_launch = FDAS_BATCH_PERSISTENT)"}
    # the default form at the persistent form's shape gives the same records
    chk = fdas.Plan(bank, N, seg_p, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb_p)
    got_p = chk.search_batch(xs[:per_call], caps=[bcap] * per_call, out=bout)
    persistent["same_records_as_default"] = all(np.array_equal(a, b) for a, b in zip(got_p, ref))
    chk.close()
    planb = fdas.Plan(bank, N, seg_b, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb_b)
    got = planb.search_batch(xs[:per_call], caps=[bcap] * per_call, out=bout)  # allocates
    counts = [len(c) for c in got]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(0, len(xs), per_call):
        chunk = xs[i:i + per_call]
        planb.search_batch(chunk, caps=[bcap] * len(chunk), out=bout)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    h2d = None
    if host is not None:
        # calls of half the trials; each call's series copied from page-locked
        # host memory on a second stream (default priority), the next call's
        # copies overlapping the current call's search; a buffer is refilled
        # only after the search that read it has finished
        hc = max(1, per_call // 2)
        staged = [torch.from_numpy(x).pin_memory() for x in host]  # new page-locked copies
        bufs = [[torch.empty_like(xs[0]) for _ in range(hc)] for _ in range(2)]
        main, side = torch.cuda.current_stream(), torch.cuda.Stream()
        loaded = [torch.cuda.Event(), torch.cuda.Event()]
        freed = [torch.cuda.Event(), torch.cuda.Event()]
        chunks = [staged[i:i + hc] for i in range(0, len(staged), hc)]

        def load(ci):
            b = ci % 2
            with torch.cuda.stream(side):
                if ci >= 2:
                    side.wait_event(freed[b])
                for d, hx in zip(bufs[b], chunks[ci]):
                    d.copy_(hx, non_blocking=True)
                loaded[b].record(side)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        load(0)
        for ci in range(len(chunks)):
            b = ci % 2
            main.wait_event(loaded[b])
            if ci + 1 < len(chunks):
                load(ci + 1)
            n = len(chunks[ci])
            planb.search_batch(bufs[b][:n], caps=[bcap] * n, out=bout)
            freed[b].record(main)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        h2d = {"value": round(len(staged) / th, 3), "unit": "DM trials/s",
               "ms_per_trial": round(1e3 * th / len(staged), 4), "trials_per_call": hc,
               "data": f"the same {len(staged)} series copied from page-locked host memory, {hc} per call, the "
                       "next call's copies overlapping the current call on a second stream"}
        del staged, bufs
    planb.close()
    return {"value": round(len(xs) / tb, 3), "unit": "DM trials/s", "trials": len(xs),
            "h2d_included": h2d,
            "trials_per_call": per_call, "ms_per_trial": round(1e3 * tb / len(xs), 4),
            "launch": "per-trial graphs on two streams (fdas_opts.batch_launch = FDAS_BATCH_STREAMS, the default)",
            "persistent": persistent,
            "candidates_per_trial": {"min": min(counts), "max": max(counts), "mean": round(sum(counts) / len(counts), 1)},
            "data": "64 distinct trials, seeds 1000-1063, 0-3 pulsars each, resident in HBM",
            "autotuned": {"segment": seg_b, "templates_per_block": tpb_b,
                          "segment_dft_plus_correlate_ms": round(tune_ms, 4)},
            "path_roofline": path_roofline(path_bytes(N, bank.nz), len(xs) / tb)}


def bench_plain_resident(plan, x, out_buf, steps: int):
    """The plain per-trial loop on the same trial with the series already
    resident in HBM (no host-to-device copy): fdas_search per step,
    candidates to page-locked host memory."""
    import torch
    plan.search(x, out=out_buf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.search(x, out=out_buf)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"value": round(1.0 / dt, 3), "unit": "DM trials/s", "steps": steps, "ms_per_step": round(1e3 * dt, 4),
            "data": "the same SKA-shaped trial, series resident in HBM (fdas_search)"}


def _replay(fdas, srv, trace, ring, paced_speedup, inflight):
    """Submit the trace's requests (from the ring of host series) and collect
    results.  paced_speedup > 0: request i is submitted at t_arrival / speedup;
    else as soon as fewer than `inflight` are outstanding.  Returns
    (wall seconds, latencies in s, candidates found, and the records of the
    first request with a pulsar of each length)."""
    import numpy as np
    lat, found = [], 0
    keep = {}  # tag -> length, for the first pulsar request of each length
    kept = {}
    t0 = time.perf_counter()
    nxt = 0
    done = 0
    slot = {n: 0 for n in C4_LENGTHS}
    while done < len(trace):
        while nxt < len(trace):
            e = trace[nxt]
            if paced_speedup > 0:
                if time.perf_counter() - t0 < e["t_arrival"] / paced_speedup:
                    break
            elif nxt - done >= inflight:
                break
            n = e["nsamp"]
            if e["has_pulsar"]:
                x = ring[n][0]
                if n not in keep.values():
                    keep[nxt] = n
            else:
                x = ring[n][1 + slot[n] % (RING - 1)]
                slot[n] += 1
            srv.submit(x, tag=nxt)
            nxt += 1
        r = srv.poll(timeout_ms=1)
        if r is None:
            continue
        lat.append(r[3])
        found += r[2]
        done += 1
        if r[0] in keep:
            kept[keep[r[0]]] = r[1]
    return time.perf_counter() - t0, np.asarray(lat), found, kept


def bench_plain_tuned(fdas, bank, host, out_buf, steps: int, seg: int, tpb: int):
    """The headline's plain loop (fdas_search_host per trial: the series
    copied from page-locked host memory, the next copy overlapping the search,
    the records to page-locked memory) with the segment length and templates
    per block the autotuner picked instead of the named 8192-bin segments."""
    import torch
    plan = fdas.Plan(bank, N, seg, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb)
    for i in range(3):
        plan.search_host(host[i % HOST_COPIES], next=host[(i + 1) % HOST_COPIES], out=out_buf)
    counts = set()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(3, 3 + steps):
        _, nf = plan.search_host(host[i % HOST_COPIES], next=host[(i + 1) % HOST_COPIES], out=out_buf)
        counts.add(nf)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    plan.close()
    return {"value": round(steps / t, 3), "unit": "DM trials/s", "steps": steps, "ms_per_step": round(1e3 * t / steps, 4),
            "segment": seg, "templates_per_block": tpb, "candidates_per_trial": sorted(counts),
            "data": "the headline's trial and loop (PCIe included) at the autotuned shape"}


def bench_served(fdas, bank, ring, requests: int, paced: int, speedup: float, seg: int, tpb: int):
    """The served trace: saturated replay (throughput) and a paced replay of
    its first `paced` requests at `speedup` x real time (latency), with the
    autotuned segment length and templates per block."""
    import numpy as np
    import synth
    trace = synth.served_trace()[:requests]
    srv = fdas.Server(bank, seg, N, max_slots=4, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb)
    srv.submit(ring[N][1], tag=1 << 40)  # warm the buffers of the longest length
    srv.poll(timeout_ms=120000)
    log(f"served: saturated replay of {len(trace)} requests")
    ts, lat_s, found, kept = _replay(fdas, srv, trace, ring, 0.0, inflight=8)
    # each length's first pulsar request against the same series searched
    # alone with fdas_search (whose candidates the GPU tests compare with
    # the FP64 oracle at these sizes)
    import torch
    same = {}
    for n, recs in sorted(kept.items()):
        pl = fdas.Plan(bank, n, seg, nharm_max=NHARM, sigma=SIGMA, templates_per_block=tpb)
        want, _ = pl.search(torch.from_numpy(ring[n][0]).cuda())
        pl.close()
        same[str(n)] = {"candidates": int(len(recs)), "equal_alone": bool(np.array_equal(recs, want))}
    mean_bytes = sum(path_bytes(e["nsamp"], bank.nz) for e in trace) / len(trace)
    out = {"value": round(len(trace) / ts, 3), "unit": "DM trials/s", "requests": len(trace),
           "segment": seg, "templates_per_block": tpb,
           "path_roofline": path_roofline(mean_bytes, len(trace) / ts),
           "mix": "20/30/50 % of 2^21/2^22/2^23 samples, 5 % with a pulsar",
           "arrival": "saturated: next request submitted while 8 are in flight; host series, PCIe included",
           "data": f"ring of {RING} seeded host series per length (one with a pulsar), recycled",
           "candidates": int(found),
           "served_vs_alone": same,
           "latency_ms": {"p50": round(1e3 * float(np.percentile(lat_s, 50)), 2),
                          "p99": round(1e3 * float(np.percentile(lat_s, 99)), 2)},
           "realtime_need": {"value": round(6000 / 530.0, 3), "unit": "DM trials/s"}}
    if paced > 0:
        sub = trace[:paced]
        log(f"served: {len(sub)} requests paced at {speedup:g}x real time")
        tp, lat_p, _, _ = _replay(fdas, srv, sub, ring, speedup, inflight=1 << 30)
        out["paced"] = {"requests": len(sub), "speedup": speedup,
                        "offered_rate": round(speedup * 6000 / 530.0, 3), "unit": "DM trials/s",
                        "wall_s": round(tp, 3),
                        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat_p, 50)), 2),
                                       "p99": round(1e3 * float(np.percentile(lat_p, 99)), 2)}}
    srv.close()
    return out


def bench_template_sweep(fdas, xs, pinned, steps: int = 8):
    """Plain per-trial rate against the number of templates (z in
    [-zmax, zmax], step 2) at 2^23 samples, 8192-bin segments, 16 harmonics
    (candidates into the same page-locked buffer as the plain loop)."""
    import torch
    out = []
    for zmax in (50.0, 100.0, 200.0, 400.0):
        bank = fdas.make_templates(zmax, DZ)
        plan = fdas.Plan(bank, N, SEG, nharm_max=NHARM, sigma=SIGMA)
        plan.search(xs[0], out=pinned)
        torch.cuda.synchronize()
        plan.enable_timing(True)
        t0 = time.perf_counter()
        for i in range(steps):
            plan.search(xs[i % len(xs)], out=pinned)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st, nt = plan.stage_times()
        out.append({"templates": bank.nz, "value": round(1.0 / dt, 3), "unit": "DM trials/s",
                    "correlate_ms": round(st["correlate"] / nt, 4),
                    "harmonic_sum_ms": round(st["harmonic_sum"] / nt, 4),
                    "realtime_multiple": round(1.0 / dt / (6000 / 530.0), 2)})
        plan.close()
        bank.close()
    return out


def bench_small(fdas, steps: int = 200):
    """The small plain configuration: 2^17 samples with one drifting tone,
    101 templates, 2048-bin segments, one harmonic, 6 sigma (latency per call,
    candidates to the host included: into a page-locked buffer, as in the
    headline loop, and, for comparison, into pageable memory)."""
    import numpy as np
    import torch
    import synth
    x = torch.from_numpy(synth.single_tone_series().x).cuda()
    bank = fdas.make_templates(100.0, DZ)
    plan = fdas.Plan(bank, 1 << 17, 2048, nharm_max=1, sigma=SIGMA)
    pin = fdas.pinned_candidates(1 << 16)

    def run(**kw):
        for _ in range(5):
            plan.search(x, **kw)
        torch.cuda.synchronize()
        lat = []
        for _ in range(steps):
            t0 = time.perf_counter()
            plan.search(x, **kw)
            lat.append(time.perf_counter() - t0)
        return lat

    lat = run(out=pin, cap=1 << 16)
    lat_pageable = run()
    plan.close()
    bank.close()
    return {"value": round(1.0 / float(np.mean(lat)), 3), "unit": "DM trials/s", "calls": steps,
            "records": "page-locked host buffer",
            "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 4),
                           "p99": round(1e3 * float(np.percentile(lat, 99)), 4)},
            "pageable": {"value": round(1.0 / float(np.mean(lat_pageable)), 3),
                         "p50_ms": round(1e3 * float(np.percentile(lat_pageable, 50)), 4)}}


def bench_refine(fdas, plan, x, h: int, top: int = 256, levels: int = 6, reps: int = 5):
    """Candidate refinement on the SKA-shaped trial: the `top` most significant
    records of a plain search refined by fdas_refine (FP64 Fourier
    interpolation, pattern search of `levels` levels), timed per call (H2D
    and D2H of the records included); and the small configuration with every
    candidate refined inside fdas_search."""
    import numpy as np
    import torch
    import synth
    cands, n = plan.search(x)
    sel = cands[np.argsort(-cands["sigma"], kind="stable")[:top]]
    plan.refine(sel, levels)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ref = plan.refine(sel, levels)
    dt = (time.perf_counter() - t0) / reps
    # response evaluations: (1 + 8 levels) points x nharm harmonics x ~2h + 1/2 offsets
    evals = float(np.sum((1 + 8 * levels) * sel["nharm"].astype(np.float64) * (2 * h + 0.5)))
    gain = ref["power"].astype(np.float64) / sel["power"].astype(np.float64)
    out = {"records": int(len(sel)), "of": int(n), "levels": levels, "ms_per_call": round(1e3 * dt, 3),
           "us_per_record": round(1e6 * dt / max(len(sel), 1), 2),
           "response_evals_per_s": round(evals / dt, 1),
           "power_gain": {"median": round(float(np.median(gain)), 4), "max": round(float(np.max(gain)), 4)}}
    xs = torch.from_numpy(synth.single_tone_series().x).cuda()
    bank = fdas.make_templates(100.0, DZ)
    lat = {}
    for lv in (0, levels):
        p = fdas.Plan(bank, 1 << 17, 2048, nharm_max=1, sigma=SIGMA, refine_levels=lv)
        for _ in range(5):
            c, _n = p.search(xs)
        torch.cuda.synchronize()
        t = []
        for _ in range(50):
            s0 = time.perf_counter()
            c, _n = p.search(xs)
            t.append(time.perf_counter() - s0)
        lat[lv] = (float(np.percentile(t, 50)), c)
        p.close()
    bank.close()
    best = lat[levels][1][np.argmax(lat[levels][1]["power"])]
    out["small_in_search"] = {"candidates": int(len(lat[levels][1])),
                              "latency_p50_ms": {"plain": round(1e3 * lat[0][0], 4),
                                                 "refined": round(1e3 * lat[levels][0], 4)},
                              "strongest": {"r": float(best["r"]), "z": float(best["z"]),
                                            "power": float(best["power"]),
                                            "grid_power": float(np.max(lat[0][1]["power"]))}}
    return out


def bench_interbin(fdas, bank, xs, pinned, steps: int = 8):
    """The SKA-shaped trial with the half-bin plane (2 Nb columns: templates
    at integer and half-bin offsets, harmonic sums on half bins)."""
    import numpy as np
    import torch
    plan = fdas.Plan(bank, N, SEG, nharm_max=NHARM, sigma=SIGMA, interbin=True)
    for i in range(2):
        plan.search(xs[i % len(xs)], out=pinned)
    torch.cuda.synchronize()
    plan.enable_timing(True)
    counts = []
    t0 = time.perf_counter()
    for i in range(steps):
        _, n = plan.search(xs[i % len(xs)], out=pinned)
        counts.append(n)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st, nt = plan.stage_times()
    out = {"value": round(1.0 / dt, 3), "unit": "DM trials/s", "steps": steps, "ms_per_step": round(1e3 * dt, 4),
           "plane_columns": plan.plane_columns, "device_bytes": plan.device_bytes,
           "correlate_ms": round(st["correlate"] / nt, 4), "harmonic_sum_ms": round(st["harmonic_sum"] / nt, 4),
           "candidates_per_trial": [int(c) for c in counts[:len(xs)]]}
    plan.close()
    return out


DD_NCHAN, DD_FTOP, DD_FOFF, DD_TSAMP, DD_NDM, DD_DMMAX = 64, 1500.0, 4.0, 64e-6, 256, 500.0


def bench_dedisperse(fdas, steps: int = 3):
    """De-dispersion front end at the SKA series length: a 64-channel 8-bit
    filterbank (1500 MHz top, 4 MHz channels, 64 us samples: 2^23 output
    samples is 537 s), 256 DM trials over [0, 500] pc cm^-3.  The filterbank
    is seeded uniform noise drawn on the device (a timing input; the tests
    check the sums bit for bit on synthetic filterbanks)."""
    import numpy as np
    import torch
    dms = np.linspace(0.0, DD_DMMAX, DD_NDM)
    f_bot = DD_FTOP - DD_FOFF * (DD_NCHAN - 1)
    dmax = int(np.floor(4.148808e3 * DD_DMMAX * (1 / f_bot ** 2 - 1 / DD_FTOP ** 2) / DD_TSAMP + 0.5))
    nsamp = N + dmax
    g = torch.Generator(device="cuda")
    g.manual_seed(6)
    fil = torch.randint(0, 256, (DD_NCHAN, nsamp), dtype=torch.uint8, device="cuda", generator=g)
    out = torch.empty((DD_NDM, N), dtype=torch.float32, device="cuda")
    fdas.dedisperse(fil, DD_FTOP, DD_FOFF, DD_TSAMP, dms, N, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fdas.dedisperse(fil, DD_FTOP, DD_FOFF, DD_TSAMP, dms, N, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    written = DD_NDM * N * 4
    return {"value": round(DD_NDM / dt, 1), "unit": "DM trials/s", "dm_trials": DD_NDM, "channels": DD_NCHAN,
            "nsamp_out": N, "max_delay": dmax, "ms_per_call": round(1e3 * dt, 3),
            "series_written_GBs": round(written / dt / 1e9, 1),
            "channel_bytes_added_per_s": round(DD_NDM * DD_NCHAN * N / dt, 1),
            "data": "seeded uniform 8-bit noise drawn on the device (torch generator, seed 6)"}


TD_ALPHA_MAX, TD_NALPHA = 0.02, 201


def bench_time_domain(fdas, xs, pinned, steps: int = 3):
    """The time-domain resampling search (the other method of Sec. 1) on the
    SKA-shaped trials: 201 acceleration trials |alpha| <= 0.02 (the drift
    relative to the mean frequency; the injected pulsars have |z| / r up to
    0.018), one 2^23-sample resampling and real DFT per trial, harmonic sums
    along each trial's spectrum."""
    import torch
    plan = fdas.TdPlan(N, TD_ALPHA_MAX, TD_NALPHA, nharm_max=NHARM, sigma=SIGMA)
    plan.search(xs[0], out=pinned)
    torch.cuda.synchronize()
    plan.enable_timing(True)
    counts = []
    t0 = time.perf_counter()
    for i in range(steps):
        _, n = plan.search(xs[i % len(xs)], out=pinned)
        counts.append(int(n))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st, nt = plan.stage_times()
    out = {"value": round(1.0 / dt, 3), "unit": "DM trials/s", "steps": steps, "ms_per_step": round(1e3 * dt, 3),
           "trials": TD_NALPHA, "alpha_max": TD_ALPHA_MAX,
           "spectra_ms": round(st["r2c"] / nt, 3), "harmonic_sum_ms": round(st["harmonic_sum"] / nt, 3),
           "candidates_per_trial": counts}
    plan.close()
    return out


C5_ZMAX, C5_DZ, C5_N = 400.0, 1.0, 1 << 22


def bench_precision(fdas, ntrials: int, band: int):
    """C5: the three correlators on 16 trials of 2^22 samples (801 templates);
    power error and candidate agreement against the FP64 oracle on a band of
    `band` bins around the strongest pulsar of the first trial that has one
    (one harmonic, 6 sigma)."""
    import numpy as np
    import torch

    import oracle as O
    import synth
    trials = synth.precision_trials(ntrials)
    xs = [torch.from_numpy(t.x).cuda() for t in trials]
    jref = next((j for j, t in enumerate(trials) if t.pulsars), 0)
    ref = trials[jref]
    nb = C5_N // 2
    taps, zs, h = O.template_taps(C5_ZMAX, C5_DZ)
    centre = int(round(max(ref.pulsars, key=lambda p: p.amp).r)) if ref.pulsars else nb // 3
    k0 = int(min(max(centre - band // 2, h), nb - band - h))
    Xh = O.normalise(O.real_spectrum(ref.x), 1024)
    t0 = time.perf_counter()
    P_orc = O.correlate(Xh[k0 - h:k0 + band + h], taps)[:, h:h + band]
    t_orc = time.perf_counter() - t0
    thr = O.thresholds(SIGMA, [1])[1]
    pk = O.find_peaks(P_orc, thr)
    inner = (pk[:, 1] >= 1) & (pk[:, 1] < band - 1)
    o_set = {(int(iz), int(k) + k0) for iz, k in pk[inner]}
    bank = fdas.make_templates(C5_ZMAX, C5_DZ)
    plane = torch.empty((bank.nz, nb), dtype=torch.float32, device="cuda")
    big = P_orc >= 1.0
    out = {"trials": ntrials, "nsamp": C5_N, "templates": bank.nz, "nharm": 1,
           "oracle_band": {"k0": k0, "bins": band, "trial_seed": ref.seed, "oracle_s": round(t_orc, 2),
                           "oracle_candidates": len(o_set)}}
    for corr in ("fft", "bf16", "f16"):
        plan = fdas.Plan(bank, C5_N, SEG, nharm_max=1, sigma=SIGMA, correlator=corr)
        plan.search(xs[0])
        torch.cuda.synchronize()
        plan.enable_timing(True)
        t0 = time.perf_counter()
        for x in xs:
            plan.search(x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st, nt = plan.stage_times()
        plan.enable_timing(False)
        cands, n = plan.search(xs[jref], plane=plane)
        torch.cuda.synchronize()
        P = plane[:, k0:k0 + band].cpu().numpy().astype(np.float64)
        err = np.abs(P - P_orc)
        rel = err[big] / P_orc[big]
        sel = (cands["nharm"] == 1) & (cands["k"] >= k0 + 1) & (cands["k"] < k0 + band - 1)
        g_set = {(int(c["iz"]), int(c["k"])) for c in cands[sel]}
        both = len(g_set & o_set)
        out[corr] = {"value": round(ntrials / dt, 3), "unit": "DM trials/s",
                     "correlate_ms": round(st["correlate"] / nt, 4),
                     "power_rel_err": {"max": float(rel.max()), "rms": float(np.sqrt(np.mean(rel ** 2))),
                                       "over": "cells with P >= 1 in the band"},
                     "candidates": {"gpu": len(g_set), "oracle": len(o_set), "common": both,
                                    "agreement": round(both / max(1, len(o_set | g_set)), 4)}}
        plan.close()
    del plane
    bank.close()
    return out


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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64, help="trials per fdas_search_batch call")
    ap.add_argument("--batch-trials", type=int, default=64, help="distinct trials in the batched run (0 = skip)")
    ap.add_argument("--served", type=int, default=6000, help="requests of the served trace replayed (0 = skip)")
    ap.add_argument("--paced", type=int, default=1000, help="requests replayed at their arrival times")
    ap.add_argument("--speedup", type=float, default=10.0, help="time compression of the paced replay")
    ap.add_argument("--precision-trials", type=int, default=16, help="trials of the precision comparison (0 = skip)")
    ap.add_argument("--precision-band", type=int, default=65536, help="oracle band of the precision comparison")
    ap.add_argument("--sweep", type=int, default=1, help="template-count sweep 51/101/201/401 (0 = skip)")
    ap.add_argument("--cpu-bins", type=int, default=1 << 17, help="oracle sample width in bins (0 = skip)")
    ap.add_argument("--plain-only", action="store_true", help="only the plain per-trial loop (profiling)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the search runs on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    # host inputs of the batched and served runs, generated in a process pool
    # before anything touches the GPU
    extra = not args.plain_only
    specs = []
    if extra and args.batch_trials > 0:
        specs += [("batch", i) for i in range(args.batch_trials)]
    if extra and args.served > 0:
        specs += [("ring", (n, 60000 + 100 * c + i, i == 0)) for c, n in enumerate(C4_LENGTHS) for i in range(RING)]
    if specs:
        log(f"generating {len(specs)} host series")
    gen = generate(specs)
    batch_host = gen[:args.batch_trials] if extra and args.batch_trials > 0 else []
    ring_host = gen[len(batch_host):]
    ring = {n: ring_host[c * RING:(c + 1) * RING] for c, n in enumerate(C4_LENGTHS)} if ring_host else {}

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
    L = (SEG - 2 * h) & ~3
    nb = N // 2
    nseg = -(-nb // L)
    torch.cuda.synchronize()

    out = pinned = fdas.pinned_candidates(1 << 22)  # page-locked record buffer, reused every step
    # the trial in page-locked host memory, four copies so that consecutive
    # steps read different host buffers; step i searches copy i mod 4 and
    # starts the copy of the next step's series (Sec. 4 step 1, overlapped)
    host = [torch.from_numpy(trials[0].x).pin_memory() for _ in range(HOST_COPIES)]
    # Python's cyclic garbage collector stays off from here on: a full
    # collection over the objects of torch and the host series took ~50 ms
    # once in a while, inside a timed loop
    gc.collect()
    gc.disable()
    log(f"warmup {args.warmup}")
    for i in range(args.warmup):
        plan.search_host(host[i % HOST_COPIES], next=host[(i + 1) % HOST_COPIES], out=out)
    torch.cuda.synchronize()
    lat = []
    counts = set()
    log(f"timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):  # the warm-up staged copy warmup % 4
        s0 = time.perf_counter()
        _, nf = plan.search_host(host[i % HOST_COPIES], next=host[(i + 1) % HOST_COPIES], out=out)
        lat.append(time.perf_counter() - s0)
        counts.add(nf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # Stage times (and the correlation kernel's duration for the roofline)
    # from HIP events in a loop of their own on the same trial: the events put
    # gaps of ~8 us between the stages' kernels, which the timed loops above
    # and below do without.
    xs0 = xs[0]
    plan.enable_timing(True)
    for _ in range(STAGE_STEPS):
        plan.search(xs0, out=out)
    torch.cuda.synchronize()
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
        "config": {"workload": "SKA-shaped single trial (seed 2): 2^23 float32 samples of white noise plus "
                               "4 pulsars x 8 harmonics, 201 templates z in [-200,200] step 2, 8192-bin "
                               "segments, 1/2/4/8/16 harmonic sums, 6 sigma; every step copies the series "
                               "from page-locked host memory (the next step's copy overlapping the search) "
                               "and returns the sorted candidates to page-locked host memory",
                   "nsamp": N, "templates": nz, "segment": SEG, "halfwidth": h, "segments": nseg,
                   "path": "plain (fdas_search_host per trial, host-to-device copy included)",
                   "candidates_per_trial": sorted(counts)},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 4),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 4)},
        "stages_ms": {k: round(v / max(ntimed, 1), 4) for k, v in stages.items()},
        "stages_from": f"{STAGE_STEPS} searches of the same trial, resident in HBM, with HIP events between the stages",
        # the whole path against the HBM roof (bytes the method must move per trial)
        "path_roofline": path_roofline(path_bytes(N, nz), value),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": traffic, "kernel": "k_correlate (fused multiply, inverse DFT, power)",
                     "algorithmic_flops": flops, "launch_ms": round(corr_ms, 4),
                     "hbm_GBs": round(correlate_bytes(nseg, nz, SEG, nb) / (corr_ms * 1e-3) / 1e9, 1)},
    }
    log("plain search with the series resident in HBM")
    out["plain_resident"] = bench_plain_resident(plan, xs[0], pinned, min(args.steps, 50))
    tuned = tuned_p = None
    if extra:
        # segment length and templates per block for the batched and served
        # forms (and the persistent launch, over its own lengths)
        tuned = fdas.autotune(bank, N, nharm_max=NHARM, sigma=SIGMA)
        tuned_p = fdas.autotune(bank, N, nharm_max=NHARM, sigma=SIGMA, batch_launch="persistent")
        log(f"autotuned shape {tuned[0]}-point segments, {tuned[1]} templates per block; plain loop at it")
        out["plain_autotuned"] = bench_plain_tuned(fdas, bank, host, pinned, min(args.steps, 50), tuned[0], tuned[1])
        out["plain_autotuned"]["segment_dft_plus_correlate_ms"] = round(tuned[2], 4)

    if extra:
        log("small configuration latency")
        out["small"] = bench_small(fdas)
        log("candidate refinement")
        out["refine"] = bench_refine(fdas, plan, xs[0], h)

    if extra and args.sweep:
        log("template-count sweep")
        out["template_sweep"] = bench_template_sweep(fdas, xs, pinned)

    if extra:
        log("half-bin plane")
        out["interbin"] = bench_interbin(fdas, bank, xs, pinned)
        log("time-domain resampling search")
        out["time_domain"] = bench_time_domain(fdas, xs, pinned)
        log("de-dispersion front end")
        out["dedisperse"] = bench_dedisperse(fdas)

    if batch_host:
        bxs = [torch.from_numpy(x).to(dev) for x in batch_host]
        out["batched"] = bench_batched(fdas, bank, bxs, args.batch, tuned, tuned_p, host=batch_host)
        del batch_host
        del bxs
    plan.close()

    if ring:
        out["served"] = bench_served(fdas, bank, ring, args.served, args.paced, args.speedup, tuned[0], tuned[1])

    if extra and args.precision_trials > 0:
        log("precision variant: FFT FP32 vs BF16 / FP16 matrix correlators")
        out["precision"] = bench_precision(fdas, args.precision_trials, args.precision_band)

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
