#!/usr/bin/env python3
"""Throughput of the u ubar -> n photon |M|^2 path on one MI355X.

One step = one heget_xsec pass over a batch of synthetic phase-space points:
counter-based random numbers -> RAMBO -> cuts -> compaction -> helicity-summed
|M|^2 (shared-prefix tree over the n! orderings) -> weights -> compensated
reduction to sigma +- err.  Inputs are generated on the device (nothing is
read from the host inside the timed region).

Default workload: u ubar -> 4 photons at sqrt(shat) = 1 TeV, 2^20 points
(seed 1), pT > 20 GeV, |eta| < 2.5, Delta R > 0.4; amplitudes in FP32 with
FP64 ordering/helicity sums (the FP64-amplitude form is measured beside it).

value = points whose |M|^2 was evaluated (points passing the cuts) per second
of the whole step.  The roofline object is for the amplitude kernel: its
algorithmic flops (heget_me2_flops, counted on the schedule actually run)
times the points per launch, over its average launch time measured with HIP
events on the launch stream.  cpu_baseline times the FP64 CPU oracle
(brute-force ordering sum) on a bounded sample of the same points.  Beside
the headline line: the amplitude kernels alone for n = 2..8 (per_n), the
n = 8 workload (2^18 points at 2 TeV, FP32 and FP64), the mixed n = 2..7
batch, the paper's per-event helicity sampling against the helicity sum
(sigma and its error per unit time), and the per-point error against the
oracle.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X vector peaks (256 CUs at 2.4 GHz): the roofline denominators.
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
# One non-packed FMA per lane per clock (256 CUs x 4 SIMDs x 16 lanes x 2 flop
# x 2.4 GHz), reported beside the published figure for reference only.
NONPACKED_FMA_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def peak_of(prec_name):
    return PEAK_FP32_VECTOR_TFLOPS if prec_name == "fp32" else PEAK_FP64_VECTOR_TFLOPS


def _workloads():
    from workloads import MIXED_BATCH, WORKLOADS
    return WORKLOADS, MIXED_BATCH


def settle(H, torch, n, cfg, ms):
    """Run passes, untimed, for `ms` of wall time: the device raises its clock
    only after some milliseconds of sustained load, so a timed region that
    starts from idle reads 10-15% slow over its first few hundred passes."""
    if ms <= 0:
        return
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(50):
            H.xsec_device(n, cfg, buf)
        torch.cuda.synchronize()


def run_steps(H, torch, n, cfg, steps, warmup, nstreams=1):
    """Enqueue `steps` full passes back to back, step k on stream k mod nstreams
    (the library keeps one scratch set per stream, so passes on different
    streams are independent and the next pass's generation can fill the issue
    slots the current pass's amplitude kernel and small kernels leave idle);
    each writes its result record into its own slot of a device buffer (no
    host callback).  The step time is taken without per-kernel events (an
    event record stalls the stream by a few microseconds); the amplitude kernel
    is then timed over at least 200 further passes, on one stream, with HIP
    events on the launch stream."""
    kreps = max(steps, 200)
    total = warmup + steps + kreps
    buf = torch.zeros((total, 64), dtype=torch.uint8, device="cuda")
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(nstreams - 1)]
    # every stream's first pass sizes its scratch set: keep that out of the timing
    for s in streams[warmup:]:
        H.xsec_device(n, cfg, buf[0], stream=s)
    for k in range(warmup):
        H.xsec_device(n, cfg, buf[k], stream=streams[k % nstreams])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        H.xsec_device(n, cfg, buf[k], stream=streams[k % nstreams])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H.timing_enable(True)
    H.timing_read(reset=True)
    for k in range(warmup + steps, total):
        H.xsec_device(n, cfg, buf[k])
    torch.cuda.synchronize()
    me2_ms, launches = H.timing_read(reset=True)
    H.timing_enable(False)
    host = buf.cpu().numpy()
    res = [H.result_from_bytes(host[k]) for k in range(total)]
    assert all(r == res[0] for r in res), "steps disagree"
    return (t1 - t0) * 1e3 / steps, me2_ms / max(launches, 1), launches, res[0]


def mixed_batch(H, torch, prec, steps):
    """n = 2..7 with 2^22..2^17 points, sqrt(shat) uniform in [200 GeV, 2 TeV]:
    one heget_xsec_batch (persistent amplitude launch, graph-captured) against
    one heget_xsec call per n."""
    _, mixed = _workloads()
    ns = [s["n"] for s in mixed]
    cfgs = [H.Config(mode=s["mode"], prec=prec, seed=s["seed"], npoints=s["npoints"],
                     sqrt_shat_lo=s["lo"], sqrt_shat_hi=s["hi"], pt_min=s["cuts"][0],
                     eta_max=s["cuts"][1], dr_min=s["cuts"][2]) for s in mixed]
    res = H.xsec_batch(ns, cfgs)  # capture + warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        H.xsec_batch(ns, cfgs)
    t_batch = (time.perf_counter() - t0) / steps
    for n, c in zip(ns, cfgs):
        H.xsec(n, c)
    t0 = time.perf_counter()
    for _ in range(steps):
        for n, c in zip(ns, cfgs):
            H.xsec(n, c)
    t_single = (time.perf_counter() - t0) / steps
    acc = sum(r["n_acc"] for r in res)
    gen = sum(c.npoints for c in cfgs)
    schedule = {1: "persistent kernel", 2: "parallel graph branches"}.get(H.batch_schedule_in_use(ns, cfgs))
    return {"workload": "mixed n=2..7, 2^22..2^17 points, sqrt(shat) uniform in [200, 2000] GeV",
            "points_generated": gen, "points_evaluated": acc,
            "batch_ms": t_batch * 1e3, "one_launch_per_n_ms": t_single * 1e3,
            "batch_points_per_s": acc / t_batch, "speedup_vs_per_n": t_single / t_batch,
            "schedule": schedule,
            "sigma_fb": {str(n): r["sigma_fb"] for n, r in zip(ns, res)}}


def per_n(H, torch, tune, ns=range(2, 9)):
    """Amplitude kernel alone (heget_me2_device) for n = 2..8 on device-generated
    points (sqrt(shat) = 1 TeV, seed 11, no cuts so every point is a valid input),
    FP32 and FP64, with HIP-event timing of the kernel on its launch stream."""
    out = []
    for n in ns:
        npts = 1 << {2: 22, 3: 21, 4: 20, 5: 18, 6: 16, 7: 15, 8: 14}[n]
        mom = torch.empty(((n + 2) * 4, npts), dtype=torch.float64, device="cuda")
        w = torch.empty(npts, dtype=torch.float64, device="cuda")
        H.gen_points_device(n, 1000.0, mom, w, None, 11)
        me2 = torch.empty(npts, dtype=torch.float64, device="cuda")
        row = {"n": n, "points": npts}
        for prec, name in ((H.FP32, "fp32"), (H.FP64, "fp64")):
            if tune:
                H.autotune(n, prec, min(npts, 1 << 18))
            # warm-up at the steady clock: launches for at least 100 ms
            t0, launched = time.perf_counter(), 0
            while launched < 3 or time.perf_counter() - t0 < 0.1:
                for _ in range(5):
                    H.me2_device(n, mom, me2, prec)
                torch.cuda.synchronize()
                launched += 5
            per_launch = (time.perf_counter() - t0) / launched
            H.timing_enable(True)
            H.timing_read(reset=True)
            reps = max(3, int(0.05 / per_launch))
            for _ in range(reps):
                H.me2_device(n, mom, me2, prec)
            torch.cuda.synchronize()
            ms, launches = H.timing_read(reset=True)
            H.timing_enable(False)
            ms /= max(launches, 1)
            f, shape = H.me2_flops(n, prec)
            tf = f * npts / (ms * 1e-3) / 1e12
            row[name] = {"points_per_s": npts / (ms * 1e-3), "kernel_ms": ms, "tflops": tf,
                         "frac": tf / peak_of(name), "peak": peak_of(name),
                         "frac_of_nonpacked_fma": tf / NONPACKED_FMA_TFLOPS,
                         "shape": shape, "flops_per_point": f}
        print(f"bench: per-n n={n} FP32 {row['fp32']['points_per_s']:.3e} pts/s "
              f"({row['fp32']['frac']:.2f}), FP64 {row['fp64']['points_per_s']:.3e} "
              f"({row['fp64']['frac']:.2f})", file=sys.stderr, flush=True)
        if n <= 5:
            # the general-frame evaluator composed from the HELAS library, same points
            frame = {}
            for prec, name in ((H.FP32, "fp32"), (H.FP64, "fp64")):
                fn = min(npts, 1 << 18)
                sub = mom[:, :fn].contiguous()
                fout = torch.empty(fn, dtype=torch.float64, device="cuda")
                H.me2_frame_device(n, sub, fout, prec)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    H.me2_frame_device(n, sub, fout, prec)
                e1.record()
                torch.cuda.synchronize()
                fms = e0.elapsed_time(e1) / 3
                frame[name] = {"points": fn, "kernel_ms": fms, "points_per_s": fn / (fms * 1e-3)}
            row["helas_frame"] = frame
            print(f"bench: per-n n={n} HELAS frame evaluator FP32 {frame['fp32']['points_per_s']:.3e} "
                  f"pts/s, FP64 {frame['fp64']['points_per_s']:.3e}", file=sys.stderr, flush=True)
        out.append(row)
        del mom, w, me2
    return out


def cpu_model():
    """Host CPU model name and clock (lscpu, else /proc/cpuinfo)."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    model = info.get("Model name")
    mhz = info.get("CPU max MHz") or info.get("CPU MHz")
    if (model is None or mhz is None) and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model is None:
                model = line.split(":", 1)[1].strip()
            if line.startswith("cpu MHz") and mhz is None:
                mhz = line.split(":", 1)[1].strip()
    return {"model": model, "max_mhz": float(mhz) if mhz else None,
            "logical_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


def _survivors(O, n, sqrt_s, seed, cuts, count, start=0):
    out = []
    while len(out) < count:
        ev = O.cm_events(n, sqrt_s, seed, start, 4 * count)
        start += ev.shape[0]
        out.extend(p for p in ev if O.pass_cuts(p[2:], 0.0, *cuts))
    import numpy as np
    return np.array(out[:count])


def _error_stats(got, ref):
    """Per-point relative error |got/ref - 1|: quantiles and a log10 histogram."""
    import numpy as np
    rel = np.abs(got / ref - 1.0)
    edges = list(range(-17, -2))  # decades 1e-17 .. 1e-3
    lg = np.log10(np.maximum(rel, 1e-300))
    hist = {"below_1e-17": int(np.sum(lg < -17))}
    for lo in edges[:-1]:
        hist[f"1e{lo}..1e{lo + 1}"] = int(np.sum((lg >= lo) & (lg < lo + 1)))
    hist["above_1e-3"] = int(np.sum(lg >= -3))
    return {"points": int(rel.size), "median": float(np.median(rel)),
            "p99": float(np.quantile(rel, 0.99)), "p99_9": float(np.quantile(rel, 0.999)),
            "max": float(rel.max()), "nonfinite": int(np.sum(~np.isfinite(got))),
            "log10_histogram": hist}


def oracle_leg(H, n, wl, budget_s, golden_n8):
    """The FP64 CPU oracle on the host cores: its throughput on a bounded
    sample of the timed workload (all cores, then one core), and the per-point
    error of the device |M|^2 (FP32 and FP64 amplitudes) against it for
    n = 4..8 at the workloads' kinematics."""
    import numpy as np
    import oracle as O

    cuts = wl["cuts"]
    cal = _survivors(O, n, wl["sqrt_s"], wl["seed"], cuts, 256)
    t0 = time.perf_counter()
    O.me2_batch(cal)
    dt = time.perf_counter() - t0
    count = int(min(max(256, budget_s / max(dt, 1e-6) * 256), 1 << 20))
    ev = _survivors(O, n, wl["sqrt_s"], wl["seed"], cuts, count)
    t0 = time.perf_counter()
    ref, threads = O.me2_batch(ev)
    dt_all = time.perf_counter() - t0
    # one core, as the paper's single-threaded CPU program (first points of the same sample)
    O.set_threads(1)
    try:
        rate1 = count / dt_all / max(threads, 1)
        c1 = int(min(count, max(64, 0.5 * budget_s * rate1)))
        t0 = time.perf_counter()
        O.me2_batch(ev[:c1])
        dt_one = time.perf_counter() - t0
    finally:
        O.set_threads(0)
    base = {"value": count / dt_all, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 brute-force |M|^2 (all n! orderings x all helicities) of the first {count} "
                      f"points passing the cuts (seed {wl['seed']}, n={n}, sqrt(shat)={wl['sqrt_s']:.0f} GeV), "
                      f"{dt_all:.1f} s",
            "one_core": {"value": c1 / dt_one, "unit": "points/s", "cores": 1,
                         "sample": f"the first {c1} points of the same sample, {dt_one:.1f} s"},
            "cpu": cpu_model()}

    acc = {}

    def record(key, pts, want, what):
        row = {"what": what}
        for prec, name in ((H.FP32, "fp32"), (H.FP64, "fp64")):
            row[name] = _error_stats(H.me2(pts, prec), want)
        acc[key] = row
        print(f"bench: accuracy {key} FP32 median {row['fp32']['median']:.2e} p99.9 "
              f"{row['fp32']['p99_9']:.2e}; FP64 max {row['fp64']['max']:.2e}", file=sys.stderr, flush=True)

    record(f"n{n}", ev, ref, f"the cpu_baseline sample above ({count} points), brute-force oracle")
    # n = 5..7 at sqrt(shat) = 1 TeV (seed 1, paper cuts): the oracle's subset
    # recursion (equal to the brute-force sum, pinned by the oracle tests)
    for m, cnt in ((5, 4096), (6, 2048), (7, 1024)):
        if m == n:
            continue
        pts = _survivors(O, m, 1000.0, 1, cuts, cnt)
        want, _ = O.me2_subsets_batch(pts)
        record(f"n{m}", pts, want, f"first {cnt} points passing the cuts, n={m}, sqrt(shat)=1 TeV, seed 1, "
                                   "oracle subset recursion")
    # n = 8: the stored oracle values of the first 1024 survivors of the n = 8 workload
    if golden_n8 and os.path.exists(golden_n8):
        idx, want = [], []
        for line in open(golden_n8):
            if line.strip() and not line.startswith("#"):
                a, b = line.split()
                idx.append(int(a))
                want.append(float(b))
        pts = np.array([O.cm_event(8, 2000.0, 4, i) for i in idx])
        record("n8", pts, np.array(want), f"first {len(idx)} survivors of the n=8 workload (2 TeV, seed 4), "
                                          "stored oracle values (tests/golden)")
    return base, acc


def config_n8(H, torch, wl, reps):
    """The n = 8 workload end to end (2^18 points at 2 TeV, paper cuts): FP32 and
    FP64 amplitudes, whole pass and amplitude kernel timed (HIP events on the
    launch stream), with the kernel's roofline against the published peak."""
    n = wl["n"]
    base = dict(mode=wl["mode"], seed=wl["seed"], npoints=wl["npoints"], sqrt_s=wl["sqrt_s"],
                pt_min=wl["cuts"][0], eta_max=wl["cuts"][1], dr_min=wl["cuts"][2])
    out = {"workload": "uubar_8a_2TeV_2p18", "process": "u ubar -> 8 photons", "sqrt_shat_GeV": wl["sqrt_s"],
           "points_generated": wl["npoints"], "seed": wl["seed"],
           "cuts": "pT>%g GeV, |eta|<%g, dR>%g" % tuple(wl["cuts"])}
    for prec, name in ((H.FP32, "fp32"), (H.FP64, "fp64")):
        cfg = H.Config(prec=prec, **base)
        buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
        H.xsec_device(n, cfg, buf)  # sizes scratch, raises the clock
        torch.cuda.synchronize()
        H.timing_enable(True)
        H.timing_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(reps):
            H.xsec_device(n, cfg, buf)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        kms, launches = H.timing_read(reset=True)
        H.timing_enable(False)
        kms /= max(launches, 1)
        r = H.result_from_bytes(buf.cpu().numpy())
        f, shape = H.me2_flops(n, prec)
        ach = f * r["n_acc"] / (kms * 1e-3) / 1e12
        out[name] = {"points_per_s": r["n_acc"] / dt, "ms_per_pass": dt * 1e3, "points_evaluated": r["n_acc"],
                     "sigma_fb": r["sigma_fb"], "sigma_err_fb": r["err_fb"],
                     "roofline": {"bound": "alu", "achieved": ach, "peak": peak_of(name), "unit": "TFLOP/s",
                                  "frac": ach / peak_of(name), "kernel": "me2_kernel<{},8,{}>".format(
                                      "float" if name == "fp32" else "double",
                                      ",".join(str(v) for v in shape)),
                                  "kernel_ms": kms, "flops_per_point": f}}
        print(f"bench: n=8 workload {name} {dt * 1e3:.1f} ms/pass, kernel {kms:.1f} ms, "
              f"{r['n_acc'] / dt:.3e} pts/s, frac {ach / peak_of(name):.2f}", file=sys.stderr, flush=True)
    out["fp32_over_fp64"] = out["fp32"]["points_per_s"] / out["fp64"]["points_per_s"]
    return out


def sampling_leg(H, torch, n, base, reps):
    """The paper's per-event helicities against the helicity sum on one
    workload, FP32 amplitudes: sigma and its Monte-Carlo error per unit time.
    One pass draws one configuration per point (estimator 2^(n+1)|M_h|^2);
    the figure of merit of a mode is 1 / (err^2 * time per pass)."""
    out = {}
    for sampling, name in ((0, "summed"), (1, "sampled")):
        cfg = H.Config(prec=H.FP32, helicity_sampling=sampling, **base)
        buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
        H.xsec_device(n, cfg, buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            H.xsec_device(n, cfg, buf)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        r = H.result_from_bytes(buf.cpu().numpy())
        out[name] = {"ms_per_pass": dt * 1e3, "sigma_fb": r["sigma_fb"], "sigma_err_fb": r["err_fb"],
                     "rel_err": r["err_fb"] / r["sigma_fb"], "merit_per_s": 1.0 / (r["err_fb"] ** 2 * dt)}
    out["sampled_merit_over_summed"] = out["sampled"]["merit_per_s"] / out["summed"]["merit_per_s"]
    print(f"bench: n={n} helicity sampling {out['sampled']['ms_per_pass']:.3f} ms/pass "
          f"(summed {out['summed']['ms_per_pass']:.3f}), rel err {out['sampled']['rel_err']:.2e} "
          f"(summed {out['summed']['rel_err']:.2e}), merit ratio {out['sampled_merit_over_summed']:.2f}",
          file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # a step takes well under a millisecond: enough steps that the timed region
    # sees the device at its steady clock (short runs read 10-15% slower)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="uubar_4a_1TeV_2p20")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and per-point accuracy)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed n=2..7 batch")
    ap.add_argument("--no-n8", action="store_true", help="skip the n=8 workload (2^18 points at 2 TeV)")
    ap.add_argument("--no-sampling", action="store_true",
                    help="skip the helicity-sampling leg (sigma and its error per unit time)")
    ap.add_argument("--no-per-n", action="store_true", help="skip the per-n amplitude kernel timings")
    ap.add_argument("--per-n-list", default="2,3,4,5,6,7,8",
                    help="photon counts of the per-n section (comma-separated)")
    ap.add_argument("--no-tune", action="store_true", help="use the untuned kernel shapes")
    ap.add_argument("--settle-ms", type=float, default=1000.0,
                    help="untimed passes for this long before the warmup steps (clock ramp-up)")
    ap.add_argument("--streams", type=int, default=1,
                    help="consecutive steps go to this many streams in turn (1: one stream)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (scale for rocprofv3 FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the |M|^2 path "
              "has no multi-GPU execution in this library", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0908_4403_amd as H

    workloads, _ = _workloads()
    wl = workloads[args.workload]
    n = wl["n"]
    torch.cuda.set_device(0)
    base = dict(mode=wl["mode"], seed=wl["seed"], npoints=wl["npoints"], sqrt_s=wl["sqrt_s"],
                sqrt_shat_lo=wl.get("lo", 0.0), sqrt_shat_hi=wl.get("hi", 0.0),
                pt_min=wl["cuts"][0], eta_max=wl["cuts"][1], dr_min=wl["cuts"][2])
    tuned = {}
    if not args.no_tune:
        for prec, name in ((H.FP32, "fp32"), (H.FP64, "fp64")):
            tuned[name] = H.autotune(n, prec, min(wl["npoints"], 1 << 18))
        print(f"bench: tuned shapes {tuned}", file=sys.stderr, flush=True)

    if args.copy_calibration:
        from paper_0908_4403_amd.profiling import CALIB_BYTES
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    print(f"bench: {args.workload} FP32 steps={args.steps} warmup={args.warmup} streams={args.streams}",
          file=sys.stderr, flush=True)
    settle(H, torch, n, H.Config(prec=H.FP32, **base), args.settle_ms)
    ms32, k32, l32, r32 = run_steps(H, torch, n, H.Config(prec=H.FP32, **base), args.steps, args.warmup,
                                    args.streams)
    print(f"bench: FP32 {ms32:.3f} ms/step, me2 kernel {k32:.3f} ms", file=sys.stderr, flush=True)
    ms64, k64, l64, r64 = run_steps(H, torch, n, H.Config(prec=H.FP64, **base),
                                    max(3, args.steps // 2), 1, args.streams)
    print(f"bench: FP64 {ms64:.3f} ms/step, me2 kernel {k64:.3f} ms", file=sys.stderr, flush=True)

    n_acc = r32["n_acc"]
    f32, shape32 = H.me2_flops(n, H.FP32)
    f64, shape64 = H.me2_flops(n, H.FP64)
    ach32 = f32 * n_acc / (k32 * 1e-3) / 1e12
    ach64 = f64 * n_acc / (k64 * 1e-3) / 1e12

    mixed = None
    if not args.no_mixed:
        print("bench: mixed n=2..7 batch", file=sys.stderr, flush=True)
        mixed = mixed_batch(H, torch, H.FP32, 3)
        print(f"bench: mixed batch {mixed['batch_ms']:.2f} ms vs per-n {mixed['one_launch_per_n_ms']:.2f} ms",
              file=sys.stderr, flush=True)

    pern = None if args.no_per_n else per_n(H, torch, not args.no_tune,
                                            [int(x) for x in args.per_n_list.split(",")])
    n8 = None if args.no_n8 else config_n8(H, torch, workloads["uubar_8a_2TeV_2p18"], 1)
    sampling = None
    if not args.no_sampling:
        w8 = workloads["uubar_8a_2TeV_2p18"]
        base8 = dict(mode=w8["mode"], seed=w8["seed"], npoints=w8["npoints"], sqrt_s=w8["sqrt_s"],
                     pt_min=w8["cuts"][0], eta_max=w8["cuts"][1], dr_min=w8["cuts"][2])
        sampling = {args.workload: sampling_leg(H, torch, n, base, 50),
                    "uubar_8a_2TeV_2p18": sampling_leg(H, torch, w8["n"], base8, 2)}

    cpu, accuracy = None, None
    if not args.no_cpu_baseline:
        print("bench: oracle leg (cpu baseline, per-point accuracy)", file=sys.stderr, flush=True)
        golden = os.path.join(ROOT, "tests", "golden", "me2_n8_2TeV_seed4_subsets.txt")
        cpu, accuracy = oracle_leg(H, n, wl, args.cpu_seconds, golden)

    peak = H.valu_peak()
    print(f"bench: FMA probe FP32 {peak['fp32_tflops']:.1f}, FP64 {peak['fp64_tflops']:.1f} TFLOP/s",
          file=sys.stderr, flush=True)
    kname = "me2_kernel<float,{},{}>".format(n, ",".join(str(v) for v in shape32))
    from paper_0908_4403_amd.profiling import read_traffic
    traffic_md = os.path.join(ROOT, "profiles", f"me2_kernel_{args.workload}_hbm_traffic.md")
    traffic = read_traffic(traffic_md, kname)

    line = {
        "metric": "phase-space points/s of helicity-summed |M|^2, n=4..8, FP32-batched vs FP64 plain",
        "value": n_acc / (ms32 * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "process": f"u ubar -> {n} photons",
                   "streams": args.streams, "settle_ms": args.settle_ms,
                   "sqrt_shat_GeV": wl["sqrt_s"], "points_generated": wl["npoints"],
                   "points_evaluated": n_acc, "seed": wl["seed"],
                   "cuts": "pT>%g GeV, |eta|<%g, dR>%g" % tuple(wl["cuts"]), "sigma_fb": r32["sigma_fb"],
                   "sigma_err_fb": r32["err_fb"]},
        "roofline": {"bound": "alu", "achieved": ach32, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach32 / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": kname,
                     "kernel_ms": k32,
                     "kernel_share_of_step": k32 / ms32,
                     "flops_per_point": f32,
                     "frac_of_nonpacked_fma": ach32 / NONPACKED_FMA_TFLOPS,
                     "fma_probe_tflops": peak["fp32_tflops"]},
        "fp64_plain": {"value": r64["n_acc"] / (ms64 * 1e-3), "ms_per_step": ms64, "kernel_ms": k64,
                       "achieved_tflops": ach64, "peak": PEAK_FP64_VECTOR_TFLOPS,
                       "frac": ach64 / PEAK_FP64_VECTOR_TFLOPS,
                       "fma_probe_tflops": peak["fp64_tflops"],
                       "sigma_fb": r64["sigma_fb"], "flops_per_point": f64},
        "fp32_over_fp64": (n_acc / ms32) / (r64["n_acc"] / ms64),
        "generated_points_per_s": wl["npoints"] / (ms32 * 1e-3),
        "tuned_shapes": tuned,
        "n8_workload": n8,
        "helicity_sampling": sampling,
        "per_n": pern,
        "mixed_batch": mixed,
        "accuracy_vs_oracle": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
