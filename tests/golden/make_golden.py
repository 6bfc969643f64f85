"""Write the stored oracle values the GPU tests compare against.

Calls only the FP64 CPU oracle (oracle/).  Each output file records the
workload, the oracle function used and this command:

    python tests/golden/make_golden.py [name ...]

Files (tests/golden/):
  me2_n7_1500GeV_seed7.txt      |M|^2, sum over orderings, first 48 points passing the cuts
  me2_n8_2TeV_seed4_orderings.txt   the same for n = 8 (first 8 points)
  me2_n8_2TeV_seed4_subsets.txt     n = 8, first 1024 points, subset recursion
  xsec_*.txt                    cross sections of workloads or of their first points
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from workloads import MIXED_BATCH, WORKLOADS  # noqa: E402


def survivors(n, sqrt_s, seed, count, cuts):
    idx = []
    start = 0
    while len(idx) < count:
        ev = O.cm_events(n, sqrt_s, seed, start, 4 * count)
        for i, p in enumerate(ev):
            if O.pass_cuts(p[2:], 0.0, *cuts):
                idx.append(start + i)
        start += ev.shape[0]
    return idx[:count]


def write_me2(fname, n, sqrt_s, seed, count, method):
    cuts = (20.0, 2.5, 0.4)
    idx = survivors(n, sqrt_s, seed, count, cuts)
    ev = np.array([O.cm_event(n, sqrt_s, seed, i) for i in idx])
    t0 = time.time()
    if method == "orderings":
        me, threads = O.me2_batch(ev)
    else:
        me, threads = O.me2_subsets_batch(ev)
    dt = time.time() - t0
    with open(os.path.join(HERE, fname), "w") as f:
        f.write(f"# FP64 oracle |M|^2 (oracle.me2_{'batch' if method == 'orderings' else 'subsets_batch'}, "
                f"{method}) of u ubar -> {n} photons\n")
        f.write(f"# points: oracle.cm_event(n={n}, sqrt_shat={sqrt_s}, seed={seed}, point) for the first "
                f"{count} points passing pT>20, |eta|<2.5, dR>0.4\n")
        f.write(f"# written by: python tests/golden/make_golden.py ({threads} threads, {dt:.0f} s)\n")
        f.write(f"# n={n} sqrt_shat={sqrt_s} seed={seed}\n# point_index me2_GeV^{4 - 2 * n}\n")
        for i, m in zip(idx, me):
            f.write(f"{i} {m:.17g}\n")
    print(fname, f"{dt:.1f}s", flush=True)


def write_xsec(fname, n, mode, sqrt_s, lo, hi, seed, npoints, cuts, method=0, note=""):
    cfg = O.Config(mode=mode, seed=seed, npoints=npoints, sqrt_s=sqrt_s, sqrt_shat_lo=lo,
                   sqrt_shat_hi=hi, pt_min=cuts[0], eta_max=cuts[1], dr_min=cuts[2],
                   me2_method=method)
    t0 = time.time()
    r = O.xsec(n, cfg)
    dt = time.time() - t0
    with open(os.path.join(HERE, fname), "w") as f:
        f.write(f"# FP64 oracle cross section (oracle.xsec, me2_method={method}) {note}\n")
        f.write(f"# written by: python tests/golden/make_golden.py ({r['threads']} threads, {dt:.0f} s)\n")
        f.write(f"n {n}\nmode {mode}\nsqrt_s {sqrt_s!r}\nsqrt_shat_lo {lo!r}\nsqrt_shat_hi {hi!r}\n")
        f.write(f"seed {seed}\nnpoints {npoints}\npt_min {cuts[0]!r}\neta_max {cuts[1]!r}\ndr_min {cuts[2]!r}\n")
        for k in ("sigma_fb", "err_fb", "sum_w", "sum_w2"):
            f.write(f"{k} {r[k]:.17g}\n")
        f.write(f"n_gen {r['n_gen']}\nn_acc {r['n_acc']}\n")
    print(fname, f"sigma={r['sigma_fb']:.6g} +- {r['err_fb']:.2g} fb, {dt:.1f}s", flush=True)


def jobs():
    c2 = WORKLOADS["uubar_4a_1TeV_2p20"]
    c3 = WORKLOADS["pp_5a_14TeV_2p22"]
    c5 = WORKLOADS["uubar_8a_2TeV_2p18"]
    J = {
        "me2_n7": lambda: write_me2("me2_n7_1500GeV_seed7.txt", 7, 1500.0, 7, 48, "orderings"),
        "me2_n8_orderings": lambda: write_me2("me2_n8_2TeV_seed4_orderings.txt", 8, 2000.0, 4, 8, "orderings"),
        "me2_n8_subsets": lambda: write_me2("me2_n8_2TeV_seed4_subsets.txt", 8, 2000.0, 4, 1024, "subsets"),
        "xsec_c2": lambda: write_xsec("xsec_uubar_4a_1TeV_2p20.txt", 4, 0, c2["sqrt_s"], 0.0, 0.0,
                                      c2["seed"], c2["npoints"], c2["cuts"], note="full workload"),
        "xsec_c3": lambda: write_xsec("xsec_pp_5a_14TeV_first2p16.txt", 5, 2, c3["sqrt_s"], c3["lo"], 0.0,
                                      c3["seed"], 1 << 16, c3["cuts"], note="first 2^16 points"),
        "xsec_c5": lambda: write_xsec("xsec_uubar_8a_2TeV_first2p12.txt", 8, 0, c5["sqrt_s"], 0.0, 0.0,
                                      c5["seed"], 1 << 12, c5["cuts"], method=1, note="first 2^12 points"),
    }
    prefix = {2: 1 << 16, 3: 1 << 15, 4: 1 << 14, 5: 1 << 13, 6: 1 << 11, 7: 1 << 9}
    for s in MIXED_BATCH:
        n = s["n"]
        J[f"xsec_mixed_n{n}"] = (lambda s=s, n=n: write_xsec(
            f"xsec_mixed_n{n}_first{prefix[n]}.txt", n, 1, 0.0, s["lo"], s["hi"], s["seed"], prefix[n],
            s["cuts"], method=1 if n >= 6 else 0, note=f"mixed batch slice n={n}, first {prefix[n]} points"))
    return J


if __name__ == "__main__":
    J = jobs()
    for name in (sys.argv[1:] or list(J)):
        J[name]()
