"""Named synthetic workloads (inputs only; no arithmetic of the method).

Each entry fixes the process, kinematics, sample size, random stream and
cuts of one benchmark workload.  Modes: 0 fixed sqrt(shat), 1 sqrt(shat)
uniform in [lo, hi], 2 pp at hadronic sqrt_s with the toy parton densities.
Cuts are (pT_min [GeV], |eta|_max, Delta R_min); a bound <= 0 is off.
"""

PAPER_CUTS = (20.0, 2.5, 0.4)  # eq. (9)

WORKLOADS = {
    # u ubar -> 2 photons at 500 GeV; the closed-form cross section pins it
    "uubar_2a_500GeV_16k": dict(n=2, mode=0, sqrt_s=500.0, npoints=16384, seed=0,
                                cuts=(20.0, 2.5, 0.0)),
    # u ubar -> 4 photons at 1 TeV: the headline throughput workload
    "uubar_4a_1TeV_2p20": dict(n=4, mode=0, sqrt_s=1000.0, npoints=1 << 20, seed=1,
                               cuts=PAPER_CUTS),
    # pp -> 5 photons at 14 TeV with toy densities, sqrt(shat) >= 150 GeV
    "pp_5a_14TeV_2p22": dict(n=5, mode=2, sqrt_s=14000.0, lo=150.0, npoints=1 << 22, seed=2,
                             cuts=PAPER_CUTS),
    # u ubar -> 8 photons at 2 TeV
    "uubar_8a_2TeV_2p18": dict(n=8, mode=0, sqrt_s=2000.0, npoints=1 << 18, seed=4,
                               cuts=PAPER_CUTS),
}

# mixed batch: n = 2..7 with 2^22 .. 2^17 points, sqrt(shat) uniform in [200 GeV, 2 TeV]
MIXED_BATCH = [dict(n=n, mode=1, lo=200.0, hi=2000.0, npoints=1 << (24 - n), seed=3,
                    cuts=PAPER_CUTS) for n in range(2, 8)]
