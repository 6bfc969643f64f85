"""heget_xsec_device_noalloc (the cross section on the library's static
workspace) against heget_xsec_device on the same configurations.

Both run the same kernels in the same launch configuration, so the result
records must agree bit for bit (stronger than the sigma bars).  Each case makes
two calls in a row, the second with fewer points, so stale workspace contents
from the larger call would show.
"""
import pytest

pytestmark = pytest.mark.gpu


def _H():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_0908_4403_amd as H
    return torch, H


def _pair(torch, H, n, cfg):
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    H.xsec_device(n, cfg, a)
    H.xsec_device_noalloc(n, cfg, b)
    torch.cuda.synchronize()
    return H.result_from_bytes(a.cpu().numpy()), H.result_from_bytes(b.cpu().numpy())


CASES = [
    # (n, prec name, mode, sqrt_s, lo, hi, first npoints, second npoints, sampling)
    (4, "FP32", 0, 1000.0, 0.0, 0.0, 1 << 18, 1 << 14, 0),
    (2, "FP64", 0, 500.0, 0.0, 0.0, 1 << 18, 3000, 0),
    (5, "FP32", 2, 14000.0, 150.0, 0.0, 1 << 16, 777, 0),
    (6, "FP64", 1, 0.0, 200.0, 2000.0, 1 << 12, 1 << 9, 0),
    (8, "FP32", 0, 2000.0, 0.0, 0.0, 1 << 11, 300, 0),
    (3, "FP32", 0, 1000.0, 0.0, 0.0, 1 << 17, 5000, 1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}_{c[1]}_mode{c[2]}_s{c[8]}")
def test_noalloc_matches_xsec_device(case):
    torch, H = _H()
    n, prec, mode, sqrt_s, lo, hi, np1, np2, samp = case
    for k, npts in enumerate((np1, np2)):
        print(f"noalloc case n={n} {prec} mode={mode} npoints={npts} sampling={samp}", flush=True)
        cfg = H.Config(mode=mode, prec=getattr(H, prec), seed=17 + k, npoints=npts, sqrt_s=sqrt_s,
                       sqrt_shat_lo=lo, sqrt_shat_hi=hi, pt_min=20.0, eta_max=2.5, dr_min=0.4,
                       helicity_sampling=samp)
        want, got = _pair(torch, H, n, cfg)
        assert got["n_gen"] == want["n_gen"] == npts
        assert got["n_acc"] == want["n_acc"] > 0
        for key in ("sigma_fb", "err_fb", "sum_w", "sum_w_comp", "sum_w2"):
            assert got[key] == want[key], (key, got, want)


def test_noalloc_refuses_more_than_its_workspace():
    torch, H = _H()
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    cfg = H.Config(prec=H.FP32, seed=1, npoints=1 << 20, sqrt_s=1000.0)
    with pytest.raises(RuntimeError, match="static workspace"):
        H.xsec_device_noalloc(4, cfg, out)
    # the library stays usable after the refusal
    small = H.Config(prec=H.FP32, seed=1, npoints=1 << 12, sqrt_s=1000.0)
    H.xsec_device_noalloc(4, small, out)
    torch.cuda.synchronize()
    assert H.result_from_bytes(out.cpu().numpy())["n_gen"] == 1 << 12
