"""Image-quality metrics on the GPU against the FP64 oracle on the same image,
and the paper's qualitative claim on a synthetic point-target phantom: the
higher orders raise contrast and narrow the lateral profile."""
import sys

import numpy as np
import pytest

from oracle import display as D
from oracle import metrics as M
from paper_2203_14906_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2203_14906_amd import hodmas
    return hodmas


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_metrics(img, dx, t, b, bins):
    snr, cr = M.snr_cr(img, t, b)
    return dict(snr_db=snr, cr_db=cr, gcnr=M.gcnr(img, t, b, bins), fwhm_m=M.fwhm(img, t, dx))


@pytest.mark.parametrize("seed,bins", [(1, 256), (2, 64), (3, 4096)])
def test_metrics_match_oracle(hd, seed, bins):
    rng = np.random.default_rng(seed)
    nz, nx = 120, 150
    img = rng.rayleigh(0.3, (nz, nx)).astype(np.float32)
    zz, xx = np.mgrid[0:nz, 0:nx]
    img += (3.0 * np.exp(-0.5 * (((xx - 70.3) / 2.5) ** 2 + ((zz - 50.0) / 2.0) ** 2))).astype(np.float32)
    t, b = (60, 81, 44, 57), (100, 150, 0, 120)
    got = hd.image_metrics(torch.from_numpy(img).cuda(), 0.1e-3, t, b, bins)
    ref = oracle_metrics(img.astype(np.float64), 0.1e-3, t, b, bins)
    say("seed %d bins %d: %s" % (seed, bins, {k: round(got[k], 6) for k in ref}))
    for k, v in ref.items():
        assert got[k] == pytest.approx(v, rel=1e-9, abs=1e-12), k


def test_higher_orders_raise_contrast_and_narrow_targets(hd):
    # one point absorber in noise, envelope images per order
    n, S = 128, 2048
    geom = ph.Geometry(n)
    src = np.array([[0.0, 20e-3, 1.0]])
    rf = ph.synthesize_rf(src, geom.positions(), S)
    rng = np.random.default_rng(9)
    rf = rf + rng.standard_normal(rf.shape) * np.sqrt(np.mean(rf ** 2)) * 10 ** (-20 / 20)
    rf = (rf / np.abs(rf).max()).astype(np.float32)
    grid = ph.Grid(nx=160, nz=128, x0_m=-6e-3, dx_m=0.075e-3, z0_m=15.2e-3, dz_m=0.075e-3)
    plan = hd.Plan(geom, grid, S, "f32", max_order=5)
    disp = hd.Display(grid.nx, grid.nz, grid.dz_m, 1540.0, 2e6, 9e6, 63, 60.0)
    dev = torch.from_numpy(rf).cuda()
    iz0 = int(round((20e-3 - grid.z0_m) / grid.dz_m))
    ix0 = int(round((0.0 - grid.x0_m) / grid.dx_m))
    t = (ix0 - 6, ix0 + 7, iz0 - 6, iz0 + 7)
    b = (0, 40, 0, 128)
    res = {}
    for k in (1, 2, 3, 5):
        img = plan.beamform(dev, k)
        env = torch.empty_like(img)
        disp.run(img, env)
        res[k] = hd.image_metrics(env, grid.dx_m, t, b, 256)
        say("order %d: SNR %.1f dB  CR %.1f dB  gCNR %.3f  FWHM %.3f mm" %
            (k, res[k]["snr_db"], res[k]["cr_db"], res[k]["gcnr"], res[k]["fwhm_m"] * 1e3))
    assert res[5]["cr_db"] > res[2]["cr_db"] > res[1]["cr_db"]
    assert res[5]["fwhm_m"] < res[1]["fwhm_m"]
    disp.close()
    plan.close()
