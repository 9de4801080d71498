"""Display chain on the GPU against the FP64 oracle on the same input image:
envelope within 1e-5 relative L2 (FP32 FIR and FFT), dB image within 1e-3 dB
away from the clipping floor and clipped where the oracle is clipped."""
import sys

import numpy as np
import pytest

from oracle import display as D
from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_ENV = 1e-5
TOL_DB = 1e-3


@pytest.fixture(scope="module")
def hd():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2203_14906_amd import hodmas
    return hodmas


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_both(hd, img, dz, f_lo, f_hi, numtaps, dr, with_env=True):
    nz, nx = img.shape
    disp = hd.Display(nx, nz, dz, 1540.0, f_lo, f_hi, numtaps, dr)
    dev = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    env = torch.full_like(dev, float("nan")) if with_env else None
    env, db = disp.run(dev, env)
    torch.cuda.synchronize()
    _, env_o, db_o = D.display(img.astype(np.float32).astype(np.float64), dz, 1540.0, f_lo, f_hi, numtaps, dr)
    disp.close()
    return (env.cpu().numpy().astype(np.float64) if env is not None else None), \
        db.cpu().numpy().astype(np.float64), env_o, db_o


def check_db(db, db_o, dr, what):
    floor = -dr
    open_ = db_o > floor + 0.01
    err = np.abs(db - db_o)[open_].max() if open_.any() else 0.0
    say("%-40s dB max err %.2e over %d pixels" % (what, err, int(open_.sum())))
    assert err <= TOL_DB, what
    clipped = db_o < floor - 0.01
    assert np.all(db[clipped] == floor), what
    assert db.max() <= 0.0 and db.min() >= floor


@pytest.mark.parametrize("nz,nx", [(2, 5), (64, 37), (512, 130), (1024, 3), (8192, 4), (256, 1)])
def test_random_images(hd, nz, nx):
    rng = np.random.default_rng(nz + nx)
    img = rng.standard_normal((nz, nx))
    dz = 0.075e-3
    numtaps = min(63, 2 * (nz // 2) - 1) if nz > 2 else 1
    env, db, env_o, db_o = run_both(hd, img, dz, 2e6, 8e6, numtaps, 60.0)
    err = np.linalg.norm(env - env_o) / np.linalg.norm(env_o)
    say("random %dx%d taps %d: envelope rel L2 %.2e" % (nz, nx, numtaps, err))
    assert err <= TOL_ENV
    check_db(db, db_o, 60.0, "random %dx%d" % (nz, nx))


def test_beamformed_image_and_in_place_db(hd):
    # a GPU-beamformed config-1 image (DAS and DMAS-3) through the display chain
    f = ph.config_frame(1)
    arr = ph.to_fp32(f.rf)
    plan = hd.Plan(f.geometry, f.grid, arr.shape[1], "f32", max_order=4)
    dev = torch.from_numpy(arr).cuda()
    for k in (1, 3):
        img = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
        # config 1 samples depth at 0.156 mm: c / dz = 9.9 MHz, so the band is 1-4 MHz
        env, db, env_o, db_o = run_both(hd, img, f.grid.dz_m, 1e6, 4e6, 31, 50.0)
        err = np.linalg.norm(env - env_o) / np.linalg.norm(env_o)
        say("config 1 k=%d envelope rel L2 %.2e" % (k, err))
        assert err <= TOL_ENV
        check_db(db, db_o, 50.0, "config 1 k=%d" % k)
        _, db2, _, _ = run_both(hd, img, f.grid.dz_m, 1e6, 4e6, 31, 50.0, with_env=False)
        assert np.array_equal(db, db2)            # dB computed in place over the envelope
    plan.close()


def test_zero_image_and_pure_tone(hd):
    env, db, _, _ = run_both(hd, np.zeros((128, 9)), 0.1e-3, 1e6, 4e6, 15, 40.0)
    assert np.all(env == 0.0) and np.all(db == -40.0)
    # a tone at the band centre: envelope = amplitude away from the ends
    nz, dz = 1024, 0.05e-3
    fs = 1540.0 / dz
    f0 = 5e6
    z = np.arange(nz)
    amps = np.array([0.5, 1.0, 2.0])
    img = amps[None, :] * np.cos(2 * np.pi * f0 / fs * z + 0.2)[:, None]
    env, _, env_o, _ = run_both(hd, img, dz, 3e6, 7e6, 101, 60.0)
    interior = slice(150, nz - 150)
    np.testing.assert_allclose(env[interior], np.broadcast_to(amps, env[interior].shape), rtol=2e-3)
    np.testing.assert_allclose(env, env_o, rtol=0, atol=2e-5 * amps.max())


def test_display_abi_errors(hd):
    import ctypes
    disp = hd.Display(8, 64, 0.1e-3, 1540.0, 1e6, 3e6, 31, 60.0)
    a = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(a.data_ptr())
    L = hd.lib
    assert L.hodmas_display_run(disp.handle, p, None, p, None) == hd.EINVAL     # dB over the input
    assert L.hodmas_display_run(disp.handle, p, p, ctypes.c_void_p(a.data_ptr() + 0), None) == hd.EINVAL
    assert L.hodmas_display_run(disp.handle, None, None, p, None) == hd.EINVAL
    with pytest.raises(ValueError):
        disp.run(torch.zeros((64, 9), dtype=torch.float32, device="cuda"))
    disp.close()


def test_display_batch_equals_single_runs(hd):
    """hodmas_display_run_batch over 21 images (two full launch pairs of 16 and
    a remainder of 5), some with envelope outputs and some without: each image
    equals its own hodmas_display_run bit for bit, and its own maximum sets its
    dB scale (images of very different amplitudes in one launch)."""
    nz, nx, dz = 256, 40, 0.075e-3
    rng = np.random.default_rng(5)
    disp = hd.Display(nx, nz, dz, 1540.0, 2e6, 8e6, 31, 50.0)
    imgs = [torch.from_numpy((rng.standard_normal((nz, nx)) * 10.0 ** (i % 5)).astype(np.float32)).cuda()
            for i in range(21)]
    envs = [torch.full_like(imgs[0], float("nan")) if i % 3 else None for i in range(21)]
    envs_b, dbs_b = disp.run_batch(imgs, envs)
    torch.cuda.synchronize()
    for i, im in enumerate(imgs):
        env1 = torch.empty_like(im)
        _, db1 = disp.run(im, env1)
        torch.cuda.synchronize()
        assert torch.equal(db1, dbs_b[i]), "image %d dB" % i
        if envs[i] is not None:
            assert torch.equal(env1, envs_b[i]), "image %d envelope" % i
    _, db_only = disp.run_batch(imgs[:3])
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(db_only[i], dbs_b[i])
    with pytest.raises(ValueError):
        disp.run_batch([])
    disp.close()
