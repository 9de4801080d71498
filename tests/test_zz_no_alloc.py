"""hodmas_display_run_static -- the display chain without a plan and without
any allocation (its scratch is a fixed device array of the library) -- called
through the C ABI and checked against the plan entry point hodmas_display_run
and against the FP64 oracle to the display chain's bars (envelope 1e-5
relative L2, dB within 1e-3 dB away from the clipping floor), on two calls in
a row, the second with a smaller image, so the second reads nothing the first
left behind in the shared array."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import display as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_ENV = 1e-5
TOL_DB = 1e-3
C = 1540.0


@pytest.fixture(scope="module")
def hd():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2203_14906_amd import hodmas
    return hodmas


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(g, o):
    return np.linalg.norm(g - o) / np.linalg.norm(o)


def static_call(hd, img, dz, f_lo, f_hi, numtaps, dr, with_env=True):
    """The C entry point, arguments marshalled by hand (no plan, no allocation
    inside the call: the outputs are allocated here beforehand)."""
    nz, nx = img.shape
    desc = hd.DisplayDesc(nx, nz, dz, C, f_lo, f_hi, numtaps, dr)
    env = torch.full_like(img, float("nan")) if with_env else None
    db = torch.full_like(img, float("nan"))
    torch.cuda.synchronize()
    st = hd.lib.hodmas_display_run_static(ctypes.byref(desc), ctypes.c_void_p(img.data_ptr()),
                                          ctypes.c_void_p(env.data_ptr()) if env is not None else None,
                                          ctypes.c_void_p(db.data_ptr()), None)
    assert st == hd.OK, hd.status_string(st)
    torch.cuda.synchronize()
    return (env.cpu().numpy().astype(np.float64) if env is not None else None), db.cpu().numpy().astype(np.float64)


def plan_call(hd, img, dz, f_lo, f_hi, numtaps, dr):
    nz, nx = img.shape
    disp = hd.Display(nx, nz, dz, C, f_lo, f_hi, numtaps, dr)
    env, db = disp.run(img, torch.empty_like(img))
    torch.cuda.synchronize()
    disp.close()
    return env.cpu().numpy().astype(np.float64), db.cpu().numpy().astype(np.float64)


def check(env, db, env_ref, db_ref, dr, what):
    err_env = rel_l2(env, env_ref) if env is not None else 0.0
    open_ = db_ref > -dr + 0.01
    err_db = np.abs(db - db_ref)[open_].max() if open_.any() else 0.0
    say("%-48s envelope rel L2 %.2e, dB max err %.2e" % (what, err_env, err_db))
    assert err_env <= TOL_ENV, what
    assert err_db <= TOL_DB, what
    clipped = db_ref < -dr - 0.01
    assert np.all(db[clipped] == -dr), what


@pytest.mark.parametrize("first,second", [((512, 512), (256, 37)), ((1024, 130), (64, 5))])
def test_static_display_two_calls_second_smaller(hd, first, second):
    rng = np.random.default_rng(first[0] + second[1])
    dz, f_lo, f_hi, nt, dr = 0.075e-3, 2e6, 8e6, 63, 60.0
    for shape in (first, second):
        host = rng.standard_normal(shape).astype(np.float32)
        img = torch.from_numpy(host).cuda()
        env, db = static_call(hd, img, dz, f_lo, f_hi, nt, dr)
        env_p, db_p = plan_call(hd, img, dz, f_lo, f_hi, nt, dr)
        _, env_o, db_o = D.display(host.astype(np.float64), dz, C, f_lo, f_hi, nt, dr)
        same = np.array_equal(env, env_p) and np.array_equal(db, db_p)
        say("static display %s: bitwise equal to the plan path: %s" % (shape, same))
        check(env, db, env_p, db_p, dr, "static vs plan entry point %s" % (shape,))
        check(env, db, env_o, db_o, dr, "static vs oracle %s" % (shape,))


def test_static_display_in_place_db_and_limits(hd):
    rng = np.random.default_rng(3)
    host = rng.standard_normal((128, 64)).astype(np.float32)
    img = torch.from_numpy(host).cuda()
    dz, f_lo, f_hi, nt, dr = 0.05e-3, 3e6, 9e6, 31, 50.0
    _, db = static_call(hd, img, dz, f_lo, f_hi, nt, dr, with_env=False)
    _, env_o, db_o = D.display(host.astype(np.float64), dz, C, f_lo, f_hi, nt, dr)
    check(None, db, env_o, db_o, dr, "static, dB only (in place)")
    # refused on the host before any launch
    L = hd.lib
    out = torch.empty_like(img)
    p_img, p_out = ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(out.data_ptr())
    big = hd.DisplayDesc(65537, 128, dz, C, f_lo, f_hi, nt, dr)
    assert L.hodmas_display_run_static(ctypes.byref(big), p_img, None, p_out, None) == hd.EUNSUPPORTED
    odd = hd.DisplayDesc(64, 100, dz, C, f_lo, f_hi, nt, dr)
    assert L.hodmas_display_run_static(ctypes.byref(odd), p_img, None, p_out, None) == hd.EINVAL
    ok = hd.DisplayDesc(64, 128, dz, C, f_lo, f_hi, nt, dr)
    assert L.hodmas_display_run_static(ctypes.byref(ok), p_img, None, p_img, None) == hd.EINVAL
    assert L.hodmas_display_run_static(None, p_img, None, p_out, None) == hd.EINVAL
    even = hd.DisplayDesc(64, 128, dz, C, f_lo, f_hi, 30, dr)
    assert L.hodmas_display_run_static(ctypes.byref(even), p_img, None, p_out, None) == hd.EINVAL
