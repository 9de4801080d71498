"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use this module.  It widens the stored RF exactly to float64 (FP32 and FP16 by
value, int16 ADC codes as code * dequant_scale) and calls the plain C oracle in
``hodmas_oracle.c``; the product path never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hodmas_oracle.c")
_LIB = os.path.join(_HERE, "libhodmas_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2 + OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, i32, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
        pd = ctypes.POINTER(ctypes.c_double)
        pi32 = ctypes.POINTER(ctypes.c_int32)
        L.hodmas_oracle_tof.restype = d
        L.hodmas_oracle_tof.argtypes = [d, d, d, d, d, d]
        L.hodmas_oracle_sample.restype = d
        L.hodmas_oracle_sample.argtypes = [pd, i64, d]
        L.hodmas_oracle_signed_root.restype = d
        L.hodmas_oracle_signed_root.argtypes = [d, i32]
        L.hodmas_oracle_esym.restype = d
        L.hodmas_oracle_esym.argtypes = [pd, i32, i32]
        L.hodmas_oracle_beamform.restype = i32
        L.hodmas_oracle_beamform.argtypes = [i32, pd, d, d, d, i64, pd, i64,
                                             i32, i32, d, d, d, d, i32, pd]
        L.hodmas_oracle_beamform_weighted.restype = i32
        L.hodmas_oracle_beamform_weighted.argtypes = [i32, pd, d, d, d, i64, pd, i64,
                                                      i32, i32, d, d, d, d, i32, i32, pd]
        L.hodmas_oracle_coherence.restype = d
        L.hodmas_oracle_coherence.argtypes = [pd, i32]
        L.hodmas_oracle_beamform_pixels.restype = i32
        L.hodmas_oracle_beamform_pixels.argtypes = [i32, pd, d, d, d, i64, pd, i64,
                                                    d, d, d, d, i32, i64, pi32, pi32, pd]
        L.hodmas_oracle_max_threads.restype = i32
        L.hodmas_oracle_max_threads.argtypes = []
        L.hodmas_oracle_set_threads.restype = None
        L.hodmas_oracle_set_threads.argtypes = [i32]
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def widen(rf, dequant_scale=None) -> np.ndarray:
    """Stored RF -> float64 exactly: floats by value, int16 codes times the
    (float32) dequantisation scale, the product taken in float64."""
    rf = np.asarray(rf)
    if rf.dtype == np.int16:
        if dequant_scale is None:
            raise ValueError("int16 RF needs a dequant_scale")
        return rf.astype(np.float64) * np.float64(np.float32(dequant_scale))
    if rf.dtype in (np.float16, np.float32, np.float64):
        return rf.astype(np.float64)
    raise TypeError("unsupported RF dtype %s" % rf.dtype)


def element_positions(n_elements: int, pitch: float, element_x=None) -> np.ndarray:
    """Centred uniform linear array at z = 0 unless positions are given."""
    if element_x is not None:
        return np.ascontiguousarray(element_x, dtype=np.float64)
    return (np.arange(n_elements, dtype=np.float64) - (n_elements - 1) / 2.0) * pitch


def tof(xe, xp, zp, c, fs, t0=0.0) -> float:
    return lib().hodmas_oracle_tof(xe, xp, zp, c, fs, t0)


def sample(s, t) -> float:
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib().hodmas_oracle_sample(_pd(s), s.shape[0], t)


def signed_root(v, order) -> float:
    return lib().hodmas_oracle_signed_root(float(v), int(order))


def esym(y, order) -> float:
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().hodmas_oracle_esym(_pd(y), y.shape[0], int(order))


def coherence(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().hodmas_oracle_coherence(_pd(v), v.shape[0])


def beamform(rf, geometry, grid, order, dequant_scale=None, pixels=None, weighting=None):
    """Image [nz][nx] (float64) -- or values at ``pixels`` = (ix, iz) arrays.
    ``weighting="cf"`` multiplies each pixel by its coherence factor (whole
    images only).

    ``geometry``/``grid`` carry the attributes of ``phantom.Geometry`` /
    ``phantom.Grid`` (duck-typed)."""
    x = np.ascontiguousarray(widen(rf, dequant_scale))
    n_el, n_s = x.shape
    ex = element_positions(n_el, geometry.pitch_m, getattr(geometry, "element_x_m", None))
    if ex.shape[0] != n_el:
        raise ValueError("element positions do not match the channel count")
    c, fs, t0 = geometry.sound_speed_m_s, geometry.fs_hz, geometry.t0_s
    L = lib()
    wcode = {None: 0, "cf": 1}[weighting]
    if pixels is None:
        img = np.zeros((grid.nz, grid.nx), dtype=np.float64)
        rc = L.hodmas_oracle_beamform_weighted(n_el, _pd(ex), c, fs, t0, n_s, _pd(x), n_s,
                                               grid.nx, grid.nz, grid.x0_m, grid.dx_m, grid.z0_m,
                                               grid.dz_m, int(order), wcode, _pd(img))
    else:
        if wcode:
            raise ValueError("weighting applies to whole images")
        ix = np.ascontiguousarray(pixels[0], dtype=np.int32)
        iz = np.ascontiguousarray(pixels[1], dtype=np.int32)
        img = np.zeros(ix.shape[0], dtype=np.float64)
        pi32 = ctypes.POINTER(ctypes.c_int32)
        rc = L.hodmas_oracle_beamform_pixels(n_el, _pd(ex), c, fs, t0, n_s, _pd(x), n_s,
                                             grid.x0_m, grid.dx_m, grid.z0_m, grid.dz_m, int(order),
                                             ix.shape[0], ix.ctypes.data_as(pi32),
                                             iz.ctypes.data_as(pi32), _pd(img))
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments (rc=%d)" % rc)
    return img


def max_threads() -> int:
    return int(lib().hodmas_oracle_max_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (timing only; results do not depend on it)."""
    lib().hodmas_oracle_set_threads(int(n))
