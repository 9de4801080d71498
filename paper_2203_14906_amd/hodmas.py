"""Thin ctypes binding of ``libhodmas.so`` (declared in ``include/hodmas.h``).

Argument marshalling only: every step of the beamforming runs in the HIP
library.  Device memory and streams come from PyTorch (``torch.Tensor`` on a
ROCm device, ``torch.cuda.Stream``); nothing here computes image values.
If the library is missing this module raises on import -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhodmas.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBUSY = range(6)
F32, F16, I16 = 0, 1, 2
MAX_ORDER = 6
FLAG_ACC_PLAIN = 0x1
FLAG_HOST_ONLY = 0x2
FLAG_FORCE_CHECK = 0x4
FLAG_TUNE_BATCH = 0x8
FLAG_CF = 0x10
FLAG_MIRROR = 0x20
FLAG_NO_SHARE = 0x40
INFO_SHARED_DELAYS = 0x10000

_DTYPE_NAMES = {"f32": F32, "f16": F16, "i16": I16, "float32": F32, "float16": F16, "int16": I16}


class HodmasError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, status_string(status), status))


class Geometry(ctypes.Structure):
    _fields_ = [("n_elements", ctypes.c_int32), ("pitch_m", ctypes.c_double),
                ("sound_speed_m_s", ctypes.c_double), ("fs_hz", ctypes.c_double),
                ("t0_s", ctypes.c_double), ("element_x_m", ctypes.POINTER(ctypes.c_double))]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("x0_m", ctypes.c_double),
                ("dx_m", ctypes.c_double), ("z0_m", ctypes.c_double), ("dz_m", ctypes.c_double)]


class RfDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("channel_stride", ctypes.c_int64), ("dequant_scale", ctypes.c_float),
                ("frame_max", ctypes.c_float)]


class Tiling(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("split", ctypes.c_int32), ("chunk", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_elements", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("max_order", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("tiling", Tiling), ("n_tiles", ctypes.c_int32), ("max_window", ctypes.c_int32),
                ("active_pairs", ctypes.c_int64), ("lds_bytes", ctypes.c_int64),
                ("table_bytes", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class TileDesc(ctypes.Structure):
    _fields_ = [("ix0", ctypes.c_int32), ("iz0", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("n_active", ctypes.c_int32), ("window", ctypes.c_int32),
                ("check", ctypes.c_int32), ("first_entry", ctypes.c_int32),
                ("xa", ctypes.c_double), ("za", ctypes.c_double)]


class ChanEntry(ctypes.Structure):
    _fields_ = [("a", ctypes.c_float), ("d0sq", ctypes.c_float), ("d0", ctypes.c_float),
                ("frac0", ctypes.c_float), ("lo", ctypes.c_float), ("hi", ctypes.c_float),
                ("off", ctypes.c_int32), ("channel", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("n_units", ctypes.c_int64), ("grid", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int64), ("pixel_channels", ctypes.c_int64)]


class StageEntry(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_int32), ("first_sample", ctypes.c_int32)]


class Rect(ctypes.Structure):
    _fields_ = [("ix0", ctypes.c_int32), ("ix1", ctypes.c_int32), ("iz0", ctypes.c_int32),
                ("iz1", ctypes.c_int32)]


class Metrics(ctypes.Structure):
    _fields_ = [("snr_db", ctypes.c_double), ("cr_db", ctypes.c_double), ("gcnr", ctypes.c_double),
                ("fwhm_m", ctypes.c_double), ("mu_in", ctypes.c_double), ("mu_out", ctypes.c_double),
                ("sigma_out", ctypes.c_double)]


class Peaks(ctypes.Structure):
    _fields_ = [("fp32_add", ctypes.c_double), ("fp32_fma", ctypes.c_double), ("fp32_fma_sgpr", ctypes.c_double),
                ("exp2", ctypes.c_double), ("log2", ctypes.c_double), ("sqrt", ctypes.c_double),
                ("rcp", ctypes.c_double), ("hbm_copy_tb_s", ctypes.c_double), ("compute_units", ctypes.c_int32),
                ("int_bfi", ctypes.c_double), ("fract", ctypes.c_double), ("loop_cycles_sgpr", ctypes.c_double),
                ("loop_cycles_vgpr", ctypes.c_double)]


class DisplayDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("dz_m", ctypes.c_double),
                ("sound_speed_m_s", ctypes.c_double), ("f_lo_hz", ctypes.c_double),
                ("f_hi_hz", ctypes.c_double), ("numtaps", ctypes.c_int32),
                ("dynamic_range_db", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhodmas.so is not built (run __graft_entry__.build() or "
                          "python paper_2203_14906_amd/build.py)")
    # One process must hold one HIP runtime.  PyTorch ships its own
    # libamdhip64; loading it first makes libhodmas.so bind to that copy, so
    # tensors from torch and pointers handed to the library belong to the same
    # runtime (loading the library first maps the system runtime beside
    # torch's, and device copies then fail).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
    L.hodmas_plan.restype = i32
    L.hodmas_plan.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Grid), ctypes.POINTER(RfDesc),
                              i32, u32, ctypes.POINTER(Tiling), ctypes.POINTER(vp)]
    L.hodmas_beamform.restype = i32
    L.hodmas_beamform.argtypes = [vp, vp, i32, vp, vp]
    L.hodmas_beamform_orders.restype = i32
    L.hodmas_beamform_orders.argtypes = [vp, vp, i32, ctypes.POINTER(vp), vp]
    L.hodmas_destroy.restype = i32
    L.hodmas_destroy.argtypes = [vp]
    L.hodmas_status_string.restype = ctypes.c_char_p
    L.hodmas_status_string.argtypes = [i32]
    L.hodmas_plan_get_info.restype = i32
    L.hodmas_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.hodmas_plan_tables.restype = i32
    L.hodmas_plan_tables.argtypes = [vp, ctypes.POINTER(ctypes.POINTER(TileDesc)),
                                     ctypes.POINTER(ctypes.POINTER(ChanEntry)),
                                     ctypes.POINTER(ctypes.POINTER(StageEntry)),
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]
    L.hodmas_batch_create.restype = i32
    L.hodmas_batch_create.argtypes = [i32, ctypes.c_int64, ctypes.c_int64, u32, ctypes.POINTER(vp)]
    L.hodmas_batch_set.restype = i32
    L.hodmas_batch_set.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                   ctypes.POINTER(vp), i32, vp]
    L.hodmas_batch_launch.restype = i32
    L.hodmas_batch_launch.argtypes = [vp, vp]
    L.hodmas_batch_capture.restype = i32
    L.hodmas_batch_capture.argtypes = [vp]
    L.hodmas_batch_replay.restype = i32
    L.hodmas_batch_replay.argtypes = [vp, vp]
    L.hodmas_batch_get_info.restype = i32
    L.hodmas_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.hodmas_batch_destroy.restype = i32
    L.hodmas_batch_destroy.argtypes = [vp]
    L.hodmas_autotune.restype = i32
    L.hodmas_autotune.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Grid), ctypes.POINTER(RfDesc),
                                  i32, u32, ctypes.c_char_p, ctypes.POINTER(Tiling)]
    L.hodmas_version.restype = ctypes.c_char_p
    L.hodmas_version.argtypes = []
    L.hodmas_display_taps.restype = i32
    L.hodmas_display_taps.argtypes = [ctypes.POINTER(DisplayDesc), ctypes.POINTER(ctypes.c_double)]
    L.hodmas_display_plan.restype = i32
    L.hodmas_display_plan.argtypes = [ctypes.POINTER(DisplayDesc), ctypes.POINTER(vp)]
    L.hodmas_display_run.restype = i32
    L.hodmas_display_run.argtypes = [vp, vp, vp, vp, vp]
    L.hodmas_display_destroy.restype = i32
    L.hodmas_display_destroy.argtypes = [vp]
    L.hodmas_display_run_batch.restype = i32
    L.hodmas_display_run_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
    L.hodmas_display_run_static.restype = i32
    L.hodmas_display_run_static.argtypes = [ctypes.POINTER(DisplayDesc), vp, vp, vp, vp]
    L.hodmas_image_metrics.restype = i32
    L.hodmas_image_metrics.argtypes = [vp, i32, i32, ctypes.c_double, ctypes.POINTER(Rect), ctypes.POINTER(Rect),
                                       i32, vp, ctypes.POINTER(Metrics)]
    L.hodmas_sync.restype = i32
    L.hodmas_sync.argtypes = [vp]
    L.hodmas_measure_peaks.restype = i32
    L.hodmas_measure_peaks.argtypes = [ctypes.POINTER(Peaks), vp]
    return L


lib = _load()


def status_string(status: int) -> str:
    return lib.hodmas_status_string(int(status)).decode()


def version() -> str:
    return lib.hodmas_version().decode()


def _check(status, what):
    if status != OK:
        raise HodmasError(status, what)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _c_structs(geometry, grid, n_samples, dtype, dequant_scale, frame_max, channel_stride):
    n = int(geometry.n_elements)
    ex = getattr(geometry, "element_x_m", None)
    keep = None
    g = Geometry(n, float(geometry.pitch_m), float(geometry.sound_speed_m_s), float(geometry.fs_hz),
                 float(geometry.t0_s), None)
    if ex is not None:
        keep = (ctypes.c_double * n)(*[float(v) for v in ex])
        g.element_x_m = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    gr = Grid(int(grid.nx), int(grid.nz), float(grid.x0_m), float(grid.dx_m), float(grid.z0_m),
              float(grid.dz_m))
    dt = _DTYPE_NAMES[dtype] if isinstance(dtype, str) else int(dtype)
    stride = int(channel_stride if channel_stride is not None else n_samples)
    rd = RfDesc(dt, int(n_samples), stride, float(dequant_scale), float(frame_max))
    return g, gr, rd, keep


def autotune(geometry, grid, n_samples, dtype="f32", order=6, *, dequant_scale=1.0, frame_max=0.0,
             channel_stride=None, flags=0, cache_path=None):
    """Fastest tiling (tile_x, tile_z, split, chunk) for this plan and order,
    measured on the current device (see hodmas_autotune)."""
    g, gr, rd, keep = _c_structs(geometry, grid, n_samples, dtype, dequant_scale, frame_max, channel_stride)
    t = Tiling()
    _check(lib.hodmas_autotune(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(rd), int(order), int(flags),
                               cache_path.encode() if cache_path else None, ctypes.byref(t)),
           "hodmas_autotune")
    return (t.tile_x, t.tile_z, t.split, t.chunk)


class Plan:
    """A resident plan: geometry, grid, RF layout and the device delay tables."""

    def __init__(self, geometry, grid, n_samples, dtype="f32", *, max_order=MAX_ORDER,
                 dequant_scale=1.0, frame_max=0.0, channel_stride=None, flags=0, tiling=None):
        self.n_elements = int(geometry.n_elements)
        self.n_samples = int(n_samples)
        self.nx, self.nz = int(grid.nx), int(grid.nz)
        self.dtype = _DTYPE_NAMES[dtype] if isinstance(dtype, str) else int(dtype)
        self.channel_stride = int(channel_stride if channel_stride is not None else n_samples)
        self.max_order = int(max_order)
        ex = getattr(geometry, "element_x_m", None)
        self._ex = None
        g = Geometry(self.n_elements, float(geometry.pitch_m), float(geometry.sound_speed_m_s),
                     float(geometry.fs_hz), float(geometry.t0_s), None)
        if ex is not None:
            self._ex = (ctypes.c_double * self.n_elements)(*[float(v) for v in ex])
            g.element_x_m = ctypes.cast(self._ex, ctypes.POINTER(ctypes.c_double))
        gr = Grid(self.nx, self.nz, float(grid.x0_m), float(grid.dx_m), float(grid.z0_m),
                  float(grid.dz_m))
        rd = RfDesc(self.dtype, self.n_samples, self.channel_stride, float(dequant_scale),
                    float(frame_max))
        til = None
        if tiling is not None:
            til = ctypes.byref(Tiling(*[int(v) for v in tiling]))
        handle = ctypes.c_void_p()
        _check(lib.hodmas_plan(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(rd), self.max_order,
                               int(flags), til, ctypes.byref(handle)), "hodmas_plan")
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self) -> PlanInfo:
        inf = PlanInfo()
        _check(lib.hodmas_plan_get_info(self._h, ctypes.byref(inf)), "hodmas_plan_get_info")
        return inf

    def tables(self):
        """Host copies of the plan tables as lists of ctypes records."""
        t = ctypes.POINTER(TileDesc)()
        e = ctypes.POINTER(ChanEntry)()
        s = ctypes.POINTER(StageEntry)()
        nt, ne = ctypes.c_int32(), ctypes.c_int64()
        _check(lib.hodmas_plan_tables(self._h, ctypes.byref(t), ctypes.byref(e), ctypes.byref(s),
                                      ctypes.byref(nt), ctypes.byref(ne)), "hodmas_plan_tables")
        return t[:nt.value], e[:ne.value], s[:ne.value]

    def beamform(self, rf, order, out=None, stream=None):
        """Beamform ``rf`` (device tensor [N][stride] of the plan's dtype) at
        ``order`` into ``out`` (device float32 [nz][nx]); returns ``out``."""
        import torch
        if out is None:
            out = torch.empty((self.nz, self.nx), dtype=torch.float32, device=rf.device)
        _check_tensor(rf, self)
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != self.nx * self.nz:
            raise ValueError("out must be a contiguous float32 tensor of nz*nx elements")
        if not out.is_cuda:
            raise ValueError("out must live on the GPU")
        _check(lib.hodmas_beamform(self._h, ctypes.c_void_p(rf.data_ptr()), int(order),
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "hodmas_beamform")
        return out

    def beamform_orders(self, rf, max_order, outs=None, stream=None):
        """Orders 1..max_order of ``rf`` in one pass; returns the list of images
        (``outs[k-1]`` receives order k)."""
        import torch
        _check_tensor(rf, self)
        if outs is None:
            outs = [torch.empty((self.nz, self.nx), dtype=torch.float32, device=rf.device)
                    for _ in range(max_order)]
        if len(outs) < max_order:
            raise ValueError("need one output image per order")
        for o in outs[:max_order]:
            if o.dtype != torch.float32 or not o.is_contiguous() or o.numel() != self.nx * self.nz or not o.is_cuda:
                raise ValueError("each output must be a contiguous float32 GPU tensor of nz*nx elements")
        ptrs = (ctypes.c_void_p * max_order)(*[o.data_ptr() for o in outs[:max_order]])
        _check(lib.hodmas_beamform_orders(self._h, ctypes.c_void_p(rf.data_ptr()), int(max_order), ptrs,
                                          _stream_handle(stream)), "hodmas_beamform_orders")
        return outs[:max_order]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.hodmas_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many frames (own plan, order, storage each) in one persistent launch."""

    def __init__(self, max_frames, max_units, max_lds_bytes=0, flags=0):
        h = ctypes.c_void_p()
        _check(lib.hodmas_batch_create(int(max_frames), int(max_units), int(max_lds_bytes), int(flags),
                                       ctypes.byref(h)), "hodmas_batch_create")
        self._h = h
        self._keep = None

    def set(self, plans, rfs, orders, images, stream=None):
        n = len(plans)
        if not (len(rfs) == len(orders) == len(images) == n):
            raise ValueError("plans, rfs, orders and images must have the same length")
        for p, r, o in zip(plans, rfs, images):
            _check_tensor(r, p)
            if not o.is_cuda or o.dtype.__str__() != "torch.float32" or not o.is_contiguous() or \
                    o.numel() != p.nx * p.nz:
                raise ValueError("each image must be a contiguous float32 GPU tensor of nz*nx elements")
        ph = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
        pr = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rfs])
        po = (ctypes.c_int32 * n)(*[int(k) for k in orders])
        pi = (ctypes.c_void_p * n)(*[o.data_ptr() for o in images])
        _check(lib.hodmas_batch_set(self._h, ph, pr, po, pi, n, _stream_handle(stream)),
               "hodmas_batch_set")
        self._keep = (list(plans), list(rfs), list(images))   # keep the memory alive

    def launch(self, stream=None):
        _check(lib.hodmas_batch_launch(self._h, _stream_handle(stream)), "hodmas_batch_launch")

    def capture(self):
        _check(lib.hodmas_batch_capture(self._h), "hodmas_batch_capture")

    def replay(self, stream=None):
        _check(lib.hodmas_batch_replay(self._h, _stream_handle(stream)), "hodmas_batch_replay")

    def info(self) -> BatchInfo:
        inf = BatchInfo()
        _check(lib.hodmas_batch_get_info(self._h, ctypes.byref(inf)), "hodmas_batch_get_info")
        return inf

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.hodmas_batch_destroy(self._h)
        self._h = ctypes.c_void_p()
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_TORCH_DT = {F32: "float32", F16: "float16", I16: "int16"}


def _check_tensor(rf, plan):
    import torch
    if not rf.is_cuda:
        raise ValueError("rf must live on the GPU")
    if str(rf.dtype).split(".")[-1] != _TORCH_DT[plan.dtype]:
        raise ValueError("rf dtype %s does not match the plan (%s)" % (rf.dtype, _TORCH_DT[plan.dtype]))
    if rf.dim() != 2 or rf.shape[0] != plan.n_elements or rf.stride(1) != 1 or \
            rf.stride(0) != plan.channel_stride or rf.shape[1] < plan.n_samples:
        raise ValueError("rf must be [n_elements][>= n_samples] with row stride %d" % plan.channel_stride)
    return torch


def _display_desc(nx, nz, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps, dynamic_range_db):
    return DisplayDesc(int(nx), int(nz), float(dz_m), float(sound_speed_m_s), float(f_lo_hz), float(f_hi_hz),
                       int(numtaps), float(dynamic_range_db))


def display_taps(nz, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps, nx=1, dynamic_range_db=60.0):
    """The band-pass taps the display chain uses (host computation)."""
    d = _display_desc(nx, nz, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps, dynamic_range_db)
    out = (ctypes.c_double * max(1, int(numtaps)))()
    _check(lib.hodmas_display_taps(ctypes.byref(d), out), "hodmas_display_taps")
    return [out[i] for i in range(int(numtaps))]


def display_static(image, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps=63, dynamic_range_db=60.0,
                   envelope=None, db=None, stream=None):
    """hodmas_display_run_static: the display chain of one image without a
    plan; its scratch is a fixed device array of the library.  The outputs
    must be given (this call allocates nothing)."""
    import torch
    if db is None:
        raise ValueError("db must be given: this call allocates nothing")
    for t in (image, envelope, db):
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                              or t.dim() != 2 or tuple(t.shape) != tuple(image.shape)):
            raise ValueError("images must be contiguous float32 GPU tensors [nz][nx] of one shape")
    nz, nx = image.shape
    d = _display_desc(nx, nz, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps, dynamic_range_db)
    _check(lib.hodmas_display_run_static(ctypes.byref(d), ctypes.c_void_p(image.data_ptr()),
                                         ctypes.c_void_p(envelope.data_ptr()) if envelope is not None else None,
                                         ctypes.c_void_p(db.data_ptr()), _stream_handle(stream)),
           "hodmas_display_run_static")
    return envelope, db


class Display:
    """Display chain of beamformed images [nz][nx]: band-pass along depth,
    Hilbert envelope, log compression (see hodmas_display_run)."""

    def __init__(self, nx, nz, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps=63, dynamic_range_db=60.0):
        self.nx, self.nz = int(nx), int(nz)
        d = _display_desc(nx, nz, dz_m, sound_speed_m_s, f_lo_hz, f_hi_hz, numtaps, dynamic_range_db)
        self._h = ctypes.c_void_p()
        _check(lib.hodmas_display_plan(ctypes.byref(d), ctypes.byref(self._h)), "hodmas_display_plan")

    def run(self, image, envelope=None, db=None, stream=None):
        """Returns (envelope or None, dB image); allocates outputs not given."""
        import torch
        for t in (image, envelope, db):
            if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                                  or tuple(t.shape) != (self.nz, self.nx)):
                raise ValueError("images must be contiguous float32 GPU tensors [nz][nx]")
        if db is None:
            db = torch.empty_like(image)
        _check(lib.hodmas_display_run(self._h, ctypes.c_void_p(image.data_ptr()),
                                      ctypes.c_void_p(envelope.data_ptr()) if envelope is not None else None,
                                      ctypes.c_void_p(db.data_ptr()), _stream_handle(stream)),
               "hodmas_display_run")
        return envelope, db

    def run_batch(self, images, envelopes=None, dbs=None, stream=None):
        """The chain over a list of images of this shape (up to 16 per launch
        pair).  Returns (envelopes or None, dB images); allocates the dB
        images not given."""
        import torch
        n = len(images)
        if n < 1 or (envelopes is not None and len(envelopes) != n) or (dbs is not None and len(dbs) != n):
            raise ValueError("images, envelopes and dbs must be non-empty lists of one length")
        if dbs is None:
            dbs = [torch.empty_like(im) for im in images]
        for t in list(images) + list(dbs) + list(envelopes or []):
            if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                                  or tuple(t.shape) != (self.nz, self.nx)):
                raise ValueError("images must be contiguous float32 GPU tensors [nz][nx]")
        arr = ctypes.c_void_p * n
        pi = arr(*[im.data_ptr() for im in images])
        pd = arr(*[d.data_ptr() for d in dbs])
        pe = arr(*[(e.data_ptr() if e is not None else None) for e in envelopes]) if envelopes is not None else None
        _check(lib.hodmas_display_run_batch(self._h, pi, pe, pd, n, _stream_handle(stream)),
               "hodmas_display_run_batch")
        return envelopes, dbs

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.hodmas_display_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def image_metrics(image, dx_m, target, background, bins=256, stream=None):
    """SNR, CR, gCNR and FWHM of an envelope image (a [nz][nx] float32 GPU
    tensor); target and background are (ix0, ix1, iz0, iz1) pixel rectangles."""
    import torch
    if image.dtype != torch.float32 or not image.is_cuda or not image.is_contiguous() or image.dim() != 2:
        raise ValueError("image must be a contiguous float32 GPU tensor [nz][nx]")
    nz, nx = image.shape
    t, b, m = Rect(*[int(v) for v in target]), Rect(*[int(v) for v in background]), Metrics()
    _check(lib.hodmas_image_metrics(ctypes.c_void_p(image.data_ptr()), int(nx), int(nz), float(dx_m),
                                    ctypes.byref(t), ctypes.byref(b), int(bins), _stream_handle(stream),
                                    ctypes.byref(m)), "hodmas_image_metrics")
    return {f: getattr(m, f) for f, _ in Metrics._fields_}


def measure_peaks(stream=None):
    """Measured VALU issue rates (1e12 lane-operations/s) and HBM copy rate
    (1e12 B/s) of the current device (see hodmas_measure_peaks)."""
    p = Peaks()
    _check(lib.hodmas_measure_peaks(ctypes.byref(p), _stream_handle(stream)), "hodmas_measure_peaks")
    return {f: getattr(p, f) for f, _ in Peaks._fields_}


def sync(stream=None):
    """Wait for `stream` and raise HodmasError if its work or an earlier
    asynchronous launch failed (see hodmas_sync)."""
    _check(lib.hodmas_sync(_stream_handle(stream)), "hodmas_sync")
