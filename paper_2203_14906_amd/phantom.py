"""Seeded synthetic photoacoustic RF frames (input generator only).

This module produces the inputs that both the GPU path and the CPU oracle
consume.  It models the forward problem only -- point and line absorbers that
emit an N-shaped (Gaussian-derivative) pulse, one-way propagation to a linear
array, 1/r amplitude decay and additive Gaussian channel noise -- and holds
none of the beamforming arithmetic (no delay-and-gather, no roots, no
symmetric sums).

The recipe stands in for the k-Wave simulations and ex-vivo acquisitions of
the paper (Sec. III, Sec. IV), which are not available: homogeneous medium,
128/64/256-element arrays, a 5 MHz pulse, additive noise at a stated SNR and a
frame normalised to max|RF| = 1.  Storage forms: FP32, FP16 (round to nearest
even) and int16 14-bit ADC codes with a seeded full-scale factor.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

SOUND_SPEED = 1540.0        # m/s
FS = 40e6                   # Hz
PITCH = 0.3e-3              # m
PULSE_F0 = 5e6              # Hz, spectral peak of the Gaussian-derivative pulse
ADC_FULL_SCALE = 8191       # 14-bit signed codes


@dataclass
class Geometry:
    n_elements: int
    pitch_m: float = PITCH
    sound_speed_m_s: float = SOUND_SPEED
    fs_hz: float = FS
    t0_s: float = 0.0
    element_x_m: np.ndarray | None = None   # None: centred uniform array at z = 0

    def positions(self) -> np.ndarray:
        if self.element_x_m is not None:
            return np.asarray(self.element_x_m, dtype=np.float64)
        i = np.arange(self.n_elements, dtype=np.float64)
        return (i - (self.n_elements - 1) / 2.0) * self.pitch_m


@dataclass
class Grid:
    nx: int
    nz: int
    x0_m: float
    dx_m: float
    z0_m: float
    dz_m: float


@dataclass
class Frame:
    rf: np.ndarray                  # float64 [N][S], max|rf| = 1
    geometry: Geometry
    grid: Grid
    sources: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))  # (x, z, amplitude)
    seed: int = 0


def field_of_view(n_elements: int, n_samples: int, pitch: float = PITCH):
    """Lateral width W = N * pitch, depth D = 20 mm * S / 1024."""
    return n_elements * pitch, 20e-3 * n_samples / 1024.0


def make_grid(nx: int, nz: int, width: float, depth: float) -> Grid:
    """Pixel centres tile [-W/2, W/2] x [0, D] uniformly."""
    dx = width / nx
    dz = depth / nz
    return Grid(nx=nx, nz=nz, x0_m=-width / 2.0 + dx / 2.0, dx_m=dx, z0_m=dz / 2.0, dz_m=dz)


def _line_sources(rng, width, depth, n_lines, spacing=0.05e-3, thickness=0.2e-3):
    pts = []
    for _ in range(n_lines):
        length = rng.uniform(5e-3, 15e-3)
        angle = rng.uniform(0.0, np.pi)
        cx = rng.uniform(-width / 2.0, width / 2.0)
        cz = rng.uniform(1e-3, depth)
        amp = rng.uniform(0.3, 0.8)
        n_along = max(int(round(length / spacing)), 1)
        along = (np.arange(n_along) - (n_along - 1) / 2.0) * spacing
        n_across = max(int(round(thickness / spacing)), 1)
        across = (np.arange(n_across) - (n_across - 1) / 2.0) * spacing
        a, b = np.meshgrid(along, across, indexing="ij")
        ux, uz = np.cos(angle), np.sin(angle)
        x = cx + a * ux - b * uz
        z = cz + a * uz + b * ux
        keep = (z > 0.5e-3)
        w = np.full(x.shape, amp / n_across)
        pts.append(np.stack([x[keep], z[keep], w[keep]], axis=1))
    if not pts:
        return np.zeros((0, 3))
    return np.concatenate(pts, axis=0)


def synthesize_rf(sources: np.ndarray, elem_x: np.ndarray, n_samples: int,
                  c: float = SOUND_SPEED, fs: float = FS, f0: float = PULSE_F0,
                  half_width: int = 9) -> np.ndarray:
    """Sum of Gaussian-derivative pulses -(A/r) (u/sigma) exp(-u^2 / 2 sigma^2),
    u = t - r/c, one pulse per (source, element) pair, sampled at n/fs."""
    n = elem_x.shape[0]
    rf = np.zeros((n, n_samples), dtype=np.float64)
    if sources.shape[0] == 0:
        return rf
    sigma = 1.0 / (2.0 * np.pi * f0)
    sx, sz, amp = sources[:, 0], sources[:, 1], sources[:, 2]
    r = np.sqrt((sx[:, None] - elem_x[None, :]) ** 2 + sz[:, None] ** 2)   # [M, N]
    arrival = r / c * fs                                                   # samples
    base = np.floor(arrival).astype(np.int64)
    scale = amp[:, None] / (r * 1e3)                                       # 1/r, r in mm
    chan = np.broadcast_to(np.arange(n)[None, :], r.shape)
    for off in range(-half_width, half_width + 1):
        idx = base + off
        u = (idx - arrival) / (sigma * fs)
        val = -scale * u * np.exp(-0.5 * u * u)
        ok = (idx >= 0) & (idx < n_samples)
        flat = chan[ok] * n_samples + idx[ok]
        rf += np.bincount(flat, weights=val[ok], minlength=n * n_samples).reshape(n, n_samples)
    return rf


def add_noise(rf: np.ndarray, snr_db: float, rng) -> np.ndarray:
    """Per-channel white Gaussian noise, sigma_i = rms(clean_i) * 10^(-SNR/20)."""
    rms = np.sqrt(np.mean(rf * rf, axis=1, keepdims=True))
    rms = np.where(rms > 0, rms, np.max(rms) if np.max(rms) > 0 else 1.0)
    return rf + rng.standard_normal(rf.shape) * rms * 10.0 ** (-snr_db / 20.0)


def make_frame(n_elements: int, n_samples: int, nx: int, nz: int, *, n_points: int,
               n_lines: int = 0, snr_db: float = 20.0, seed: int = 0,
               pitch: float = PITCH) -> Frame:
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = Geometry(n_elements=n_elements, pitch_m=pitch)
    width, depth = field_of_view(n_elements, n_samples, pitch)
    px = rng.uniform(-width / 2.0, width / 2.0, n_points)
    pz = rng.uniform(1e-3, depth, n_points)
    pa = rng.uniform(0.5, 1.0, n_points)
    sources = np.stack([px, pz, pa], axis=1) if n_points else np.zeros((0, 3))
    lines = _line_sources(rng, width, depth, n_lines)
    sources = np.concatenate([sources, lines], axis=0)
    rf = synthesize_rf(sources, geom.positions(), n_samples)
    rf = add_noise(rf, snr_db, rng)
    peak = np.max(np.abs(rf))
    if peak > 0:
        rf = rf / peak
    return Frame(rf=rf, geometry=geom, grid=make_grid(nx, nz, width, depth),
                 sources=sources, seed=seed)


def to_fp32(rf: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(rf, dtype=np.float32)


def to_fp16(rf: np.ndarray) -> np.ndarray:
    """IEEE half, round to nearest even (numpy's cast)."""
    return np.ascontiguousarray(rf, dtype=np.float16)


def to_int16(rf: np.ndarray, seed: int):
    """14-bit ADC codes round(rf * u * 8191), u ~ U[0.5, 0.95] seeded.
    Returns (codes int16, dequant_scale float32) with rf ~= codes * scale."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    u = rng.uniform(0.5, 0.95)
    codes = np.clip(np.rint(rf * u * ADC_FULL_SCALE), -ADC_FULL_SCALE, ADC_FULL_SCALE)
    return np.ascontiguousarray(codes.astype(np.int16)), np.float32(1.0 / (u * ADC_FULL_SCALE))


# Workload presets: channel count, samples per channel, grid side, phantom class.
CONFIGS = {
    1: dict(n_elements=64, n_samples=1024, nx=128, nz=128, n_points=5, n_lines=0, snr_db=20.0,
            orders=(1, 2, 3, 4), storage=("f32",)),
    2: dict(n_elements=128, n_samples=2048, nx=512, nz=512, n_points=50, n_lines=3, snr_db=10.0,
            orders=(1, 2, 3, 4, 5, 6), storage=("f32",)),
    3: dict(n_elements=256, n_samples=2048, nx=1024, nz=1024, n_points=50, n_lines=3, snr_db=10.0,
            orders=(1, 2, 3, 4, 5, 6), storage=("i16", "f16")),
}


def config_frame(cfg: int, frame: int = 0) -> Frame:
    p = CONFIGS[cfg]
    return make_frame(p["n_elements"], p["n_samples"], p["nx"], p["nz"], n_points=p["n_points"],
                      n_lines=p["n_lines"], snr_db=p["snr_db"], seed=1000 * cfg + frame)


def mixed_batch_specs(n_frames: int = 256, seed: int = 4000):
    """Frame shapes of the mixed batch: N in {64,128,256}, S in {1024,2048,4096},
    square grid side in {256,512,768,1024}, order in 1..6, uniform and seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for f in range(n_frames):
        specs.append(dict(n_elements=int(rng.choice([64, 128, 256])),
                          n_samples=int(rng.choice([1024, 2048, 4096])),
                          side=int(rng.choice([256, 512, 768, 1024])),
                          order=int(rng.integers(1, 7)),
                          seed=seed + 1 + f))
    return specs
