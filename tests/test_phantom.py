"""The seeded input generator: determinism, normalisation and storage forms."""
import numpy as np

from paper_2203_14906_amd import phantom as ph


def test_seeded_and_normalised():
    a = ph.make_frame(16, 256, 8, 8, n_points=3, n_lines=1, snr_db=20.0, seed=9)
    b = ph.make_frame(16, 256, 8, 8, n_points=3, n_lines=1, snr_db=20.0, seed=9)
    c = ph.make_frame(16, 256, 8, 8, n_points=3, n_lines=1, snr_db=20.0, seed=10)
    np.testing.assert_array_equal(a.rf, b.rf)
    assert not np.array_equal(a.rf, c.rf)
    assert np.max(np.abs(a.rf)) == 1.0
    assert a.rf.shape == (16, 256)


def test_config_shapes():
    f = ph.config_frame(1)
    assert f.rf.shape == (64, 1024)
    assert (f.grid.nx, f.grid.nz) == (128, 128)
    width, depth = ph.field_of_view(64, 1024)
    assert abs(width - 19.2e-3) < 1e-12 and abs(depth - 20e-3) < 1e-12
    assert abs(f.grid.x0_m + width / 2 - f.grid.dx_m / 2) < 1e-15


def test_storage_forms():
    f = ph.make_frame(8, 128, 4, 4, n_points=2, seed=1)
    h = ph.to_fp16(f.rf)
    assert h.dtype == np.float16
    np.testing.assert_array_equal(h, f.rf.astype(np.float16))
    codes, scale = ph.to_int16(f.rf, seed=1)
    assert codes.dtype == np.int16 and scale.dtype == np.float32
    assert np.abs(codes).max() <= 8191
    err = np.abs(codes * np.float64(scale) - f.rf).max()
    assert err <= 0.5 * float(scale) * 1.0001


def test_mixed_batch_specs():
    specs = ph.mixed_batch_specs()
    assert len(specs) == 256
    assert {s["n_elements"] for s in specs} <= {64, 128, 256}
    assert {s["n_samples"] for s in specs} <= {1024, 2048, 4096}
    assert {s["side"] for s in specs} <= {256, 512, 768, 1024}
    assert {s["order"] for s in specs} == set(range(1, 7))
    assert specs == ph.mixed_batch_specs()
