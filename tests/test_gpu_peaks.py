"""The measured-peak probes return plausible rates for an MI355X-class device
and keep their expected order (plain FP32 faster than transcendentals)."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    assert torch.cuda.is_available()
    from paper_2203_14906_amd import hodmas
    p = hodmas.measure_peaks()
    print(p, flush=True)
    assert p["compute_units"] >= 1
    per_cu = {k: p[k] / p["compute_units"] for k in ("fp32_add", "fp32_fma", "fp32_fma_sgpr", "exp2", "log2",
                                                      "sqrt", "rcp")}
    # lane-operations per CU per second: at most 4 SIMDs x 64 lanes x 3 GHz
    for k, v in per_cu.items():
        assert 0.0 < v <= 4 * 64 * 3e9 / 1e12, k
    for t in ("exp2", "log2", "sqrt", "rcp"):
        assert p[t] < p["fp32_add"]
    assert 0.5 < p["hbm_copy_tb_s"] < 20.0
    # the bitwise class issues no faster than FP32 adds; the inner-loop mix
    # costs between one and ten cycles per instruction (27 per element)
    assert 0.0 < p["int_bfi"] <= p["fp32_add"] * 1.05 and 0.0 < p["fract"] <= p["fp32_add"] * 1.05
    for k in ("loop_cycles_sgpr", "loop_cycles_vgpr"):
        assert 27.0 < p[k] < 270.0, k
