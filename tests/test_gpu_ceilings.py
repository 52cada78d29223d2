"""GPU: the VALU ceiling microbenchmarks behind the benchmark's roofline.

The measured rates must be positive, the transcendentals (a wave64
instruction holds its SIMD for twice as long) slower than FP32 FMA, and FP32
FMA with register operands no faster than the unpacked limit of the device
(CUs x 64 lanes x clock, with a 10 % margin for clock reporting).  The
literal-multiplier form is only required to be positive."""
import pytest

from paper_2503_18356_amd import racipe as rp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_valu_ceilings_are_plausible():
    c = rp.valu_ceilings()
    print("[gpu] ceilings (lane-ops/s):", {k: f"{v:.3e}" for k, v in c.items()}, flush=True)
    assert all(v > 1e11 for v in c.values()), c
    for t in ("v_exp_f32", "v_log_f32", "v_rcp_f32"):
        assert c[t] < c["fp32_fma"], (t, c)
    props = torch.cuda.get_device_properties(0)
    clock_hz = 2.4e9  # MI355X peak engine clock; the measured rate must not exceed the unpacked limit
    limit = props.multi_processor_count * 64 * clock_hz * 1.1
    assert c["fp32_fma"] <= limit, (c["fp32_fma"], limit)
