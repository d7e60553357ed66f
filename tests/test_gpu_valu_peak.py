"""GPU: the vector FMA rate measurement (measurement support for the
roofline): positive, below the published peaks (FP32 157.3 TFLOP/s assumes
packed FP32, which the build disables, so at most about half of it is
attainable; FP64 78.6 TFLOP/s), and argument errors."""
import pytest

pytestmark = pytest.mark.gpu


def test_fma_rates_are_plausible():
    import paper_1305_6861_amd as ps
    with ps.Context() as ctx:
        f32, f64 = ctx.valu_peak(32), ctx.valu_peak(64)
        print(f"[valu] FMA rate FP32 {f32:.1f} TFLOP/s, FP64 {f64:.1f} TFLOP/s", flush=True)
        assert 10.0 < f32 <= 157.3 * 0.55
        assert 10.0 < f64 <= 78.6 * 1.05
        with pytest.raises(ps.PsError) as ei:
            ctx.valu_peak(16)
        assert ei.value.status == 1
