"""The measured peaks the bench reports its roofline fractions against as well (needs an
MI355X): each lies between a third of the datasheet value and slightly above it (FP64 matrix
and vector 78.6 TFLOP/s, FP32 matrix 157.3 TFLOP/s, HBM 8 TB/s)."""
import pytest

from test_gpu_parity import torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def test_peak_probe_is_plausible(torch_dev):
    from paper_2508_04370_amd import qdmf as Q
    print("[gpu case] peak probe", flush=True)
    m = Q.qdmf_peak_probe(0, None)
    print("  measured:", m)
    for key, sheet in (("mfma_f64_tflops", 78.6), ("mfma_f32_tflops", 157.3), ("valu_f64_tflops", 78.6),
                       ("hbm_gbs", 8000.0)):
        assert sheet / 3 < m[key] < 1.1 * sheet, (key, m[key])
