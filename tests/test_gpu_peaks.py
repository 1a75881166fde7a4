"""The peak probes (hom_peak_probe) return rates in the range an MI355X can reach: each below
1.2x the published peak of its unit and above a floor that only a broken probe would miss."""
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_peak_probes_plausible():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    p = hom.peak_probes()
    say(f"[peaks] {p}")
    bounds = {"hbm_read_gb_s": (1000, 8000 * 1.2), "hbm_write_gb_s": (1000, 8000 * 1.2),
              "fp64_fma_tflops": (10, 78.6 * 1.2), "fp32_fma_tflops": (10, 157.3 * 1.2),
              "fp32_exp2_g_per_s": (100, 1e5), "mfma_f64_tflops": (10, 78.6 * 1.2),
              "mfma_bf16_tflops": (200, 2500 * 1.2), "exp_f64_g_per_s": (10, 1e5),
              "sincos_f64_g_per_s": (10, 1e5)}
    for k, (lo, hi) in bounds.items():
        assert lo <= p[k] <= hi, (k, p[k])
