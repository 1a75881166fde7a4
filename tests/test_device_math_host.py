"""Accuracy of the FP64 exponential and sine/cosine of the evaluation's terms (hom_device.h:
exp_eval, sincos_turns), measured on the host against long-double libm over the argument ranges
the kernels give them: e^x for x in [-745, 300] (shifted term magnitudes, with the lag margin
above 0), sin and cos of 2 pi t for t in [-1/2, 1/2] (phases reduced to half a turn).

Both functions are __host__ __device__ and compiled from the same header for the GPU; the host
build here uses the same source with the host compiler's IEEE double arithmetic and fused
multiply-adds, as the device code does."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def measured(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("devmath") / "device_math_host")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                           "-ffp-contract=fast", "-I",
                           os.path.join(ROOT, "paper_2111_14317_amd", "csrc"),
                           os.path.join(HERE, "device_math_host.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    out = subprocess.check_output([exe, "4000000"], text=True).split()
    return {out[i]: float(out[i + 1]) for i in range(0, len(out), 2)}


def test_exp_within_one_ulp(measured):
    print(measured)
    assert measured["exp_max_ulp"] <= 1.0
    assert measured["exp_subnormal_max_abs"] <= 2.0 ** -1073  # at most one subnormal step


def test_sincos_within_two_and_a_half_ulp(measured):
    assert measured["sin_max_ulp"] <= 2.5
    assert measured["cos_max_ulp"] <= 2.5


def test_special_arguments(measured):
    assert measured["special_ok"] == 1
