"""The start-point kernel's 64-bit quotients (hom_intdiv.h: divmod62, an FP64 estimate corrected in
int64) equal exact 64-bit division for dividends below 2^62 and divisors below 2^31: edge cases and
4e6 random cases, run on the host from the same __host__ __device__ source."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_divmod62_equals_exact_division(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "intdiv_host")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_2111_14317_amd", "csrc"),
                           os.path.join(HERE, "intdiv_host.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe, "2000000"], capture_output=True, text=True)
    print(out.stdout)
    last = out.stdout.strip().splitlines()[-1].split()  # "checks <count> bad <count>"
    assert out.returncode == 0 and last[0] == "checks" and last[2] == "bad"
    assert int(last[3]) == 0 and int(last[1]) > 4000000
