"""The issue probe behind the roofline model of bench.py.

On one SIMD, a wave of vector FMAs does not issue while a wave beside it
runs FP64 matrix-core instructions (its time is the sum of both), and it
mostly does while BF16 or INT8 matrix-core instructions run.  The probe is
built with the library (paper_2003_11183_amd/probe).
"""

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

PROBE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2003_11183_amd", "probe",
                     "issue_probe")


def test_fp64_matrix_instructions_hold_the_simd():
    if not os.path.exists(PROBE):
        pytest.skip("issue probe not built")
    out = subprocess.run([PROBE], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=60)
    assert out.returncode == 0, out.stdout
    rows = {}
    for line in out.stdout.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 5 and cells[1].isdigit():
            rows[(cells[0], cells[2])] = (int(cells[1]), int(cells[3]))
    for v in ("FP32", "FP64"):
        alone = rows[("nothing", v)][1]
        mfma64, beside64 = rows[("512 x 4 FP64 16x16x4 MFMA", v)]
        mfma16, beside16 = rows[("512 x 4 BF16 16x16x32 MFMA", v)]
        mfma8, beside8 = rows[("512 x 4 INT8 16x16x64 MFMA", v)]
        # FP64 MFMAs: the vector wave's time is about the sum of both
        assert beside64 > 0.85 * (alone + mfma64), (v, alone, mfma64, beside64)
        # BF16 and INT8 MFMAs: the vector wave loses well under half of their time
        assert beside16 < alone + 0.6 * mfma16, (v, alone, mfma16, beside16)
        assert beside8 < alone + 0.6 * mfma8, (v, alone, mfma8, beside8)
