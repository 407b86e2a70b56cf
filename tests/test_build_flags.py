"""The build keeps packed FP32 instructions (v_pk_fma_f32 and kin) out of the
gfx950 code: the feature flag in the library's hipcc command takes effect in
the device pass (hipcc's host pass prints that it does not know the feature,
which is harmless).  Checked on a small kernel whose float2 arithmetic hipcc
-O3 turns into a packed FMA without the flag (CPU only: hipcc cross-compiles)."""
import os
import shutil
import subprocess

import pytest

from paper_2211_13295_amd import build as hipbuild

SRC = r"""
#include <hip/hip_runtime.h>
__global__ void k(float2* a, const float2* b, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { float2 x = a[i], y = b[i]; a[i] = make_float2(x.x * y.x + x.y, x.y * y.y + x.x); }
}
"""


def _device_asm(tmp_path, flags):
    src = tmp_path / "pk.hip"
    src.write_text(SRC)
    out = tmp_path / "pk.s"
    subprocess.run([hipbuild.HIPCC, "-O3", "--offload-arch=gfx950", "--cuda-device-only", "-S", *flags,
                    str(src), "-o", str(out)], check=True, capture_output=True)
    return out.read_text()


@pytest.mark.skipif(not os.path.exists(hipbuild.HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_packed_fp32_is_kept_out_of_the_device_code(tmp_path):
    i = hipbuild.FLAGS.index("-packed-fp32-ops")
    feature = hipbuild.FLAGS[i - 3:i + 1]
    assert feature == ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    plain = _device_asm(tmp_path, [])
    guarded = _device_asm(tmp_path, feature)
    assert "v_pk_fma_f32" in plain
    assert "v_pk_" not in guarded
