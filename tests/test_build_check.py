"""The build's scratch-memory check: kernels whose registers spill (or whose arrays are left in private
memory) are reported from the compiler's resource-usage remarks, clean kernels are not. Compiles two
tiny kernels for gfx950 on the host (no GPU)."""
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_2109_11920_amd import build as B

SRC = r'''
#include <hip/hip_runtime.h>
__global__ void k_clean(const float *x, float *y) { y[threadIdx.x] = 2.f * x[threadIdx.x]; }
__global__ void k_private(const float *x, float *y) {
    float a[64];
    for (int i = 0; i < 64; ++i) a[i] = x[i * 64 + threadIdx.x];
    y[threadIdx.x] = a[(threadIdx.x * 7) & 63];   // dynamic index: the array lives in scratch memory
}
'''


def test_scratch_check_reports_private_arrays_only():
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "k.hip")
        open(src, "w").write(SRC)
        r = subprocess.run([hipcc] + B.common_flags() + ["-x", "hip", "-c", src, "-o", os.path.join(d, "k.o"),
                            "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        bad = B.scratch_kernels(r.stderr)
        names = [n for n, _ in bad]
        assert any("k_private" in n for n in names), bad
        assert not any("k_clean" in n for n in names), bad
    finally:
        shutil.rmtree(d)


def test_scratch_parser_on_remark_text():
    text = ("x.hip:1:1: remark: Function Name: _Z1av [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:9:1: remark: Function Name: _Z1bv [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:9:1: remark:     ScratchSize [bytes/lane]: 48 [-Rpass-analysis=kernel-resource-usage]\n")
    assert B.scratch_kernels(text) == [("_Z1bv", 48)]
