"""Host-side checks of the library's compile flags (no GPU work).

The kernels are compiled with the packed-FP32 target feature switched off, so that the
compiler never pairs two FP32 multiply-adds into one packed instruction.  The device pass of
hipcc honours the flag (its host pass prints that it does not know the feature and ignores
it, which is harmless).  These tests compile device code to gfx950 assembly: a probe whose
float2 arithmetic the compiler packs without the flag, and every kernel source of the
library with the flags the build uses."""
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1505_02976_amd import build

PACKED = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")
NOFEATURE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2 *a, const float2 *b, float s)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    float2 x = a[i], y = b[i];
    x.x = x.x * s + y.x; x.y = x.y * s + y.y;
    x.x = x.x * y.x + s; x.y = x.y * y.y + s;
    a[i] = x;
}
"""


def _device_asm(src_path, flags, out_path):
    cmd = [build.HIPCC] + flags + ["--cuda-device-only", "-S", "-x", "hip", src_path, "-o", out_path]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out_path) as fh:
        return fh.read()


def _flags_without_feature():
    f = list(build.FLAGS)
    i = f.index("-packed-fp32-ops")
    del f[i - 3:i + 1]
    return [x for x in f if x not in ("-fPIC",)]


def test_build_flags_switch_packed_fp32_off(tmp_path):
    assert all(x in build.FLAGS for x in NOFEATURE)
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    without = _device_asm(str(src), _flags_without_feature(), str(tmp_path / "without.s"))
    with_flags = _device_asm(str(src), list(build.FLAGS), str(tmp_path / "with.s"))
    # the probe is packed when the feature is on, so the check below means something
    assert PACKED.search(without), "probe no longer packs without the flag"
    assert not PACKED.search(with_flags)


def test_no_packed_fp32_in_library_kernels(tmp_path):
    sources = [s for s in build.SOURCES if s.endswith(".hip")]
    assert sources

    def one(s):
        return s, _device_asm(os.path.join(build.CSRC, s), list(build.FLAGS), str(tmp_path / (s + ".s")))

    with ThreadPoolExecutor(max_workers=min(4, len(sources))) as ex:
        results = list(ex.map(one, sources))
    bad = {s: sorted(set(m.group(0) for m in PACKED.finditer(asm))) for s, asm in results if PACKED.search(asm)}
    assert not bad, bad
