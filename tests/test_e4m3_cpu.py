"""FP32 -> fp8 E4M3 conversion (low plane of the BF16-refined form), built for the host and
checked against the format's definition: every finite E4M3 value enumerated from its
fields (OCP layout: bias 7, subnormals below 2^-6, 0x7F NaN, largest finite 448), the
nearest one chosen with ties to the even code, saturation above 448."""
import os
import struct
import subprocess

import numpy as np
import pytest

from tests.conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2406_06488_amd", "csrc")


def e4m3_values():
    vals = []
    for code in range(0x7F):  # 0x7F is NaN
        e, m = code >> 3, code & 7
        v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
        vals.append(v)
    return np.array(vals)


def reference(x, vals):
    a = abs(float(x))
    if a >= 448.0:
        code = 0x7E
    else:
        d = np.abs(vals - a)
        best = np.flatnonzero(d == d.min())
        code = int(best[0]) if len(best) == 1 else int([c for c in best if c % 2 == 0][0])
    if code == 0:
        return 0
    return code | (0x80 if x < 0 else 0)


def test_e4m3_against_definition(tmp_path):
    exe = str(tmp_path / "e4m3_check")
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "cpp", "e4m3_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("build failed:\n" + r.stderr[-4000:])
    vals = e4m3_values()
    rng = np.random.default_rng(7)
    xs = [0.0, -0.0, 448.0, 449.0, 464.0, 500.0, 1e6, 2.0 ** -6, 2.0 ** -9, 2.0 ** -10,
          3 * 2.0 ** -10, 2.0 ** -11]
    xs += list(vals) + list(-vals)
    mids = (vals[1:] + vals[:-1]) / 2.0  # exact ties between neighbouring codes
    xs += list(mids) + list(-mids)
    xs += list(np.nextafter(mids, 0)) + list(np.nextafter(mids, 1e9))
    xs += list(rng.uniform(-460, 460, 4000)) + list(rng.uniform(-0.05, 0.05, 4000))
    xs += list(np.exp(rng.uniform(np.log(1e-4), np.log(450), 4000)))
    xs = np.array(xs, dtype=np.float32)
    inp = "\n".join("%08x" % struct.unpack("<I", struct.pack("<f", float(x)))[0] for x in xs)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=60)
    assert out.returncode == 0
    got = [int(line.split()[1], 16) for line in out.stdout.split("\n") if line.strip()]
    assert len(got) == len(xs)
    bad = [(float(x), g, reference(x, vals)) for x, g in zip(xs, got) if g != reference(x, vals)]
    assert not bad, bad[:10]
