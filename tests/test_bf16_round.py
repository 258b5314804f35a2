"""The bfloat16 rounding of the FP32 multigrid levels' operator records
(faces and shift, csrc/rh_internal.h) against torch's own float32 ->
bfloat16 conversion (round to nearest, ties to even), on the host: random
values over the whole exponent range, exact ties, neighbours of ties,
zeros and subnormals."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("bf16") / "probe")
    subprocess.run([HIPCC, "-std=c++17", "-O2", "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_0908_2654_amd", "csrc"),
                    os.path.join(ROOT, "tests", "bf16_probe.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=300)
    return exe


def _run(exe, bits):
    inp = "\n".join(f"{int(b):08x}" for b in bits) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True,
                         timeout=120).stdout.split()
    h = np.array([int(x, 16) for x in out[0::2]], dtype=np.uint32)
    back = np.array([int(x, 16) for x in out[1::2]], dtype=np.uint32)
    return h, back


def test_bf16_round_matches_round_to_nearest_even(probe):
    import torch
    rng = np.random.default_rng(7)
    # positive finite values (faces and shifts are >= 0), every exponent
    exps = rng.integers(1, 254, 20000).astype(np.uint32)
    mant = rng.integers(0, 1 << 23, 20000).astype(np.uint32)
    rand = (exps << 23) | mant
    # exact ties (low 16 bits 0x8000) with even and odd kept parts, and
    # their neighbours one ulp either side
    base = (rng.integers(1, 254, 2000).astype(np.uint32) << 23) | \
           (rng.integers(0, 1 << 7, 2000).astype(np.uint32) << 16)
    ties = np.concatenate([base | 0x8000, base | 0x7FFF, base | 0x8001, base | 0x18000,
                           base | 0x17FFF, base | 0x18001])
    special = np.array([0x0, 0x1, 0x7FFF, 0x8000, 0x807FFF, 0x800000, 0x3F800000, 0x7F7F0000,
                        0x7F7F7FFF], dtype=np.uint32)
    bits = np.concatenate([rand, ties, special]).astype(np.uint32)
    h, back = _run(probe, bits)
    ref = torch.from_numpy(bits.view(np.float32).copy()).to(torch.bfloat16)
    ref_h = ref.view(torch.int16).numpy().astype(np.uint16).astype(np.uint32)
    assert np.array_equal(h, ref_h)
    # the value a stored half stands for is its upper half of an FP32 pattern
    assert np.array_equal(back, h << 16)
    # relative rounding error <= 2^-8 (8 significant bits) for normal values
    x = bits[(bits >> 23) > 0].view(np.float32).astype(np.float64)
    hb = h[(bits >> 23) > 0]
    y = (hb << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * x)
