"""The training checkpoint file on the CPU: cv_mlp_checkpoint_info (no device
needed) accepts a well-formed file and returns its fields, and refuses with
CV_EINVAL a file with a flipped byte anywhere, a truncated or extended one,
another magic, an inconsistent parameter count or a negative step.  The file
is built here from its published layout (header, three parameter arrays,
64-bit FNV-1a of everything before the hash)."""
from __future__ import annotations

import struct

import numpy as np
import pytest

DIMS = (3, 8, 5)


def fnv1a64(b: bytes) -> int:
    h = 0xCBF29CE484222325
    for c in b:
        h ^= c
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def make(dims=DIMS, step=123, key=0xDEADBEEF12345678, omega0=30.0, count=None, magic=b"CVCKP01\0"):
    n = sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(len(dims) - 1))
    rng = np.random.default_rng(3)
    body = magic + struct.pack("<i", len(dims) - 1) + struct.pack(f"<{len(dims)}i", *dims)
    body += struct.pack("<q", n if count is None else count) + struct.pack("<f", omega0)
    body += struct.pack("<qQ", step, key)
    body += rng.normal(size=3 * n).astype("<f4").tobytes()
    return body + struct.pack("<Q", fnv1a64(body))


@pytest.fixture(scope="module")
def cv():
    import paper_2507_22901_amd as cv
    cv.lib()
    return cv


def test_well_formed_file(cv, tmp_path):
    p = tmp_path / "ok.ckpt"
    p.write_bytes(make())
    dims, step, key = cv.checkpoint_info(str(p))
    assert dims == DIMS and step == 123 and key == 0xDEADBEEF12345678


def test_corrupt_files_are_refused(cv, tmp_path):
    good = make()
    bad = {}
    for pos in (0, 9, 20, 40, len(good) // 2, len(good) - 9, len(good) - 1):
        b = bytearray(good)
        b[pos] ^= 0x10
        bad[f"flip@{pos}"] = bytes(b)
    bad["truncated"] = good[:-1]
    bad["extended"] = good + b"\0"
    bad["no hash"] = good[:-8]
    bad["other magic"] = make(magic=b"CVMLP02\0")
    bad["wrong count"] = make(count=7)
    bad["negative step"] = make(step=-1)
    bad["bad omega0"] = make(omega0=float("nan"))
    bad["empty"] = b""
    for name, data in bad.items():
        p = tmp_path / "bad.ckpt"
        p.write_bytes(data)
        with pytest.raises(cv.CvError) as e:
            cv.checkpoint_info(str(p))
        assert e.value.code == cv.CV_EINVAL, name
    with pytest.raises(cv.CvError):
        cv.checkpoint_info(str(tmp_path / "missing.ckpt"))
