"""Oracle-side reader of ``.tdw`` weight files (written independently of the
library's C++ parser).

TEST INFRASTRUCTURE (oracle).  Format: b"TDW1", uint32 header length, JSON
header, zero padding to a 64-byte boundary, then float32 tensors at the
header's offsets.  Tensors are promoted to float64.
"""
import json
import struct

import numpy as np


def read_tdw(path):
    with open(path, "rb") as f:
        raw = f.read()
    if raw[:4] != b"TDW1":
        raise ValueError("not a tdw file: %r" % path)
    (n,) = struct.unpack("<I", raw[4:8])
    header = json.loads(raw[8:8 + n].decode("utf-8"))
    data_start = (8 + n + 63) // 64 * 64
    tensors = {}
    for e in header.get("tensors", []):
        count = int(np.prod(e["shape"])) if e["shape"] else 1
        off = data_start + e["offset"]
        arr = np.frombuffer(raw, dtype="<f4", count=count, offset=off)
        tensors[e["name"]] = arr.reshape(e["shape"]).astype(np.float64)
    return header, tensors
