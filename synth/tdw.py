"""Writer for the ``.tdw`` weight-file format.

Layout (all little-endian):

    bytes 0..3      magic b"TDW1"
    bytes 4..7      uint32 N, length of the JSON header in bytes
    bytes 8..8+N    JSON header, UTF-8
    padding         zero bytes up to the next multiple of 64 ("data start")
    tensor data     float32, each tensor at data_start + tensors[i]["offset"],
                    offsets multiples of 64, row-major in the declared shape

The header holds "denoiser" (architecture or analytic kind), "sampler",
"window", "decode" and "tensors" (name, shape, offset).  Conv weights are
[C_out, C_in, kh, kw]; linear weights are [out, in].
"""
import json
import struct

import numpy as np

MAGIC = b"TDW1"
ALIGN = 64


def _align(n):
    return (n + ALIGN - 1) // ALIGN * ALIGN


def write_tdw(path, header, tensors):
    """header: dict without "tensors"; tensors: list of (name, float32 ndarray)."""
    entries = []
    off = 0
    for name, arr in tensors:
        arr = np.ascontiguousarray(arr, dtype="<f4")
        entries.append({"name": name, "shape": list(arr.shape), "offset": off})
        off = _align(off + arr.nbytes)
    hdr = dict(header)
    hdr["tensors"] = entries
    blob = json.dumps(hdr, sort_keys=True).encode("utf-8")
    data_start = _align(8 + len(blob))
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<I", len(blob)))
        f.write(blob)
        f.write(b"\0" * (data_start - 8 - len(blob)))
        pos = 0
        for (name, arr), e in zip(tensors, entries):
            arr = np.ascontiguousarray(arr, dtype="<f4")
            if e["offset"] > pos:
                f.write(b"\0" * (e["offset"] - pos))
                pos = e["offset"]
            f.write(arr.tobytes())
            pos += arr.nbytes
        if off > pos:
            f.write(b"\0" * (off - pos))
