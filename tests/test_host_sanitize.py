"""The weight-file parser and the window planner built host-only under
AddressSanitizer + UndefinedBehaviorSanitizer (g++), run on the CPU: the
planner's kappa against its definition on random regions up to +-2^31, the
parser on valid files, on the malformed files the GPU edge test refuses (and
more), and on byte-level mutations of a valid header.  A sanitizer report
aborts the harness, failing the test.
"""
import json
import os
import shutil
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_08309_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("san") / "host_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(ROOT, "tests", "host_sanitize.cpp"),
           os.path.join(CSRC, "header.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def run(harness, *args):
    r = subprocess.run([harness] + [str(a) for a in args], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_planner_kappa_sanitized(harness):
    assert "kappa ok 300000" in run(harness, "kappa", 300000, 11)


def _tdw_bytes(blob, data):
    start = (8 + len(blob) + 63) // 64 * 64
    return b"TDW1" + struct.pack("<I", len(blob)) + blob + b"\0" * (start - 8 - len(blob)) + data


def test_parser_sanitized_on_valid_and_malformed_files(harness, weights, tmp_path):
    good = {c: weights(c) for c in ("c1", "lg", "lgs", "c1t2", "c1h", "cc")}
    raw = open(good["c1"], "rb").read()
    n = struct.unpack("<I", raw[4:8])[0]
    hdr = json.loads(raw[8:8 + n])
    data = raw[(8 + n + 63) // 64 * 64:]

    def edited(f):
        h = json.loads(json.dumps(hdr))
        f(h)
        return _tdw_bytes(json.dumps(h).encode(), data)

    bad = {
        "empty": b"",
        "short": b"TDW1\x05",
        "magic": b"TDW2" + raw[4:],
        "header_length": raw[:4] + struct.pack("<I", len(raw)) + raw[8:],
        "header_length_max": raw[:4] + struct.pack("<I", 0xFFFFFFFF) + raw[8:],
        "json_syntax": _tdw_bytes(b'{"denoiser": {"kind": ', data),
        "json_depth": _tdw_bytes(b"[" * 100 + b"]" * 100, data),
        "json_deeper": _tdw_bytes(b"[" * 100000, data),
        "json_root": _tdw_bytes(b"42", data),
        "json_string": _tdw_bytes(b'{"a": "\\u00', data),
        "json_number": _tdw_bytes(b'{"a": 1e99999}', data),
        "data_truncated": raw[:len(raw) - 1000],
        "integer_range": edited(lambda h: h["denoiser"].__setitem__("in_channels", 1e30)),
        "integer_fraction": edited(lambda h: h["sampler"].__setitem__("steps", 2.5)),
        "negative_steps": edited(lambda h: h["sampler"].__setitem__("steps", -3)),
        "huge_steps": edited(lambda h: h["sampler"].__setitem__("steps", 1 << 40)),
        "window_zero": edited(lambda h: h["window"].__setitem__("stride", 0)),
        "many_levels": edited(lambda h: h["denoiser"].__setitem__("channels", [16] * 40)),
        "blend_order": edited(lambda h: h["sampler"].__setitem__("blend", [0, 5, 3, 8])),
        "tensor_missing_key": edited(lambda h: h["tensors"][0].pop("offset")),
        "tensor_shape_negative": edited(lambda h: h["tensors"][0].__setitem__("shape", [-1, 3])),
        "tensor_size": edited(lambda h: h["tensors"][0].__setitem__("shape", [1 << 30, 1 << 30, 4])),
        "tensor_offset": edited(lambda h: h["tensors"][0].__setitem__("offset", -64)),
        "tensor_offset_huge": edited(lambda h: h["tensors"][0].__setitem__("offset", 1 << 62)),
        "denoiser_kind": edited(lambda h: h["denoiser"].__setitem__("kind", "transformer")),
        "eps_nan": edited(lambda h: h["window"].__setitem__("eps", float("nan"))),
        "decode_inf": edited(lambda h: h["decode"].__setitem__("sigma_low", float("inf"))),
    }
    paths = list(good.values())
    for name, content in bad.items():
        p = tmp_path / (name + ".tdw")
        p.write_bytes(content)
        paths.append(str(p))
    status = [int(v) for v in run(harness, "parse", *paths).split()]
    assert status[:len(good)] == [0] * len(good)
    refused = dict(zip(bad, status[len(good):]))
    assert all(v == -5 for v in refused.values()), refused


@pytest.mark.parametrize("config,seed", [("c1", 3), ("lgs", 5)])
def test_parser_fuzz_sanitized(harness, weights, config, seed):
    out = run(harness, "fuzz", weights(config), 20000, seed)
    assert "fuzz ok 20000" in out
