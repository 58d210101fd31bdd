"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
library's host side (JSON reader, schema checks, plan build) is built without
device code and with both sanitizers on its host pass, and a host driver
calls nf_create on every model description of the synthetic workloads and on
malformed variants of them (truncations, byte edits, hand-written edge
cases). Every call must end in a defined result -- NF_EPARSE or NF_EINVAL for
bad text, NF_EDEVICE for a valid model (no GPU here: the plan is built, then
device setup fails) -- and the sanitizers must report nothing."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2502_15253_amd import build as B
from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.skipif(not (os.path.exists(B.HIPCC) and os.path.exists(CLANG)),
                                reason="hipcc / clang++ not available")


def valid_models():
    out = {"c1": synth.config1_model(), "c2": synth.config2_model(), "c3": synth.config3_model(),
           "split": synth.split_model(), "sterile": synth.sterile_model()}
    for f in ("eq1", "3nu", "4nu"):
        out[f"tiny_{f}"] = synth.tiny_model(3, formula=f)
    return {k: synth.to_json(v) for k, v in out.items()}


HAND = {
    "empty": "",
    "deep_arrays": "[" * 5000 + "]" * 5000,
    "deep_objects": '{"a":' * 3000 + "1" + "}" * 3000,
    "huge_number": '{"params": [{"name": "a", "start": 1e999}]}',
    "neg_inf": '{"params": [{"name": "a", "start": -inf}]}',
    "hex_number": '{"params": [{"name": "a", "start": 0x10}]}',
    "nan_literal": '{"params": [{"name": "a", "start": NaN}]}',
    "bad_escape": '{"params": [{"name": "a\\q", "start": 1}]}',
    "short_unicode": '{"a": "\\u12',
    "unterminated": '{"a": "abc',
    "trailing": "{} x",
    "nul_in_string": '{"a": "\\u0000"}',
    "long_string": '{"a": "' + "x" * 200000 + '"}',
    "wrong_types": '{"params": 3, "osc": [], "datasets": "x"}',
}


def mutations(text, rng, n):
    b = text.encode()
    out = []
    cuts = rng.integers(0, len(b), n)
    for c in cuts:
        out.append(b[:c])
    alphabet = b'{}[]",:-+.eE0123456789 ntfa\\'
    for _ in range(n):
        m = bytearray(b)
        for _ in range(int(rng.integers(1, 4))):
            m[int(rng.integers(0, len(m)))] = alphabet[int(rng.integers(0, len(alphabet)))]
        out.append(bytes(m))
    return out


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("hostsan"))
    lib = B.build_host_sanitized(d)
    exe = os.path.join(d, "nf_create_driver")
    cmd = [CLANG, "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           os.path.join(ROOT, "tests", "sanitize", "nf_create_driver.cpp"), lib,
           f"-Wl,-rpath,{d}", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return d, exe


def run_driver(exe, files):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""  # host code only, never a device
    r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    return r


def test_valid_and_malformed_models_under_sanitizers(driver, tmp_path):
    d, exe = driver
    rng = np.random.default_rng(12)
    files, kind = [], {}

    def add(name, data, k):
        p = os.path.join(str(tmp_path), name)
        with open(p, "wb") as f:
            f.write(data if isinstance(data, bytes) else data.encode())
        files.append(p)
        kind[p] = k

    valid = valid_models()
    for name, text in valid.items():
        add(f"valid_{name}.json", text, "valid")
        for j, m in enumerate(mutations(text, rng, 25)):
            add(f"mut_{name}_{j}.json", m, "any")
    for name, text in HAND.items():
        add(f"hand_{name}.json", text, "bad")
    r = run_driver(exe, files)
    report = (r.stderr or "")[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr, report
    assert "runtime error:" not in r.stderr, report
    assert r.returncode == 0, report
    codes = {}
    for line in r.stdout.splitlines():
        path, mode, code = line.rsplit(" ", 2)
        codes.setdefault(path, []).append(int(code))
    assert set(codes) == set(files)
    for p, cs in codes.items():
        assert len(cs) == 2
        for c in cs:
            if kind[p] == "valid":
                assert c == nf.NF_EDEVICE, (p, c)
            elif kind[p] == "bad":
                assert c in (nf.NF_EPARSE, nf.NF_EINVAL), (p, c)
            else:
                assert c in (nf.NF_EPARSE, nf.NF_EINVAL, nf.NF_EDEVICE, nf.NF_ENOMEM), (p, c)
