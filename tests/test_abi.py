"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/nufold.h, and rejects bad model descriptions before any
device work."""
import ctypes as C
import json
import os
import re

import pytest

from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nufold.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    lib = C.CDLL(nf.LIB_PATH)
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # the binding covers the same set with the same names
    assert set(names) == set(nf.SIGNATURES)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define (NF_[A-Z0-9]+) (-?\d+)", text))
    for k, v in consts.items():
        assert getattr(nf, k) == int(v), k


def _create(text, mode=nf.NF_M64):
    h = C.c_void_p()
    code = nf.load().nf_create(C.byref(h), text.encode(), mode, None)
    msg = nf.load().nf_last_error(None).decode()
    if code == 0:
        nf.load().nf_destroy(h)
    return code, msg


@pytest.mark.parametrize("text,frag", [
    ("{", "JSON"),
    ("[]", "object"),
    ('{"params": []}', "params"),
    ('{"params": [{"name": "a", "start": 1}], "osc": {"formula": "x"}}', "formula"),
])
def test_bad_json_is_a_parse_error(text, frag):
    code, msg = _create(text)
    assert code == nf.NF_EPARSE
    assert frag.lower() in msg.lower()


def test_schema_errors_are_reported_before_device_setup():
    m = synth.config1_model()
    bad = json.loads(json.dumps(m))
    bad["datasets"][0]["norm"] = ["no_such_parameter"]
    code, msg = _create(json.dumps(bad))
    assert code == nf.NF_EPARSE and "no_such_parameter" in msg
    bad = json.loads(json.dumps(m))
    bad["datasets"][0]["edges"] = [1.0, 0.5, 2.0]
    code, msg = _create(json.dumps(bad))
    assert code == nf.NF_EPARSE and "increase" in msg
    bad = json.loads(json.dumps(m))
    bad["cov_priors"] = [dict(params=["norm", "escale.c0"], mean=[1, 0], cov=[[1, 2], [2, 1]])]
    code, msg = _create(json.dumps(bad))
    assert code == nf.NF_EPARSE and "positive definite" in msg


def test_invalid_mode_and_nulls():
    h = C.c_void_p()
    assert nf.load().nf_create(C.byref(h), b"{}", 7, None) == nf.NF_EINVAL
    assert nf.load().nf_create(None, b"{}", 0, None) == nf.NF_EINVAL
    assert nf.load().nf_num_params(None) == nf.NF_EINVAL
    nf.load().nf_destroy(None)


def test_valid_model_without_device_reports_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    code, msg = _create(json.dumps(synth.config2_model()))
    assert code == nf.NF_EDEVICE, msg
