"""The C-ABI library loads and exports every symbol include/he_mi355x.h declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "he_mi355x.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:he_status|const char\*)\s+(he_\w+)\s*\(", text, re.M)))


def test_header_declares_calls():
    names = declared()
    for n in ("he_ctx_create", "he_keygen", "he_encrypt_matrix", "he_matmul", "he_covariance", "he_decrypt"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2305_17341_amd import he
    if not os.path.exists(he.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(he.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(he.EXPORTS) == declared()


def test_binding_has_no_cpu_fallback(tmp_path, monkeypatch):
    from paper_2305_17341_amd import he
    monkeypatch.setattr(he, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(he, "_lib", None)
    with pytest.raises(RuntimeError):
        he.load()


def test_context_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2305_17341_amd import he
    if not os.path.exists(he.LIB_PATH):
        pytest.skip("library not built")
    from paper_2305_17341_amd import inputs as I
    with pytest.raises(he.HeError) as e:
        he.chain_context(I.SMALL)
    assert e.value.status == -6


def test_knobs_host_side():
    """Launch-shape knobs are host state: names and ranges are checked, and
    every knob the autotuner sweeps exists with its candidate values."""
    from paper_2305_17341_amd import autotune, he
    if not os.path.exists(he.LIB_PATH):
        pytest.skip("library not built")
    for name, values in autotune.CANDIDATES.items():
        old = he.knob_get(name)
        try:
            for v in values:
                he.knob_set(name, v)
                assert he.knob_get(name) == v
        finally:
            he.knob_set(name, old)
    for name, bad in [("ms_members", 0), ("ms_members", 9), ("mr_rotations", 65), ("ntt_interleave", 2), ("mr_group", 3),
                      ("ew_interleave", -1), ("mr_int_split", 2), ("mr_int_pass", 5), ("mr_int_chunk", 0),
                      ("mr_int_chunk", 65), ("mr_int_concurrent", 2), ("fbc_mfma", 2),
                      ("xcd_map", 2), ("sum_streams", 3), ("mr_pair", 2),
                      ("no_such_knob", 1)]:
        with pytest.raises(he.HeError) as e:
            he.knob_set(name, bad)
        assert e.value.status == -1
