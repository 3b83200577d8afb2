"""Host-side checks of the C ABI: the library loads and exports every declared symbol,
and the binding's argument checks run without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "smf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(smf_\w+)\s*\(", hdr, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("smf_setup", "smf_sample", "smf_sample_modes", "smf_get_factors", "smf_destroy",
              "smf_error_string", "smf_plan_dims"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1709_10314_amd import smf

    lib = smf.load()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(smf.EXPORTS)


def test_error_strings_and_null_handling_without_gpu():
    from paper_1709_10314_amd import smf

    lib = smf.load()
    assert smf.smf_error_string(0) == "success"
    assert "invalid" in smf.smf_error_string(-1)
    assert "unknown" in smf.smf_error_string(7)
    # NULL plan / NULL outputs are rejected before any HIP call
    assert lib.smf_sample(None, 1, 1, None, None) == smf.SMF_EINVAL
    assert lib.smf_sample_modes(None, 1, 1, None, None) == smf.SMF_EINVAL
    assert lib.smf_plan_dims(None, None) == smf.SMF_EINVAL
    assert lib.smf_get_factors(None, None, None) == smf.SMF_EINVAL
    assert lib.smf_destroy(None) == smf.SMF_OK
    assert lib.smf_setup(None, 8, 16, smf.SMF_FP64, None, None) == smf.SMF_EINVAL
    assert lib.smf_sample_batch(None, 1, None, None) == smf.SMF_EINVAL
    assert lib.smf_batch_layout(None, None) == smf.SMF_EINVAL
    assert lib.smf_autotune_batch(None, 1, None, None, None) == smf.SMF_EINVAL
    assert lib.smf_setup_batch(0, None, None, None, smf.SMF_FP32, None, None) == smf.SMF_EINVAL
    assert lib.smf_setup_grid(None, 8, None, 16, smf.SMF_FP64, None, None) == smf.SMF_EINVAL
    assert lib.smf_sample_lognormal(None, 1, 1, 0.0, 1.0, None, None) == smf.SMF_EINVAL
    assert lib.smf_transform(None, 1, None, None) == smf.SMF_EINVAL
    assert lib.smf_set_factors(None, None, None, None) == smf.SMF_EINVAL
    assert lib.smf_plan_grid(None, None, None) == smf.SMF_EINVAL
    assert lib.smf_set_ring_blocks(None, 0) == smf.SMF_EINVAL
    assert lib.smf_get_ring_blocks(None, 1, None) == smf.SMF_EINVAL
    assert lib.smf_setup_rings(None, 8, None, None, None, smf.SMF_FP32, None, None) == smf.SMF_EINVAL
    assert lib.smf_ring_layout(None, None) == smf.SMF_EINVAL
    assert lib.smf_synthesize_rings(None, 1, None, None, None) == smf.SMF_EINVAL
    assert lib.smf_sample_rings(None, 1, 1, None, None, None) == smf.SMF_EINVAL
    assert lib.smf_sample_rings_lognormal(None, 1, 1, 0.0, 1.0, None, None, None) == smf.SMF_EINVAL


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1709_10314_amd import smf

    monkeypatch.setattr(smf, "_lib", None)
    monkeypatch.setattr(smf, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        smf.load()
