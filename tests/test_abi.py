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
    assert lib.smf_sample_batch(None, None, None, None) == smf.SMF_EINVAL
    assert lib.smf_sample_batch_packed(None, 1, None, None) == smf.SMF_EINVAL
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


def _signature(name):
    hdr = open(os.path.join(ROOT, "include", "smf.h")).read()
    m = re.search(r"^\s*(?:const\s+)?\w+\s*\*?\s*" + name + r"\s*\(([^;]*)\)\s*;", hdr, re.M)
    assert m, name
    return [re.sub(r"\s+", " ", a.strip()) for a in m.group(1).split(",")]


def test_boundary_signatures():
    """The calls a user of the sampler makes, with the arguments of the setup/sample
    boundary: spectrum and grid in, an opaque plan out; a seed, a field count and a
    caller-owned device buffer per call; the batched form with one seed and one device
    buffer per field; a HIP stream on every call."""
    assert _signature("smf_setup") == ["const smf_spectrum* spec", "int n_theta", "int n_phi", "int flags",
                                       "void* hip_stream", "smf_plan** out"]
    assert _signature("smf_sample") == ["const smf_plan* plan", "uint64_t seed", "int count", "void* out_dev",
                                        "void* hip_stream"]
    assert _signature("smf_sample_modes") == ["const smf_plan* plan", "uint64_t seed", "int count",
                                              "void* g_dev", "void* hip_stream"]
    assert _signature("smf_setup_batch") == ["int n", "const smf_spectrum* specs", "const int* n_theta",
                                             "const int* n_phi", "int flags", "void* hip_stream", "smf_plan** out"]
    assert _signature("smf_sample_batch") == ["const smf_plan* plan", "const uint64_t* seeds_host",
                                              "void* const* outs_dev", "void* hip_stream"]
    assert _signature("smf_get_factors") == ["const smf_plan* plan", "double* A_host", "double* B_host"]
    assert _signature("smf_destroy") == ["smf_plan* plan"]
    assert _signature("smf_error_string") == ["int code"]


def test_flag_and_error_values():
    from paper_1709_10314_amd import smf

    hdr = open(os.path.join(ROOT, "include", "smf.h")).read()
    vals = {k: int(v) for k, v in re.findall(r"(SMF_[A-Z_0-9]+)\s*=\s*(-?\d+)", hdr)}
    assert vals["SMF_FP64"] == 1 and vals["SMF_FP32"] == 2
    assert vals["SMF_NO_MIRROR"] == 4 and vals["SMF_FUSED"] == 8
    assert vals["SMF_OK"] == 0 and vals["SMF_EINVAL"] == -1 and vals["SMF_ENOMEM"] == -2
    assert vals["SMF_EHIP"] == -3 and vals["SMF_ENUMERIC"] == -4
    for k, v in vals.items():
        assert getattr(smf, k) == v, k
