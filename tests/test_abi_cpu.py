"""Host-side checks of libsmcrt that need no GPU: the library loads, exports
every entry point its header declares, validates scenes on the host, and
computes the simulation volume by the same rule as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    from paper_2112_08035_amd import build_lib, smcrt
    if build_lib.is_stale():
        build_lib.build()
    smcrt.lib()
    return smcrt


def header_functions():
    txt = open(os.path.join(ROOT, "include", "smcrt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(smcrt_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_entry_point(S):
    names = header_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(S._SIGS), "binding and header disagree"
    assert S.smcrt_abi_version() == 1


def test_scene_validation_rejects_bad_input(S):
    with pytest.raises(S.SmcrtError):
        S.smcrt_scene_create(0.0, 1e-5, 1e-4)
    with pytest.raises(S.SmcrtError):
        S.smcrt_scene_create(1.0, -1.0, 1e-4)
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        with pytest.raises(S.SmcrtError, match="radius"):
            S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, -1])
        with pytest.raises(S.SmcrtError, match="takes"):
            S.smcrt_scene_add_primitive(h, 1, [0, 0, 0, 1])
        with pytest.raises(S.SmcrtError, match="finite"):
            S.smcrt_scene_add_primitive(h, 0, [0, float("nan"), 0, 1])
        with pytest.raises(S.SmcrtError, match="differ"):
            S.smcrt_scene_add_primitive(h, 2, [1, 1, 1, 1, 1, 1, 0.1])
        p = S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, 1])
        with pytest.raises(S.SmcrtError, match="out of range"):
            S.smcrt_scene_add_region(h, [p + 1], 0, 0.0, 0.1, 10, 0.9, 1.4)
        with pytest.raises(S.SmcrtError, match="g < 1"):
            S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.1, 10, 1.0, 1.4)
        with pytest.raises(S.SmcrtError, match="mu_a"):
            S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.0, 0.0, 0.5, 1.4)
        with pytest.raises(S.SmcrtError, match="k > 0"):
            S.smcrt_scene_add_region(h, [p], 1, 0.0, 0.1, 10, 0.5, 1.4)
        with pytest.raises(S.SmcrtError, match="lo < hi"):
            S.smcrt_scene_set_grid(h, [0, 0, 0], [1, 0, 1], [4, 4, 4])
        with pytest.raises(S.SmcrtError, match="direction"):
            S.smcrt_scene_set_source(h, 1, [0, 0, 0, 0, 0, 0])
        with pytest.raises(S.SmcrtError, match="m_survive"):
            S.smcrt_scene_set_roulette(h, 1e-4, 0)
        with pytest.raises(S.SmcrtError, match="source"):
            S.smcrt_scene_info(h)
        S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.1, 10, 0.9, 1.4)
        S.smcrt_scene_set_source(h, 0, [5.0, 0, 0])  # outside everything but inside the padded volume? no:
        nr, npr, lo, hi = S.smcrt_scene_info(h)       # the volume grows to hold the source
        assert nr == 1 and npr == 1 and hi[0] >= 5.0
    finally:
        S.smcrt_scene_destroy(h)


def test_regions_limit(S):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        p = S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, 1])
        for _ in range(16):
            S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.1, 1.0, 0.0, 1.0)
        with pytest.raises(S.SmcrtError, match="at most"):
            S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.1, 1.0, 0.0, 1.0)
    finally:
        S.smcrt_scene_destroy(h)


@pytest.mark.parametrize("name", ["sphere", "slab", "cylinder", "vessels"])
def test_volume_rule_agrees_with_oracle(S, orc, W, name):
    desc = W.vessel_scene(3, 1.0, n_caps=50, n_grid=8) if name == "vessels" else W.WORKLOADS[name](n_grid=8)
    sc = S.Scene(desc)
    _, npr, lo, hi = S.smcrt_scene_info(sc.h)
    olo, ohi = orc.bounding_box(desc)
    np.testing.assert_allclose(lo, olo, rtol=0, atol=1e-15)
    np.testing.assert_allclose(hi, ohi, rtol=0, atol=1e-15)
    assert npr == len(desc["prims"])


def test_engine_without_device_fails_cleanly_or_works(S):
    try:
        e = S.smcrt_engine_create(0)
    except S.SmcrtError as err:
        assert err.status in (S.E_HIP, S.E_INVALID)
        assert S.smcrt_last_error()
        return
    S.smcrt_engine_destroy(e)


def test_binding_fails_loudly_without_library(S, monkeypatch, tmp_path):
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        S.lib()
