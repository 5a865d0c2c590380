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
        with pytest.raises(S.SmcrtError, match="axis"):
            S.smcrt_scene_add_primitive(h, 4, [0, 0, 0, 0, 0, 0, 1.0, 0.2])
        with pytest.raises(S.SmcrtError, match="tube radius"):
            S.smcrt_scene_add_primitive(h, 4, [0, 0, 0, 0, 0, 1, 1.0, 0.0])
        with pytest.raises(S.SmcrtError, match="unknown kind"):
            S.smcrt_scene_add_primitive(h, 9, [0, 0, 0, 1])
        with pytest.raises(S.SmcrtError, match="cone ends"):
            S.smcrt_scene_add_primitive(h, 5, [0, 0, 0, 0, 0, 0, 1.0, 0.5])
        with pytest.raises(S.SmcrtError, match="cone radii"):
            S.smcrt_scene_add_primitive(h, 5, [0, 0, 0, 0, 0, 1, 0.0, 0.0])
        with pytest.raises(S.SmcrtError, match="octahedron"):
            S.smcrt_scene_add_primitive(h, 6, [0, 0, 0, 0.0])
        with pytest.raises(S.SmcrtError, match="hexagonal prism"):
            S.smcrt_scene_add_primitive(h, 7, [0, 0, 0, 0.3, -1.0])
        with pytest.raises(S.SmcrtError, match="ellipsoid"):
            S.smcrt_scene_add_primitive(h, 8, [0, 0, 0, 1.0, 0.0, 1.0])
        with pytest.raises(S.SmcrtError, match="takes 8"):
            S.smcrt_scene_add_primitive(h, 5, [0, 0, 0, 1])
        p = S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, 1])
        with pytest.raises(S.SmcrtError, match="out of range"):
            S.smcrt_scene_add_region(h, [p + 1], 0, 0.0, 0.1, 10, 0.9, 1.4)
        with pytest.raises(S.SmcrtError, match="g < 1"):
            S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.1, 10, 1.0, 1.4)
        with pytest.raises(S.SmcrtError, match="mu_a"):
            S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.0, 0.0, 0.5, 1.4)
        with pytest.raises(S.SmcrtError, match="k > 0"):
            S.smcrt_scene_add_region(h, [p], 1, 0.0, 0.1, 10, 0.5, 1.4)
        with pytest.raises(S.SmcrtError, match="unknown op"):
            S.smcrt_scene_add_region(h, [p], 4, 0.0, 0.1, 10, 0.5, 1.4)
        with pytest.raises(S.SmcrtError, match="lo < hi"):
            S.smcrt_scene_set_grid(h, [0, 0, 0], [1, 0, 1], [4, 4, 4])
        with pytest.raises(S.SmcrtError, match="direction"):
            S.smcrt_scene_set_source(h, 1, [0, 0, 0, 0, 0, 0])
        with pytest.raises(S.SmcrtError, match="m_survive"):
            S.smcrt_scene_set_roulette(h, 1e-4, 0)
        with pytest.raises(S.SmcrtError, match="source"):
            S.smcrt_scene_info(h)
        S.smcrt_scene_add_region(h, [p], 0, 0.0, 0.1, 10, 0.9, 1.4)
        S.smcrt_scene_set_source(h, 0, [5.0, 0, 0])  # a source outside every region:
        nr, npr, lo, hi = S.smcrt_scene_info(h)       # the volume grows to hold it
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


@pytest.mark.parametrize("name", ["sphere", "slab", "cylinder", "vessels", "glass_sphere", "bottle", "torus", "gallery",
                                  "shapes"])
def test_volume_rule_agrees_with_oracle(S, orc, W, name):
    if name == "vessels":
        desc = W.vessel_scene(3, 1.0, n_caps=50, n_grid=8)
    elif name == "torus":
        desc = W.torus_beam()
        desc["prims"][0]["axis"] = [0.3, -0.4, 0.9]   # a tilted ring: every axis of the box differs
    else:
        desc = W.WORKLOADS[name](n_grid=8)
    sc = S.Scene(desc)
    _, npr, lo, hi = S.smcrt_scene_info(sc.h)
    olo, ohi = orc.bounding_box(desc)
    # placed primitives' boxes come from 8 turned corners, summed in another
    # order on each side
    atol = 1e-12 if name in ("gallery", "shapes") else 1e-15
    np.testing.assert_allclose(lo, olo, rtol=0, atol=atol)
    np.testing.assert_allclose(hi, ohi, rtol=0, atol=atol)
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


# ---------------------------------------------------------------- serving
# device = -1: the request scheduler without a device (epochs complete at
# once), so admission order, the memory budget and cancellation run here.

def _small_scene(S, W, n_grid):
    return S.Scene(W.sphere_scene(n_grid=n_grid))


def test_server_dry_run_completes_in_arrival_order(S, W):
    sv = S.Server(device=-1, hbm_budget_bytes=1 << 30, epoch_packets=1000)
    try:
        sc = _small_scene(S, W, 8)
        ids = [sv.submit(sc, i, 500 + 1000 * i)[0] for i in range(6)]
        for rid in ids:
            sv.wait(rid, 10.0)
        states = [sv.poll(r) for r in ids]
        assert all(s[0] == "DONE" for s in states)
        admits = [s[2] for s in states]
        assert admits == sorted(admits)
        assert all(s[3] >= s[2] >= s[1] >= 0 for s in states)
        st = sv.stats()
        assert st["packets_done"] == sum(500 + 1000 * i for i in range(6))
        assert st["bytes_in_use"] == 0 and st["queued"] == 0 and st["active"] == 0
    finally:
        sv.close()


def test_server_budget_admits_one_at_a_time_and_rejects_oversize(S, W):
    big = _small_scene(S, W, 64)      # 64^3 doubles = 2 MiB grid
    sv = S.Server(device=-1, hbm_budget_bytes=3 << 20, epoch_packets=100)
    try:
        with pytest.raises(S.SmcrtError, match="budget"):
            sv.submit(_small_scene(S, W, 128), 1, 10)  # 16 MiB grid never fits
        ids = [sv.submit(big, i, 1000)[0] for i in range(3)]
        for rid in ids:
            sv.wait(rid, 10.0)
        t = [sv.poll(r) for r in ids]
        # only one request fits at a time: each is admitted after the previous finished
        assert t[1][2] >= t[0][3] and t[2][2] >= t[1][3]
    finally:
        sv.close()


def test_server_cancel_queued_request(S, W):
    big = _small_scene(S, W, 64)
    sv = S.Server(device=-1, hbm_budget_bytes=3 << 20, epoch_packets=10)
    try:
        a = sv.submit(big, 1, 200000)[0]   # many epochs
        b = sv.submit(big, 2, 1000)[0]     # waits for the budget
        sv.cancel(b)
        with pytest.raises(S.SmcrtError, match="cancelled"):
            sv.wait(b, 10.0)
        assert sv.poll(b)[0] == "CANCELLED"
        sv.wait(a, 30.0)
        assert sv.poll(a)[0] == "DONE"
        with pytest.raises(S.SmcrtError, match="unknown"):
            sv.poll(12345)
    finally:
        sv.close()


def test_server_footprint_is_what_a_served_request_holds(S, W):
    # served requests tally straight into their output grid (no brick grid,
    # in either precision): a request needs its grid and tables, and FP32
    # cubic voxels cost no more than FP64 ones
    G = 64 ** 3 * 8
    cubic = _small_scene(S, W, 64)
    for opts in ({}, {"precision": "f64"}, {"tally_layout": 1}):
        sv = S.Server(device=-1, hbm_budget_bytes=G + G // 8, epoch_packets=100, **opts)
        try:
            sv.wait(sv.submit(cubic, 1, 10)[0], 10.0)
        finally:
            sv.close()
    sv = S.Server(device=-1, hbm_budget_bytes=G - 1, epoch_packets=100)
    try:
        with pytest.raises(S.SmcrtError, match="budget"):
            sv.submit(cubic, 1, 10)
    finally:
        sv.close()


# ---------------------------------------------------------- voxel model

def test_geometry_mode_validation(S, W):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        with pytest.raises(S.SmcrtError, match="unknown mode"):
            S.smcrt_scene_set_geometry(h, 7)
    finally:
        S.smcrt_scene_destroy(h)
    sv = S.Server(device=-1, hbm_budget_bytes=1 << 30, epoch_packets=100)
    try:
        # the voxel model needs a grid: rejected when the scene is packed
        nogrid = S.Scene(dict(W.stack_scene([(0.1, 1.0, 1.5)]), geometry="voxel"))
        with pytest.raises(S.SmcrtError, match="voxel geometry needs a fluence grid"):
            sv.submit(nogrid, 1, 10)
        # with a grid it is accepted, and its footprint counts the voxel bytes
        sdf = S.Scene(W.sphere_scene(n_grid=64))
        vox = S.Scene(dict(W.sphere_scene(n_grid=64), geometry="voxel"))
        for sc in (sdf, vox):
            rid = sv.submit(sc, 1, 100)[0]
            sv.wait(rid, 10.0)
    finally:
        sv.close()
    # FP64 transport (no brick grid): the SDF scene's grid fits, the voxel
    # model's grid plus its voxel bytes do not
    small = S.Server(device=-1, hbm_budget_bytes=64 ** 3 * 8 + 64 ** 3 // 16, epoch_packets=100, precision="f64")
    try:
        small.submit(S.Scene(W.sphere_scene(n_grid=64)), 1, 10)
        with pytest.raises(S.SmcrtError, match="budget"):
            small.submit(S.Scene(dict(W.sphere_scene(n_grid=64), geometry="voxel")), 1, 10)
    finally:
        small.close()


def test_detector_validation(S):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        with pytest.raises(S.SmcrtError, match="face"):
            S.smcrt_scene_set_detector(h, 6, [0, 0], [1, 1], [4, 4])
        with pytest.raises(S.SmcrtError, match="lo < hi"):
            S.smcrt_scene_set_detector(h, 5, [0, 1], [1, 1], [4, 4])
        with pytest.raises(S.SmcrtError, match="negative"):
            S.smcrt_scene_set_detector(h, 5, [0, 0], [1, 1], [-1, 4])
        S.smcrt_scene_set_detector(h, 5, [0, 0], [1, 1], [4, 4])
        S.smcrt_scene_set_detector(h, 9, [0, 0], [1, 1], [0, 0])   # dims 0 remove it (face ignored)
    finally:
        S.smcrt_scene_destroy(h)


def test_detector_pixel_limit(S):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        with pytest.raises(S.SmcrtError, match="2\\^31"):
            S.smcrt_scene_set_detector(h, 5, [0, 0], [1, 1], [65536, 65536])
    finally:
        S.smcrt_scene_destroy(h)


def test_relaxation_validation(S):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        for bad in (0.99, 2.0, float("nan")):
            with pytest.raises(S.SmcrtError, match="omega"):
                S.smcrt_scene_set_relaxation(h, bad)
        S.smcrt_scene_set_relaxation(h, 1.0)
        S.smcrt_scene_set_relaxation(h, 1.9)
    finally:
        S.smcrt_scene_destroy(h)


def test_primitive_placement_and_modifier_validation(S):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        p = S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, 1.0])
        I = [1, 0, 0, 0, 1, 0, 0, 0, 1]
        with pytest.raises(S.SmcrtError, match="no primitive"):
            S.smcrt_scene_set_primitive_placement(h, 5, I, 1.0, [0, 0, 0])
        with pytest.raises(S.SmcrtError, match="orthonormal"):
            S.smcrt_scene_set_primitive_placement(h, p, [2, 0, 0, 0, 1, 0, 0, 0, 1], 1.0, [0, 0, 0])
        with pytest.raises(S.SmcrtError, match="determinant"):
            S.smcrt_scene_set_primitive_placement(h, p, [-1, 0, 0, 0, 1, 0, 0, 0, 1], 1.0, [0, 0, 0])
        with pytest.raises(S.SmcrtError, match="scale"):
            S.smcrt_scene_set_primitive_placement(h, p, I, 0.0, [0, 0, 0])
        S.smcrt_scene_set_primitive_placement(h, p, [0, -1, 0, 1, 0, 0, 0, 0, 1], 2.0, [1, 2, 3])
        with pytest.raises(S.SmcrtError, match=">= 0"):
            S.smcrt_scene_set_primitive_modifiers(h, p, -0.1, 0.0, 0.0)
        with pytest.raises(S.SmcrtError, match="finite"):
            S.smcrt_scene_set_primitive_modifiers(h, p, 0.0, 0.0, float("inf"))
        S.smcrt_scene_set_primitive_modifiers(h, p, 0.1, 0.05, 2.0)
        # a primitive is either twisted or bent
        with pytest.raises(S.SmcrtError, match="twisted or bent"):
            S.smcrt_scene_set_primitive_bend(h, p, 1.0)
        q = S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, 1.0])
        with pytest.raises(S.SmcrtError, match="finite"):
            S.smcrt_scene_set_primitive_bend(h, q, float("nan"))
        with pytest.raises(S.SmcrtError, match="no primitive"):
            S.smcrt_scene_set_primitive_bend(h, 9, 1.0)
        S.smcrt_scene_set_primitive_bend(h, q, 1.5)
        with pytest.raises(S.SmcrtError, match="twisted or bent"):
            S.smcrt_scene_set_primitive_modifiers(h, q, 0.0, 0.0, 1.0)
        S.smcrt_scene_set_primitive_modifiers(h, q, 0.02, 0.0, 0.0)   # rounding of a bent primitive
        S.smcrt_scene_set_primitive_bend(h, q, 0.0)                   # removed: a twist is allowed again
        S.smcrt_scene_set_primitive_modifiers(h, q, 0.0, 0.0, 1.0)
    finally:
        S.smcrt_scene_destroy(h)



def test_elongation_displacement_repetition_validation(S):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        p = S.smcrt_scene_add_primitive(h, 0, [0, 0, 0, 0.1])
        with pytest.raises(S.SmcrtError, match="h must be"):
            S.smcrt_scene_set_primitive_elongation(h, p, [-0.1, 0, 0])
        S.smcrt_scene_set_primitive_elongation(h, p, [0.1, 0, 0])
        with pytest.raises(S.SmcrtError, match="amplitude"):
            S.smcrt_scene_set_primitive_displacement(h, p, -1.0, 2.0)
        S.smcrt_scene_set_primitive_displacement(h, p, 0.01, 20.0)
        with pytest.raises(S.SmcrtError, match="fit their cells"):   # 0.2 + 0.01 elongated radius > half of 0.3
            S.smcrt_scene_set_primitive_repetition(h, p, [0.3, 1, 1], [2, 1, 1])
        with pytest.raises(S.SmcrtError, match="counts"):
            S.smcrt_scene_set_primitive_repetition(h, p, [1, 1, 1], [0, 1, 1])
        S.smcrt_scene_set_primitive_repetition(h, p, [1.0, 1, 1], [3, 1, 1])
    finally:
        S.smcrt_scene_destroy(h)


def test_segment_tracing_validation(S, W):
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        with pytest.raises(S.SmcrtError, match="0 or 1"):
            S.smcrt_scene_set_segment_tracing(h, 2)
        # relaxed and segment-traced steps exclude each other, in either order
        S.smcrt_scene_set_relaxation(h, 1.5)
        with pytest.raises(S.SmcrtError, match="relaxed steps"):
            S.smcrt_scene_set_segment_tracing(h, 1)
        S.smcrt_scene_set_relaxation(h, 1.0)
        S.smcrt_scene_set_segment_tracing(h, 1)
        with pytest.raises(S.SmcrtError, match="segment-traced steps"):
            S.smcrt_scene_set_relaxation(h, 1.5)
        S.smcrt_scene_set_segment_tracing(h, 0)
        S.smcrt_scene_set_relaxation(h, 1.5)
    finally:
        S.smcrt_scene_destroy(h)
    sv = S.Server(device=-1, hbm_budget_bytes=1 << 30, epoch_packets=100)
    try:
        # placed or modified primitives and the voxel model: rejected when packed
        with pytest.raises(S.SmcrtError, match="placed, modified"):
            sv.submit(S.Scene(dict(W.gallery_scene(n_grid=16), segment=True)), 1, 10)
        with pytest.raises(S.SmcrtError, match="voxel model"):
            sv.submit(S.Scene(dict(W.sphere_scene(n_grid=16), geometry="voxel", segment=True)), 1, 10)
        for name in ("glass_sphere", "bottle", "cylinder"):
            rid = sv.submit(S.Scene(dict(W.WORKLOADS[name](n_grid=16), segment=True)), 1, 10)[0]
            sv.wait(rid, 10.0)
    finally:
        sv.close()


def test_scene_distance_validation(S):
    # argument checks come before any device work
    h = S.smcrt_scene_create(1.0, 1e-5, 1e-4)
    try:
        with pytest.raises(S.SmcrtError, match="NULL engine"):
            S.smcrt_scene_distance(None, h, None, 0, 0, None, None, None, None)
    finally:
        S.smcrt_scene_destroy(h)


def test_autotune_batch_validation(S):
    with pytest.raises(S.SmcrtError, match="NULL engine"):
        S.smcrt_engine_autotune_batch(None, [], 1000)
