"""The C ABI's contract, exercised without a GPU.

Argument validation happens before any HIP call, so every error path below
runs on a host without a device.  The library must load and export every
function ``include/ps.h`` declares.
"""
import ctypes
import os
import re

import pytest

from conftest import ROOT, gpu_available
from paper_2409_02294_amd import solver as S

HEADER = os.path.join(ROOT, "include", "ps.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = S.load()
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(S.EXPORTS)


def test_status_strings():
    for code in (S.PS_OK, S.PS_ERR_INVALID, S.PS_ERR_UNSUPPORTED, S.PS_ERR_NOT_READY, S.PS_ERR_DEVICE,
                 S.PS_ERR_CAPTURE):
        assert S.ps_status_str(code)
    assert S.ps_status_str(12345) == "unknown status"


@pytest.mark.parametrize("n,dx,prec,status", [
    (0, 0.1, S.PS_F64, S.PS_ERR_INVALID),
    (-4, 0.1, S.PS_F64, S.PS_ERR_INVALID),
    (32, 0.0, S.PS_F64, S.PS_ERR_INVALID),
    (32, -1.0, S.PS_F32, S.PS_ERR_INVALID),
    (32, float("nan"), S.PS_F32, S.PS_ERR_INVALID),
    (32, float("inf"), S.PS_F32, S.PS_ERR_INVALID),
    (32, 0.1, 7, S.PS_ERR_INVALID),
    (32, 0.1, -1, S.PS_ERR_INVALID),
    (56, 0.1, S.PS_F64, S.PS_ERR_UNSUPPORTED),   # 112 = 2^4 * 7
    (44, 0.1, S.PS_F64, S.PS_ERR_UNSUPPORTED),   # 88 = 2^3 * 11
    (1024, 0.1, S.PS_F64, S.PS_ERR_UNSUPPORTED),  # beyond the largest compiled length
    (7, 0.1, S.PS_F64, S.PS_ERR_UNSUPPORTED),
])
def test_plan_create_rejects(n, dx, prec, status):
    with pytest.raises(S.PSError) as e:
        S.ps_plan_create(n, dx, prec)
    assert e.value.status == status
    assert S.ps_last_error()


def test_plan_create_null_out():
    lib = S.load()
    assert lib.ps_plan_create(None, 32, 0.1, S.PS_F64, None) == S.PS_ERR_INVALID


@pytest.mark.parametrize("n", S.SUPPORTED_N)
@pytest.mark.parametrize("prec", [S.PS_F64, S.PS_F32])
def test_plan_layout_and_query(n, prec):
    p = S.ps_plan_create(n, 1.0 / n, prec)
    try:
        info = S.ps_plan_query(p)
        assert info["n"] == n and info["p"] == 2 * n and info["h"] == n + 1
        assert not info["ready"]
        prod = 1
        for r in info["radices"]:
            assert r in (2, 3, 4, 5, 6, 8, 10, 12, 15, 16, 20)
            prod *= r
        assert prod == 2 * n
        assert info["radices"][0] == 16
        rb = 8 if prec == S.PS_F64 else 4
        h = n + 1
        assert info["ghat_bytes"] == h ** 3 * rb
        ws = S.ps_plan_workspace_bytes(p)
        # Ghat + T1 (H N N complex) + T2 (H 2N N complex) at least
        assert ws >= h ** 3 * rb + 3 * h * n * n * 2 * rb
        assert ws % 256 == 0
    finally:
        S.ps_plan_destroy(p)


def test_calls_on_unbuilt_plan():
    lib = S.load()
    p = S.ps_plan_create(32, 1.0 / 32, S.PS_F64)
    try:
        # NULL / misaligned / overlapping pointers are rejected first
        assert lib.ps_solve(p, None, 0x1000, None) == S.PS_ERR_INVALID
        assert lib.ps_solve(p, 0x1000, None, None) == S.PS_ERR_INVALID
        assert lib.ps_solve(p, 0x1004, 0x100000, None) == S.PS_ERR_INVALID
        assert lib.ps_solve(p, 0x100000, 0x100000 + 8, None) == S.PS_ERR_INVALID
        # well-formed arguments on a plan without a built kernel
        assert lib.ps_solve(p, 0x100000, 0x10000000, None) == S.PS_ERR_NOT_READY
        assert lib.ps_debug_pass(p, 0, 0x100000, 0x10000000, None) == S.PS_ERR_NOT_READY
        assert lib.ps_debug_pass(p, 5, 0x100000, 0x10000000, None) == S.PS_ERR_INVALID
        assert lib.ps_debug_pass(p, 1, 0x100000, 0x100000, None) == S.PS_ERR_INVALID
        assert lib.ps_green_build(p, None, 1.0, 2.38, None) == S.PS_ERR_INVALID
        assert lib.ps_green_build(p, 0x100010, 1.0, 2.38, None) == S.PS_ERR_INVALID
        assert lib.ps_green_build(p, 0x100000, float("nan"), 2.38, None) == S.PS_ERR_INVALID
    finally:
        S.ps_plan_destroy(p)


def test_stream_copy_contract():
    lib = S.load()
    assert lib.ps_stream_copy(None, 0x100000, 16, None) == S.PS_ERR_INVALID
    assert lib.ps_stream_copy(0x100000, None, 16, None) == S.PS_ERR_INVALID
    assert lib.ps_stream_copy(0x100008, 0x200000, 16, None) == S.PS_ERR_INVALID   # misaligned
    assert lib.ps_stream_copy(0x100000, 0x200000, 24, None) == S.PS_ERR_INVALID   # not a multiple of 16
    assert lib.ps_stream_copy(0x100000, 0x100010, 64, None) == S.PS_ERR_INVALID   # overlap


def test_null_plan_and_batch_arguments():
    lib = S.load()
    assert lib.ps_solve(None, 0x100000, 0x10000000, None) == S.PS_ERR_INVALID
    assert lib.ps_plan_workspace_bytes(None, None) == S.PS_ERR_INVALID
    assert lib.ps_plan_query(None, None) == S.PS_ERR_INVALID
    lib.ps_plan_destroy(None)
    arr = ctypes.c_void_p * 1
    assert lib.ps_solve_batched(None, 1, arr(0x1000), arr(0x2000), None) == S.PS_ERR_INVALID
    p = S.ps_plan_create(16, 1.0 / 16, S.PS_F32)
    try:
        assert lib.ps_solve_batched(arr(p), 0, arr(0x100000), arr(0x10000000), None) == S.PS_ERR_INVALID
        assert lib.ps_solve_batched(arr(p), -3, arr(0x100000), arr(0x10000000), None) == S.PS_ERR_INVALID
    finally:
        S.ps_plan_destroy(p)


@pytest.mark.skipif(gpu_available(), reason="needs a host without a GPU")
def test_device_errors_are_reported_not_raised():
    lib = S.load()
    p = S.ps_plan_create(16, 1.0 / 16, S.PS_F64)
    try:
        rc = lib.ps_green_build(p, 0x100000, 1.0, 2.38, None)
        assert rc == S.PS_ERR_DEVICE
        assert S.ps_last_error()
    finally:
        S.ps_plan_destroy(p)


def test_variant_selection_contract():
    p = S.ps_plan_create(32, 1.0 / 32, S.PS_F32)
    q = S.ps_plan_create(256, 1.0 / 256, S.PS_F64)
    try:
        lib = S.load()
        assert lib.ps_plan_set_variant(p, 7, 0) == S.PS_ERR_INVALID
        assert lib.ps_plan_set_variant(p, 6, 2) == S.PS_ERR_INVALID     # z tile: 0 (full) or 1 (half)
        assert lib.ps_plan_set_variant(p, 6, 1) == S.PS_OK
        assert S.ps_plan_query(p)["z_tile"] == 1
        assert lib.ps_plan_set_variant(q, 6, 1) == S.PS_OK
        # x passes: 8 / 16 / 32 rows per workgroup, the family in the low bit
        assert lib.ps_plan_set_variant(p, 0, 2) == S.PS_OK and lib.ps_plan_set_variant(p, 4, 4) == S.PS_OK
        assert lib.ps_plan_set_variant(p, 0, 3) == S.PS_ERR_UNSUPPORTED  # 8 rows, radix-32 family: none at P = 64
        assert lib.ps_plan_set_variant(p, 0, 6) == S.PS_ERR_INVALID
        # y passes: half tile (4: radix-16 family, 5: radix-32 family)
        assert lib.ps_plan_set_variant(p, 1, 4) == S.PS_OK and lib.ps_plan_set_variant(p, 3, 4) == S.PS_OK
        assert lib.ps_plan_set_variant(p, 1, 5) == S.PS_ERR_UNSUPPORTED
        assert lib.ps_plan_set_variant(p, 3, 8) == S.PS_ERR_INVALID
        assert lib.ps_plan_set_variant(p, 3, 6) == S.PS_ERR_UNSUPPORTED  # half-LDS y exchange: P >= 512
        assert lib.ps_plan_set_variant(q, 3, 5) == S.PS_OK
        assert lib.ps_plan_set_variant(q, 4, 5) == S.PS_OK               # 32 rows, radix-32 family, FP64 P = 512
        r = S.ps_plan_create(512, 1.0 / 512, S.PS_F64)
        try:
            assert lib.ps_plan_set_variant(r, 0, 4) == S.PS_ERR_UNSUPPORTED  # 32 FP64 rows of 1024: too much LDS
            assert lib.ps_plan_set_variant(r, 0, 2) == S.PS_OK
            # half-LDS z and y exchanges: FP64 and FP32 cubes with P >= 512
            assert lib.ps_plan_set_variant(r, 2, 5) == S.PS_OK and lib.ps_plan_set_variant(r, 2, 6) == S.PS_ERR_INVALID
            assert lib.ps_plan_set_variant(r, 1, 7) == S.PS_OK and lib.ps_plan_set_variant(r, 3, 6) == S.PS_OK
        finally:
            S.ps_plan_destroy(r)
        r = S.ps_plan_create(512, 1.0 / 512, S.PS_F32)
        try:
            assert lib.ps_plan_set_variant(r, 0, 4) == S.PS_OK and lib.ps_plan_set_variant(r, 4, 5) == S.PS_OK
            assert lib.ps_plan_set_variant(r, 2, 5) == S.PS_OK
        finally:
            S.ps_plan_destroy(r)
        assert lib.ps_plan_set_variant(p, 5, 6) == S.PS_ERR_UNSUPPORTED  # product terms: split plans only
        assert lib.ps_plan_set_variant(p, 2, 6) == S.PS_ERR_INVALID
        assert lib.ps_plan_set_variant(p, 2, 5) == S.PS_ERR_UNSUPPORTED  # P = 64
        sp = S.ps_plan_create(256, 1.0 / 256, S.PS_F32_SPLIT)
        try:
            assert lib.ps_plan_set_variant(sp, 2, 5) == S.PS_ERR_UNSUPPORTED  # split plans: radix-16 stages only
            assert lib.ps_plan_set_variant(sp, 1, 6) == S.PS_ERR_UNSUPPORTED
        finally:
            S.ps_plan_destroy(sp)
        assert lib.ps_plan_set_variant(p, 0, -1) == S.PS_ERR_INVALID
        assert lib.ps_plan_set_variant(p, 0, 1) == S.PS_ERR_UNSUPPORTED  # no radix-32 family at P = 64
        assert lib.ps_plan_set_variant(p, 2, 2) == S.PS_ERR_UNSUPPORTED
        assert lib.ps_plan_set_variant(p, 3, 3) == S.PS_ERR_UNSUPPORTED  # persistent, radix-32 family
        assert lib.ps_plan_set_variant(p, 3, 2) == S.PS_OK               # persistent, radix-16 family
        assert lib.ps_plan_set_variant(p, 2, 3) == S.PS_OK               # persistent z pass, radix-16 family
        S.ps_plan_set_variant(p, 3, 0)
        S.ps_plan_set_variant(p, 2, 0)
        assert S.ps_plan_query(p)["variant"][2] == 0
        S.ps_plan_set_variant(q, 0, 1)
        S.ps_plan_set_variant(q, 2, 2)
        v = S.ps_plan_query(q)["variant"]
        assert v[0] == 1 and v[2] == 2
        assert lib.ps_autotune(p, None, None) == S.PS_ERR_NOT_READY
    finally:
        S.ps_plan_destroy(p)
        S.ps_plan_destroy(q)


def test_spacing_contract():
    lib = S.load()
    p = S.ps_plan_create(32, 0.1, S.PS_F64)
    try:
        info = S.ps_plan_query(p)
        assert info["dx"] == 0.1 and info["dy"] == 0.1 and info["dz"] == 0.1
        for dy, dz in [(0.0, 0.1), (0.1, -1.0), (float("nan"), 0.1), (0.1, float("inf"))]:
            assert lib.ps_plan_set_spacing(p, dy, dz) == S.PS_ERR_INVALID
        S.ps_plan_set_spacing(p, 0.2, 0.05)
        info = S.ps_plan_query(p)
        assert (info["dx"], info["dy"], info["dz"]) == (0.1, 0.2, 0.05) and not info["ready"]
        assert lib.ps_plan_set_spacing(None, 0.1, 0.1) == S.PS_ERR_INVALID
    finally:
        S.ps_plan_destroy(p)


def test_tuning_cache_is_read(tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text("64 f32 0 0 0 0 0\n512 f32 0 1 1 0 1\n512 f64 1 1 2 1 1 1\n")
    p = S.ps_plan_create(256, 1.0 / 256, S.PS_F32, str(path))
    try:
        info = S.ps_plan_query(p)
        assert info["variant"] == [0, 1, 1, 0, 1] and info["z_tile"] == 0  # a line without the z tile: 0
    finally:
        S.ps_plan_destroy(p)
    p = S.ps_plan_create(256, 1.0 / 256, S.PS_F64, str(path))
    try:
        info = S.ps_plan_query(p)
        assert info["variant"] == [1, 1, 2, 1, 1] and info["z_tile"] == 1
    finally:
        S.ps_plan_destroy(p)
    # a missing file keeps the defaults (the forward y pass exchanging through
    # half the LDS and the persistent z pass at P = 512, radix-16 family
    # elsewhere)
    p = S.ps_plan_create(256, 1.0 / 256, S.PS_F32, str(tmp_path / "absent.txt"))
    try:
        assert S.ps_plan_query(p)["variant"] == [0, 6, 3, 0, 0]
    finally:
        S.ps_plan_destroy(p)
    # a split plan keeps its product-term count under a cached line; a line
    # naming variants the plan cannot run is ignored
    path.write_text("512 f32_split 0 0 0 0 0\n256 f32 0 0 9 0 0\n512 f32_split 0 1 3 0 0\n")
    p = S.ps_plan_create(256, 1.0 / 256, S.PS_F32_SPLIT, str(path))
    try:
        info = S.ps_plan_query(p)
        assert info["variant"] == [0, 0, 0, 0, 0] and info["split_terms"] == 6
    finally:
        S.ps_plan_destroy(p)
    p = S.ps_plan_create(128, 1.0 / 128, S.PS_F32, str(path))
    try:
        assert S.ps_plan_query(p)["variant"] == [0, 0, 1, 0, 0]  # zmode 9 does not exist: defaults kept
    finally:
        S.ps_plan_destroy(p)
    # measured defaults: variants and z tile
    for n, prec, want, zt in [(512, S.PS_F32, [0, 7, 3, 3, 2], 0), (512, S.PS_F64, [2, 1, 5, 2, 2], 0),
                              (256, S.PS_F64, [2, 1, 5, 0, 2], 0), (384, S.PS_F32_SPLIT, [0, 0, 1, 4, 2], 1),
                              (128, S.PS_F32, [0, 0, 1, 0, 0], 0), (512, S.PS_F32_SPLIT, [0, 0, 1, 4, 0], 1),
                              (384, S.PS_F32, [0, 7, 5, 7, 2], 0), (16, S.PS_F64, [0, 0, 1, 0, 0], 0)]:
        p = S.ps_plan_create(n, 1.0 / n, prec, None)
        try:
            info = S.ps_plan_query(p)
            assert (info["variant"], info["z_tile"]) == (want, zt), (n, prec)
        finally:
            S.ps_plan_destroy(p)


def test_split_plan_contract():
    p = S.ps_plan_create(256, 1.0 / 256, S.PS_F32_SPLIT)
    try:
        info = S.ps_plan_query(p)
        assert info["split_terms"] == 6
        assert info["variant"] == [0, 0, 4, 4, 0] and info["z_tile"] == 1
        lib = S.load()
        assert lib.ps_plan_set_variant(p, 5, 4) == S.PS_ERR_INVALID
        assert lib.ps_plan_set_variant(p, 0, 1) == S.PS_ERR_UNSUPPORTED   # keeps the radix-16 family
        assert lib.ps_plan_set_variant(p, 2, 2) == S.PS_ERR_UNSUPPORTED
        assert lib.ps_plan_set_variant(p, 2, 3) == S.PS_OK   # persistent split z pass (radix-16 family)
        assert lib.ps_plan_set_variant(p, 2, 4) == S.PS_OK
        assert lib.ps_plan_set_variant(p, 1, 2) == S.PS_OK   # persistent split y pass
        S.ps_plan_set_variant(p, 5, 3)
        assert S.ps_plan_query(p)["split_terms"] == 3
        assert S.ps_plan_workspace_bytes(p) >= S.ps_plan_workspace_bytes(S.ps_plan_create(256, 1.0 / 256, S.PS_F32))
    finally:
        S.ps_plan_destroy(p)


def test_host_solve_contract():
    # staging size and every argument check of ps_solve_host, before any HIP call
    lib = S.load()
    p = S.ps_plan_create(64, 1.0 / 64, S.PS_F32)
    q = S.ps_plan_create(48, 1.0 / 48, S.PS_F64)
    try:
        assert S.ps_host_stage_bytes(p) == 4 * 64 ** 3 * 4
        assert S.ps_host_stage_bytes(q) == 4 * ((48 ** 3 * 8 + 255) // 256 * 256)
        vp = ctypes.c_void_p
        host = [ctypes.create_string_buffer(64 ** 3 * 4) for _ in range(4)]
        rho = (vp * 2)(ctypes.addressof(host[0]), ctypes.addressof(host[1]))
        phi = (vp * 2)(ctypes.addressof(host[2]), ctypes.addressof(host[3]))
        stage, nb = 0x100000, S.ps_host_stage_bytes(p)  # never dereferenced: every case fails first
        assert lib.ps_solve_host(p, None, phi, 2, stage, nb, None) == S.PS_ERR_INVALID
        assert lib.ps_solve_host(p, rho, phi, 0, stage, nb, None) == S.PS_ERR_INVALID
        assert lib.ps_solve_host(p, rho, phi, 2, None, nb, None) == S.PS_ERR_INVALID
        assert lib.ps_solve_host(p, rho, phi, 2, stage + 8, nb, None) == S.PS_ERR_INVALID  # alignment
        assert lib.ps_solve_host(p, rho, phi, 2, stage, nb - 1, None) == S.PS_ERR_INVALID  # too small
        same = (vp * 2)(ctypes.addressof(host[0]), ctypes.addressof(host[1]))
        assert lib.ps_solve_host(p, rho, same, 2, stage, nb, None) == S.PS_ERR_INVALID    # rho is phi
        # the output of one solve on another solve's input, or on another output
        cross = (vp * 2)(ctypes.addressof(host[2]), ctypes.addressof(host[0]))
        assert lib.ps_solve_host(p, rho, cross, 2, stage, nb, None) == S.PS_ERR_INVALID
        assert "overlaps an array of solve" in lib.ps_last_error().decode()
        twice = (vp * 2)(ctypes.addressof(host[2]), ctypes.addressof(host[2]))
        assert lib.ps_solve_host(p, rho, twice, 2, stage, nb, None) == S.PS_ERR_INVALID
        assert lib.ps_solve_host(p, rho, phi, 2, stage, nb, None) == S.PS_ERR_NOT_READY   # no Green's function
        assert "ps_green_build" in lib.ps_last_error().decode()
    finally:
        S.ps_plan_destroy(p)
        S.ps_plan_destroy(q)


def test_box_plan_contract():
    # boxes of nx x ny x nz cells: argument checks, layout, defaults and the
    # variants a box may run, all before any HIP call
    lib = S.load()
    for dims, status in [((0, 16, 16), S.PS_ERR_INVALID), ((16, -8, 16), S.PS_ERR_INVALID),
                         ((16, 56, 16), S.PS_ERR_UNSUPPORTED), ((16, 16, 1024), S.PS_ERR_UNSUPPORTED)]:
        with pytest.raises(S.PSError) as e:
            S.ps_plan_create_box(*dims, 0.1, 0.1, 0.1, S.PS_F32)
        assert e.value.status == status
    for sp in [(0.0, 0.1, 0.1), (0.1, float("nan"), 0.1), (0.1, 0.1, -1.0)]:
        with pytest.raises(S.PSError) as e:
            S.ps_plan_create_box(16, 32, 48, *sp, S.PS_F64)
        assert e.value.status == S.PS_ERR_INVALID
    for prec in (S.PS_F64_PLAIN, S.PS_F32_PLAIN):
        with pytest.raises(S.PSError) as e:
            S.ps_plan_create_box(16, 32, 48, 0.1, 0.1, 0.1, prec)
        assert e.value.status == S.PS_ERR_UNSUPPORTED
    nx, ny, nz = 40, 256, 24
    p = S.ps_plan_create_box(nx, ny, nz, 0.1, 0.2, 0.3, S.PS_F32)
    try:
        info = S.ps_plan_query(p)
        assert (info["nx"], info["ny"], info["nz"]) == (nx, ny, nz)
        assert (info["dx"], info["dy"], info["dz"]) == (0.1, 0.2, 0.3)
        assert info["n"] == nx and info["p"] == 2 * nx and info["h"] == nx + 1
        hx, hpx = nx + 1, (nx + 1 + 15) // 16 * 16
        assert info["t2_offset"] - info["t1_offset"] >= max(hx, hpx) * nz * ny * 8
        assert info["t3_offset"] - info["t2_offset"] >= hx * 2 * ny * nz * 8
        assert info["variant"] == [0, 1, 1, 0, 0]  # radix-32 family for y (P = 512), wave-owned z
        assert S.ps_host_stage_bytes(p) == 4 * ((nx * ny * nz * 4 + 255) // 256 * 256)
        assert lib.ps_plan_set_variant(p, 1, 2) == S.PS_ERR_UNSUPPORTED   # persistent y pass: cubes only
        assert lib.ps_plan_set_variant(p, 1, 7) == S.PS_ERR_UNSUPPORTED   # half-LDS y exchange: cubes only
        assert lib.ps_plan_set_variant(p, 2, 3) == S.PS_ERR_UNSUPPORTED   # persistent z pass: cubes only
        assert lib.ps_plan_set_variant(p, 2, 2) == S.PS_ERR_UNSUPPORTED   # P = 48 along z: no radix-32 family
        assert lib.ps_plan_set_variant(p, 0, 1) == S.PS_ERR_UNSUPPORTED   # P = 80 along x: no radix-32 family
        assert lib.ps_plan_set_variant(p, 0, 2) == S.PS_ERR_UNSUPPORTED   # boxes: 16 rows per x tile
        assert lib.ps_plan_set_variant(p, 1, 4) == S.PS_ERR_UNSUPPORTED   # boxes: full y tile
        assert lib.ps_plan_set_variant(p, 4, 4) == S.PS_ERR_UNSUPPORTED
        assert lib.ps_plan_set_variant(p, 3, 1) == S.PS_OK
        assert lib.ps_solve(p, 0x100000, 0x10000000, None) == S.PS_ERR_NOT_READY
    finally:
        S.ps_plan_destroy(p)
    # equal lengths: exactly the cubic plan
    a = S.ps_plan_create_box(64, 64, 64, 1 / 64, 1 / 64, 1 / 64, S.PS_F32)
    b = S.ps_plan_create(64, 1 / 64, S.PS_F32)
    try:
        qa, qb = S.ps_plan_query(a), S.ps_plan_query(b)
        assert qa == qb
    finally:
        S.ps_plan_destroy(a)
        S.ps_plan_destroy(b)


def test_static_solve_contract():
    # the allocation-free solve's checks, all before any HIP call
    lib = S.load()
    assert lib.ps_solve_static(None, 0x100000, 0x10000000, None) == S.PS_ERR_INVALID
    p = S.ps_plan_create(64, 1 / 64, S.PS_F32)
    q = S.ps_plan_create(160, 1 / 160, S.PS_F32)
    r = S.ps_plan_create(32, 1 / 32, S.PS_F64_PLAIN)
    try:
        assert lib.ps_solve_static(p, None, 0x10000000, None) == S.PS_ERR_INVALID
        assert lib.ps_solve_static(p, 0x100000, 0x100000 + 64, None) == S.PS_ERR_INVALID   # overlap
        assert lib.ps_solve_static(p, 0x100000, 0x10000000, None) == S.PS_ERR_NOT_READY
        assert lib.ps_solve_static(q, 0x100000, 0x10000000, None) == S.PS_ERR_UNSUPPORTED  # beyond the scratch
        assert "static scratch" in lib.ps_last_error().decode()
        assert lib.ps_solve_static(r, 0x100000, 0x10000000, None) == S.PS_ERR_UNSUPPORTED  # plain method
    finally:
        for h in (p, q, r):
            S.ps_plan_destroy(h)
