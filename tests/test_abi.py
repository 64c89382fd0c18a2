"""The C ABI library loads and exports every entry point include/lbm.h
declares; host-side validation works without a GPU (no device calls)."""
import ctypes
import os
import re

import pytest

from paper_2408_15654_amd import lbm, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(lbm.EXPORTS) <= set(names)


def test_params_struct_matches_header_fields():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    body = text[text.index("typedef struct {"):text.index("} lbm_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decl = re.findall(r"\b(int32_t|double)\s+([^;]+);", body)
    names = []
    for _, rest in decl:
        for part in rest.split(","):
            names.append(re.sub(r"\[.*", "", part).strip())
    assert names == [f for f, _ in lbm.lbm_params._fields_]
    # 6 int32 + 16 scalar doubles + 9 rates + 3 scales, no padding
    assert ctypes.sizeof(lbm.lbm_params) == 6 * 4 + (16 + 9 + 3) * 8


def test_workspace_bytes_and_validation_without_device():
    lib = lbm.load()
    pr = workloads.c1_stationary_drop()
    for prec in ("fp64", "fp32"):
        c = lbm.to_c_params(dict(pr.params, precision=prec))
        n = lib.lbm_workspace_bytes(ctypes.byref(c))
        per_site = 2 * 26 * (8 if prec == "fp64" else 4)
        assert n >= 64 * 64 * per_site
    bad = [dict(nx=2), dict(W=0.0), dict(M=-1.0), dict(D=0.0), dict(r=-0.5),
           dict(rhoA=0.0), dict(muB=-1.0), dict(phiA=0.0, phiB=0.0),
           dict(s_free=[[2.5, 1, 1], [1, 1, 1], [1, 1, 1]]), dict(sigma0=-1.0),
           dict(fp16_scale=(2.0 ** -31, 0, 0)), dict(fp16_scale=(0, 2.0 ** 31, 0)),
           dict(fp16_scale=(0, 0, 3.0))]
    for kw in bad:
        c = lbm.to_c_params(dict(pr.params, **kw))
        assert lib.lbm_workspace_bytes(ctypes.byref(c)) == 0, kw
        h = ctypes.c_void_p()
        st = lib.lbm_create(ctypes.byref(c), ctypes.c_void_p(256), 1 << 30, None,
                            ctypes.byref(h))
        assert st == lbm.LBM_EINVAL, kw
        assert h.value is None
        assert lib.lbm_last_error(None)
    for ok in ((2.0 ** -30, 2.0 ** 30, 1.0), (0, 4096.0, 0)):
        c = lbm.to_c_params(dict(pr.params, precision="fp16dev", fp16_scale=ok))
        assert lib.lbm_workspace_bytes(ctypes.byref(c)) > 0, ok
    # too-small workspace
    c = lbm.to_c_params(pr.params)
    h = ctypes.c_void_p()
    st = lib.lbm_create(ctypes.byref(c), ctypes.c_void_p(256), 1024, None, ctypes.byref(h))
    assert st == lbm.LBM_ENOMEM
    # misaligned workspace
    st = lib.lbm_create(ctypes.byref(c), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(h))
    assert st == lbm.LBM_EINVAL
    # queries on a NULL handle
    plan = (ctypes.c_int32 * 3)(7, 7, 7)
    assert lib.lbm_get_tile_plan(None, plan) == lbm.LBM_EINVAL
    assert tuple(plan) == (7, 7, 7)


def test_largest_accepted_grids():
    """Each copy of the 26 population planes is addressed with 32-bit byte
    offsets: the largest square grid per storage precision is accepted and
    one more row and column is refused."""
    lib = lbm.load()
    pr = workloads.c1_stationary_drop()
    for prec, side, bytes_per_pop in (("fp64", 4544, 8), ("fp32", 6426, 4),
                                      ("fp16dev", 9088, 2)):
        assert 26 * side * side * bytes_per_pop <= 0xFFFFFFFF
        assert 26 * (side + 1) ** 2 * bytes_per_pop > 0xFFFFFFFF
        ok = lbm.to_c_params(dict(pr.params, nx=side, ny=side, precision=prec))
        assert lib.lbm_workspace_bytes(ctypes.byref(ok)) > 26 * side * side * bytes_per_pop
        big = lbm.to_c_params(dict(pr.params, nx=side + 1, ny=side + 1, precision=prec))
        assert lib.lbm_workspace_bytes(ctypes.byref(big)) == 0, prec


def test_grids_whose_halo_offset_would_land_are_refused():
    """Halo lanes of the step store at byte offset 0xFFFFFF00, past every
    buffer, where the hardware discards them; a grid whose population planes
    reach that offset (though they fit in 4 GiB) is refused."""
    lib = lbm.load()
    pr = workloads.c1_stationary_drop()
    for prec, nx, ny, bytes_per_pop in (("fp32", 5641, 7321, 4), ("fp64", 11, 1877171, 8),
                                        ("fp16dev", 8969, 9209, 2)):
        n = 26 * nx * ny * bytes_per_pop
        assert 0xFFFFFF00 < n <= 0xFFFFFFFF
        c = lbm.to_c_params(dict(pr.params, nx=nx, ny=ny, precision=prec))
        assert lib.lbm_workspace_bytes(ctypes.byref(c)) == 0, prec


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(ImportError):
        lbm._lib_backup = lbm._lib
        try:
            lbm._lib = None
            lbm.load(str(tmp_path / "missing.so"))
        finally:
            lbm._lib = lbm._lib_backup


def test_batch_entry_points_validate_without_device():
    lib = lbm.load()
    pr = workloads.c1_stationary_drop()
    c = lbm.to_c_params(pr.params)
    assert lib.lbm_batch_instance_bytes(ctypes.byref(c)) == lib.lbm_workspace_bytes(ctypes.byref(c))
    bad = lbm.to_c_params(dict(pr.params, W=0.0))
    assert lib.lbm_batch_instance_bytes(ctypes.byref(bad)) == 0
    assert lib.lbm_batch_overhead_bytes(0) == 0
    assert lib.lbm_batch_overhead_bytes(65537) == 0
    o1, o2 = lib.lbm_batch_overhead_bytes(1), lib.lbm_batch_overhead_bytes(1000)
    assert 0 < o1 < o2 and o2 % 256 == 0
    b = ctypes.c_void_p()
    for args in ((0, 256, 1 << 30), (8, 8, 1 << 30), (8, None, 1 << 30)):
        st = lib.lbm_batch_create(args[0], ctypes.c_void_p(args[1]) if args[1] else None,
                                  args[2], None, ctypes.byref(b))
        assert st == lbm.LBM_EINVAL, args
        assert b.value is None
        assert lib.lbm_batch_last_error(None)
    st = lib.lbm_batch_create(1000, ctypes.c_void_p(256), o2 - 256, None, ctypes.byref(b))
    assert st == lbm.LBM_ENOMEM
    # every call rejects a NULL batch
    assert lib.lbm_batch_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_batch_retire(None, 0) == lbm.LBM_EINVAL
    assert lib.lbm_batch_free_bytes(None) == 0
