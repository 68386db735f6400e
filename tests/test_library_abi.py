"""CPU checks of the C-ABI library: it builds, loads next to torch's HIP runtime, exports
every symbol include/vp.h declares, and validates configurations without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "vp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2605_21794_amd._lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libvp.so is not built (run `python -m paper_2605_21794_amd.build`)")
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    import paper_2605_21794_amd._lib as L
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"{n} has no ctypes signature"
    assert set(L.SIGNATURES) == set(names)


def test_single_hip_runtime(lib):
    import paper_2605_21794_amd._lib as L
    assert len(L._hip_runtime_paths()) <= 1


def test_workspace_sizing_and_validation(lib):
    import paper_2605_21794_amd._lib as L
    b = ctypes.c_size_t()
    for ng in (8, 64, 1024):
        c = L.vp_config(n=1000, ng=ng, precision=L.VP_FP32_COMP, L=10.0, dt=0.05, hist_cap=100)
        assert lib.vp_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == L.VP_OK
        assert b.value % 256 == 0 and b.value >= (L.VP_MAX_ACC_COPIES + 8) * ng * 4
    bad = [dict(ng=12), dict(ng=4), dict(ng=2048), dict(n=0), dict(L=-1.0), dict(dt=0.0),
           dict(precision=7), dict(sort_chunk=5000), dict(hist_cap=0), dict(solver=2),
           dict(L=float("nan")), dict(sort_every=-2), dict(projection=3),
           dict(projection=-1), dict(monopole_only=2), dict(no_self_field=3), dict(ext_mode=-1),
           dict(ext_mode=1, ext_amplitude=float("inf")), dict(element_order=3),
           dict(element_order=-1), dict(element_order=2, precision=L.VP_FP32),
           dict(element_order=2, projection=L.VP_PROJ_NODAL),
           dict(element_order=2, projection=L.VP_PROJ_CONSISTENT), dict(moment_order=1),
           dict(moment_order=4), dict(moment_order=3), dict(moment_order=3, element_order=1),
           dict(moment_order=3, element_order=2, precision=L.VP_FP32),
           dict(moment_order=3, element_order=2, monopole_only=1),
           dict(moment_order=3, element_order=2, sort_every=8)]
    for kw in bad:
        args = dict(n=1000, ng=64, precision=L.VP_FP32_COMP, L=10.0, dt=0.05, hist_cap=100)
        args.update(kw)
        c = L.vp_config(**args)
        assert lib.vp_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == L.VP_ERR_ARG, kw
        assert lib.vp_last_error()
    for proj in (L.VP_PROJ_ELEM, L.VP_PROJ_NODAL, L.VP_PROJ_CONSISTENT):
        c = L.vp_config(n=1000, ng=64, precision=L.VP_FP64, L=1.0, dt=0.1, hist_cap=1,
                        projection=proj)
        assert lib.vp_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == L.VP_OK
    c = L.vp_config(n=1000, ng=64, precision=L.VP_FP64, L=1.0, dt=0.1, sort_chunk=2049, hist_cap=1)
    assert lib.vp_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == L.VP_ERR_ARG
    # P2: twice the load-vector nodes (accumulator ring, b~, Phi), in every other precision
    sizes = {}
    for order in (0, 1, 2):
        c = L.vp_config(n=1000, ng=1024, precision=L.VP_FP64, L=1.0, dt=0.1, hist_cap=1,
                        element_order=order)
        assert lib.vp_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == L.VP_OK
        sizes[order] = b.value
    assert sizes[0] == sizes[1]
    assert sizes[2] - sizes[1] >= (3 * L.VP_MAX_ACC_COPIES + 2) * 1024 * 8
    for prec in (L.VP_FP64, L.VP_FP32_COMP, L.VP_FP32_TWOSUM):
        c = L.vp_config(n=1000, ng=64, precision=prec, L=1.0, dt=0.1, hist_cap=1, element_order=2)
        assert lib.vp_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == L.VP_OK
        for mo in (0, 2, 3):   # second moments live in the particle arrays, not the workspace
            c2 = L.vp_config(n=1000, ng=64, precision=prec, L=1.0, dt=0.1, hist_cap=1,
                             element_order=2, moment_order=mo)
            b2 = ctypes.c_size_t()
            assert lib.vp_workspace_bytes(ctypes.byref(c2), ctypes.byref(b2)) == L.VP_OK
            assert b2.value == b.value


def test_null_handles_rejected(lib):
    import paper_2605_21794_amd._lib as L
    assert lib.vp_step(None, 1) == L.VP_ERR_ARG
    assert lib.vp_deposit(None) == L.VP_ERR_ARG
    assert lib.vp_destroy(None) == L.VP_OK
    assert lib.vp_status_string(L.VP_ERR_RANGE) == b"history record out of range"
    assert lib.vp_abi_version() == L.VP_ABI_VERSION == 10
    assert ctypes.sizeof(L.vp_particles) == 8 * 8  # eight array pointers, the moments last
    assert ctypes.sizeof(L.vp_diag) == 8 * 12  # twelve 8-byte fields, stamp last
    assert lib.vp_prepare_step(None, 1) == L.VP_ERR_ARG
    assert lib.vp_wall_clock_hz(None) == L.VP_ERR_ARG


def test_status_strings_of_any_int(lib):
    """Every int has a status string; values outside the enumeration are "unknown status"
    (the library reads the argument as an int, so no out-of-range enum value is loaded)."""
    for v in (0, 1, 2, 3, 4, 5):
        assert lib.vp_status_string(v)
    for v in (-2, -1, 6, 64, 2 ** 31 - 1, -2 ** 31):
        assert lib.vp_status_string(v) == b"unknown status"
