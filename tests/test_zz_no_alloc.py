"""The allocation-free clustering entry point (vp_cluster_markers_static, whose workspace is
the library's own device array) against vp_cluster_markers with a caller workspace, through
the C ABI: bit for bit on two calls in a row, the second with a smaller input (the array
keeps the first call's contents), and the refusals of a too-large input and of bad
arguments."""
from ctypes import byref, c_int32, c_size_t, c_void_p

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("Q", "P", "qs", "ps", "psi")


def _markers(seed, m, L):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.0, L, m)
    p = np.where(rng.uniform(size=m) < 0.5, rng.normal(-1.5, 0.7, m), rng.normal(1.5, 0.7, m))
    w = rng.uniform(0.5, 1.5, m) * (L / m)
    init = rng.choice(m, size=m // 10, replace=False).astype(np.int32)
    return q, p, w, init


def _cluster(lib, torch, q, p, w, init, iters, L, static):
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    qd, pd, wd = t(q, torch.float64), t(p, torch.float64), t(w, torch.float64)
    idx = t(init, torch.int32)
    m, k = int(q.size), int(init.size)
    out = {f: torch.full((k,), -7.0, dtype=torch.float64, device=dev) for f in FIELDS}
    assign = torch.full((m,), -1, dtype=torch.int32, device=dev)
    n = c_int32(-1)
    s = c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    args_in = (c_void_p(qd.data_ptr()), c_void_p(pd.data_ptr()), c_void_p(wd.data_ptr()), m, k,
               c_void_p(idx.data_ptr()), int(iters), float(L))
    args_out = tuple(c_void_p(out[f].data_ptr()) for f in FIELDS) + (
        c_void_p(assign.data_ptr()), byref(n))
    if static:
        st = lib.vp_cluster_markers_static(*args_in, s, *args_out)
    else:
        b = c_size_t()
        assert lib.vp_cluster_workspace_bytes(m, k, byref(b)) == 0
        ws = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
        st = lib.vp_cluster_markers(*args_in, c_void_p(ws.data_ptr()), s, *args_out)
    torch.cuda.synchronize()
    res = {f: out[f][: max(0, n.value)].cpu().numpy() for f in FIELDS}
    res["assign"] = assign.cpu().numpy()
    return st, n.value, res


def test_static_workspace_matches_caller_workspace_on_two_calls(vp):
    import torch
    lib = vp.load_library()
    L = 12.0
    # the second call is smaller: it runs on what the first left in the library's array
    for seed, m in ((1, 160000), (2, 23000)):
        q, p, w, init = _markers(seed, m, L)
        st_ref, n_ref, ref = _cluster(lib, torch, q, p, w, init, 6, L, static=False)
        st, n, got = _cluster(lib, torch, q, p, w, init, 6, L, static=True)
        assert st_ref == 0 and st == 0, (st_ref, st, lib.vp_last_error())
        assert n == n_ref and n > 0.9 * init.size, (n, n_ref)
        for f in FIELDS + ("assign",):
            assert np.array_equal(got[f], ref[f]), (m, f)
        assert np.all(got["assign"] >= 0) and np.all(got["assign"] < init.size)


def test_static_workspace_refuses_what_does_not_fit(vp):
    import torch
    lib = vp.load_library()
    L = 12.0
    q, p, w, _ = _markers(3, 600000, L)
    init = np.arange(60000, dtype=np.int32)
    st, n, _ = _cluster(lib, torch, q, p, w, init, 1, L, static=True)
    assert st == vp._lib.VP_ERR_ARG and n == -1
    assert b"static workspace holds" in lib.vp_last_error()
    # an out-of-range starting index is refused (checked on the device), as is a NULL pointer
    q, p, w, init = _markers(4, 5000, L)
    init[7] = 5000
    st, _, _ = _cluster(lib, torch, q, p, w, init, 1, L, static=True)
    assert st == vp._lib.VP_ERR_ARG and b"starting indices" in lib.vp_last_error()
    n = c_int32(-1)
    assert lib.vp_cluster_markers_static(None, None, None, 10, 2, None, 1, 1.0, None, None, None,
                                         None, None, None, None, byref(n)) == vp._lib.VP_ERR_ARG
    # a call after the refusals still matches the caller-workspace version
    q, p, w, init = _markers(5, 40000, L)
    _, n_ref, ref = _cluster(lib, torch, q, p, w, init, 4, L, static=False)
    st, n, got = _cluster(lib, torch, q, p, w, init, 4, L, static=True)
    assert st == 0 and n == n_ref
    for f in FIELDS + ("assign",):
        assert np.array_equal(got[f], ref[f]), f
