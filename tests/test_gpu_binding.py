"""Device views (nh_bind_device_buffers): a solver that steps caller-owned
device tensors in place computes what a solver with its own buffers computes
(bitwise), and malformed views are rejected before anything changes."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1706_04551_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("h", "hu", "hv", "w", "p")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def stored_depth(c, dtype, H=None):
    """What a bound depth tensor holds: h in FP64; in FP32 bulk
    s = h - max(H, 0) (the surface elevation over water, the depth on land),
    formed in FP64 and rounded once, as the library stores a host state
    (against the bathymetry the caller gave, by default the FP64 one)."""
    import torch
    if dtype == torch.float64:
        return c.h
    H = c.H if H is None else H
    return (c.h - np.maximum(H, 0.0)).astype(np.float32)


def tensors(c, dtype):
    import torch
    dev = torch.device("cuda", 0)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dtype,  # noqa
                               device=dev)
    return dict(H=t(c.H), h=t(stored_depth(c, dtype)), hu=t(c.hu),
                hv=t(c.hv),
                w=torch.zeros((c.ny + 1, c.nx + 1), dtype=dtype, device=dev))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_bound_tensors_are_stepped_in_place(precision):
    import torch
    from paper_1706_04551_amd import Solver
    c = I.case_c2(n=160, precision=precision)
    steps = 15
    say(f"[bind] c2 160x160 {precision}, {steps} steps")
    a = Solver.from_case(c)
    a.run(steps)
    ra, sa = a.state(), a.stats()
    a.close()
    dtype = torch.float64 if precision == "f64" else torch.float32
    kw = c.param_dict()
    nx, ny, dx, dy = kw.pop("nx"), kw.pop("ny"), kw.pop("dx"), kw.pop("dy")
    b = Solver(nx, ny, dx, dy, precision=precision,
               stream=torch.cuda.current_stream().cuda_stream, **kw)
    T = tensors(c, dtype)
    b.bind(**T)
    b.run(steps)
    torch.cuda.synchronize()
    rb, sb = b.state(), b.stats()
    for k in FIELDS:
        assert np.array_equal(ra[k], rb[k]), k
    for k in ("t", "sweeps_total", "solves", "step"):
        assert sa[k] == sb[k], k
    # the tensors themselves hold U^n (the depth as stored in FP32:
    # h - max(H, 0))
    Hd = T["H"].double().cpu().numpy()
    dep = T["h"].double().cpu().numpy()
    if precision == "f32":
        dep = dep + np.maximum(Hd, 0.0)
    assert np.array_equal(dep, rb["h"])
    for k, f in (("hu", "hu"), ("hv", "hv"), ("w", "w")):
        assert np.array_equal(T[k].double().cpu().numpy(), rb[f]), k
    # host uploads go into the bound memory (against the bound, FP32,
    # bathymetry)
    b.set_state(c.h, c.hu, c.hv)
    torch.cuda.synchronize()
    assert np.array_equal(T["h"].double().cpu().numpy(),
                          np.asarray(stored_depth(c, dtype, Hd), np.float64))
    b.close()


def test_bathymetry_alone_then_host_state():
    import torch
    from paper_1706_04551_amd import Solver
    c = I.case_c2(n=96)
    kw = c.param_dict()
    nx, ny, dx, dy = kw.pop("nx"), kw.pop("ny"), kw.pop("dx"), kw.pop("dy")
    s = Solver(nx, ny, dx, dy, **kw)
    s.bind(H=torch.tensor(c.H, dtype=torch.float64, device="cuda"))
    s.set_state(c.h, c.hu, c.hv)
    s.run(5)
    r = Solver.from_case(c)
    r.run(5)
    assert np.array_equal(s.state()["h"], r.state()["h"])
    s.close()
    r.close()


def test_malformed_views_are_rejected():
    import torch
    from paper_1706_04551_amd import NhError, Solver
    from paper_1706_04551_amd import binding as B
    c = I.case_c2(n=64)
    s = Solver.from_case(c)
    T = tensors(c, torch.float64)
    with pytest.raises(TypeError):
        s.bind(h=T["h"].float(), hu=T["hu"], hv=T["hv"])       # dtype
    with pytest.raises(TypeError):
        s.bind(h=T["h"].cpu(), hu=T["hu"], hv=T["hv"])         # host tensor
    with pytest.raises(NhError):
        s.bind(h=T["h"], hu=T["hu"])                           # hv missing
    bad = T["h"].clone()
    bad[3, 5] = -1.0
    with pytest.raises(NhError) as e:
        s.bind(h=bad, hu=T["hu"], hv=T["hv"])
    assert e.value.status == -6                                # negative depth
    bad[3, 5] = float("nan")
    with pytest.raises(NhError):
        s.bind(h=bad, hu=T["hu"], hv=T["hv"])                  # non-finite
    with pytest.raises(NhError):
        s.bind(h=T["h"], hu=T["h"], hv=T["hv"])                # overlap
    # below the Python checks: pinned host memory, and a view that runs past
    # the end of its allocation (the library checks before any kernel runs)
    L = B.lib()
    pinned = torch.empty(c.nx * c.ny, dtype=torch.float64, pin_memory=True)
    v = B.NhDeviceViews(None, pinned.data_ptr(), T["hu"].data_ptr(),
                        T["hv"].data_ptr(), None)
    assert L.nh_bind_device_buffers(s._h, ctypes.byref(v)) == -1
    hip = ctypes.CDLL("libamdhip64.so.7")     # the runtime already loaded
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    block = ctypes.c_void_p()
    nbytes = 4 << 20                        # a whole number of pages
    assert hip.hipMalloc(ctypes.byref(block), nbytes) == 0
    tail = block.value + nbytes - 8         # last element: the view of
    v = B.NhDeviceViews(None, tail, T["hu"].data_ptr(),  # 64 x 64 cells runs
                        T["hv"].data_ptr(), None)        # 32 KB past the end
    assert L.nh_bind_device_buffers(s._h, ctypes.byref(v)) == -1
    assert b"past the end" in L.nh_last_error()
    assert hip.hipFree(block) == 0
    # nothing was adopted: the solver still steps its own state
    s.run(3)
    r = Solver.from_case(c)
    r.run(3)
    assert np.array_equal(s.state()["h"], r.state()["h"])
    s.close()
    r.close()
