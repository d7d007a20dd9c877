"""nh_run_noalloc (the entry point that allocates no device memory) against
the solver entry points it mirrors (nh_create, nh_set_bathymetry,
nh_set_state, nh_run, nh_read_state): the same kernels on the same inputs, so
the states, pressures and statistics must agree bit for bit.  Two calls in a
row per precision, the second on a smaller grid (the static scratch keeps the
first call's contents), the 1D channel, a grid beyond the scratch, and a
negative depth in the caller's buffer."""
import sys

import numpy as np
import pytest

from paper_1706_04551_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("h", "hu", "hv", "w", "p")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference(c, steps):
    from paper_1706_04551_amd import Solver
    s = Solver.from_case(c)
    s.run(steps)
    r, st = s.state(), s.stats()
    s.close()
    return r, st


def noalloc(c, steps, p0=None):
    import torch
    from paper_1706_04551_amd import run_noalloc
    dev = torch.device("cuda", 0)
    dt = torch.float64 if c.precision == "f64" else torch.float32
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt,  # noqa
                               device=dev)
    cs = (c.nx + 1,) if c.ny == 1 else (c.ny + 1, c.nx + 1)
    # the depth buffer holds h in FP64, s = h - max(H, 0) in FP32 bulk
    # (formed in FP64 and rounded once, as the library stores a host state)
    h0 = c.h
    if c.precision == "f32":
        h0 = c.h - np.maximum(c.H, 0.0)
    T = dict(H=t(c.H), h=t(h0), hu=t(c.hu),
             hv=None if c.ny == 1 else t(c.hv),
             w=torch.zeros(cs, dtype=dt, device=dev),
             p=torch.zeros(cs, dtype=torch.float64, device=dev))
    kw = c.param_dict()
    nx, ny, dx, dy = kw.pop("nx"), kw.pop("ny"), kw.pop("dx"), kw.pop("dy")
    kw["precision"] = c.precision
    stream = torch.cuda.current_stream().cuda_stream
    st = run_noalloc(nx, ny, dx, dy, T["H"], T["h"], T["hu"], T["hv"],
                     T["w"], T["p"], steps, stream=stream, **kw)
    torch.cuda.synchronize()
    out = {k: T[k].double().cpu().numpy().reshape(cs if k in ("w", "p")
                                                  else (c.ny, c.nx))
           for k in ("h", "hu", "w", "p")}
    if c.precision == "f32":
        out["h"] = out["h"] + np.maximum(
            T["H"].double().cpu().numpy().reshape(c.ny, c.nx), 0.0)
    out["hv"] = (np.zeros((c.ny, c.nx)) if c.ny == 1
                 else T["hv"].double().cpu().numpy())
    return out, st


def compare(c, steps, tag):
    say(f"[noalloc] {tag}: {c.nx}x{c.ny} {c.precision}, {steps} steps")
    ra, sa = reference(c, steps)
    rb, sb = noalloc(c, steps)
    for k in FIELDS:
        a = ra[k].reshape(rb[k].shape)
        assert np.array_equal(a, rb[k]), (tag, k, np.abs(a - rb[k]).max())
    for k in ("t", "dt", "step", "sweeps_total", "solves", "measure"):
        assert sa[k] == sb[k], (tag, k, sa[k], sb[k])
    # the clamped mass is summed by atomic adds in whatever order the
    # workgroups finish: equal up to that order's rounding
    assert abs(sa["clamped"] - sb["clamped"]) <= 1e-12 * abs(sa["clamped"])
    assert sb["step"] == steps


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_equals_solver_on_two_calls(precision):
    # the second call on a smaller grid reuses the scratch the first left
    compare(I.case_c2(n=160, precision=precision), 12, "first call")
    compare(I.case_c2(n=96, precision=precision), 9, "second, smaller")


def test_noalloc_channel_1d():
    compare(I.case_c1(steps=40), 40, "1D channel")


def test_noalloc_rejects_a_grid_beyond_the_scratch():
    # 1100^2 FP64 needs ~155 MB of intermediate arrays; the buffers are of
    # full size, so nothing would be read out of bounds either way
    import torch
    from paper_1706_04551_amd import NhError, run_noalloc
    n = 1100
    say(f"[noalloc] {n}x{n} f64 beyond the scratch")
    dev = torch.device("cuda", 0)
    H = torch.full((n, n), 5.0, dtype=torch.float64, device=dev)
    h = H.clone()
    z = torch.zeros((n, n), dtype=torch.float64, device=dev)
    hv = z.clone()
    w = torch.zeros((n + 1, n + 1), dtype=torch.float64, device=dev)
    p = w.clone()
    with pytest.raises(NhError) as e:
        run_noalloc(n, n, 1.0, 1.0, H, h, z, hv, w, p, 1, cfl=0.7)
    assert e.value.status == -1 and "scratch" in str(e.value)


def test_noalloc_rejects_a_negative_depth():
    import torch
    from paper_1706_04551_amd import NhError, run_noalloc
    c = I.case_c2(n=64)
    say("[noalloc] 64x64 f64 with a negative depth")
    dev = torch.device("cuda", 0)
    t = lambda a: torch.tensor(np.ascontiguousarray(a),  # noqa
                               dtype=torch.float64, device=dev)
    h = c.h.copy()
    h[10, 20] = -1.0
    w = torch.zeros((c.ny + 1, c.nx + 1), dtype=torch.float64, device=dev)
    with pytest.raises(NhError) as e:
        run_noalloc(c.nx, c.ny, c.dx, c.dy, t(c.H), t(h), t(c.hu), t(c.hv),
                    w, w.clone(), 1, cfl=0.7)
    assert e.value.status == -6
