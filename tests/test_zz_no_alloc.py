"""The allocation-free totals entry point (apm_totals_noalloc, through the C ABI)
against apm_totals on the same inputs: two calls in a row on one context, the second
with fewer particles, and a call from a second context with another hierarchy on the
same device (the fixed scratch is shared per device)."""

import ctypes
import sys

import numpy as np
import pytest

import apm_workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_1410_0010_amd")

DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype))).to(DEV)


def staged(w, dtype):
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, dtype) for a in (w.x, w.y, w.z, w.m))
    owner = ctx.owner(x, y, z)
    gmf = [ctx.deposit(l, x, y, z, m) for l in range(plan.nlevels)]
    fld = []
    for l in range(plan.nlevels):
        fld.append(ctx.accel(l, ctx.solve_level(l, gmf[l]), fld[l - 1] if l > 0 else None))
    ax, ay, az, pot = (torch.zeros(w.npart, dtype=x.dtype, device=DEV) for _ in range(4))
    for l in range(plan.nlevels):
        ctx.interp(l, fld[l], x, y, z, owner, ax, ay, az, pot)
    return ctx, gmf, m, owner, ax, ay, az, pot


def both(ctx, gmf, m, owner, ax, ay, az, pot, n):
    ref = ctx.totals(gmf, m[:n], owner[:n], ax[:n], ay[:n], az[:n], pot[:n])
    out = torch.full((ctx.plan.nlevels + 4,), float("nan"), dtype=torch.float64, device=DEV)
    ctx.totals_noalloc(gmf, m[:n], owner[:n], ax[:n], ay[:n], az[:n], pot[:n], out=out)
    torch.cuda.synchronize()
    return ref, out.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_totals_noalloc_matches_totals(dtype):
    w = W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=2, npart=20000)
    say(f"[noalloc] nested32 npart={w.npart} dtype={dtype.__name__}")
    ctx, gmf, m, owner, ax, ay, az, pot = staged(w, dtype)
    for n in (w.npart, w.npart // 3):                 # the second call is smaller
        ref, got = both(ctx, gmf, m, owner, ax, ay, az, pot, n)
        say(f"[noalloc] npart={n}: {got}")
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), f"npart={n}: {got} vs {ref}"
    # another context and hierarchy (one level fewer) on the same device and array
    w2 = W.workload_plummer_nested(root_n=16, sub_n=8, nlevels=1, npart=5000)
    c2 = staged(w2, dtype)
    ref, got = both(*c2, w2.npart)
    assert np.array_equal(got, ref)
    # and the first context again, after the other one used the array
    ref, got = both(ctx, gmf, m, owner, ax, ay, az, pot, w.npart)
    assert np.array_equal(got, ref)


def test_totals_noalloc_rejects_bad_arguments():
    w = W.workload_plummer_nested(root_n=16, sub_n=8, nlevels=1, npart=100)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    lib = P.lib()
    out = torch.zeros(plan.nlevels + 4, dtype=torch.float64, device=DEV)
    st = lib.apm_totals_noalloc(ctx.handle, P._apm.APM_F64, None, None, None, 0, None, None, None,
                                None, ctypes.c_void_p(out.data_ptr()))
    assert st == P._apm.APM_ERR_INVALID
    g = [torch.zeros(plan.levels[l]["gmf_elems"], dtype=torch.float64, device=DEV)
         for l in range(plan.nlevels)]
    arr = (ctypes.c_void_p * plan.nlevels)(*[t.data_ptr() for t in g])
    st = lib.apm_totals_noalloc(ctx.handle, P._apm.APM_F64, arr, None, None, -1, None, None, None,
                                None, ctypes.c_void_p(out.data_ptr()))
    assert st == P._apm.APM_ERR_RANGE
    st = lib.apm_totals_noalloc(ctx.handle, P._apm.APM_F64, arr, None, None, 0, None, None, None,
                                None, None)
    assert st == P._apm.APM_ERR_INVALID
