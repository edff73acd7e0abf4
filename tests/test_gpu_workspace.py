"""Workspace hygiene on the GPU: no kernel reads workspace memory that the same
solve did not write first (a solve on a workspace prefilled with NaN bytes and
one prefilled with zeros give bitwise identical results), plans sharing one
workspace, and non-finite sources reported by every dtype."""

import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

# (shape (nz, ny, nx), bc, dtype, extra Plan arguments, solve mode)
CASES = [
    ((12, 16, 24), "PPPPNN", "f64", {}, "solve"),
    ((12, 16, 24), "PPPPNN", "f32", {}, "solve"),
    ((12, 16, 24), "PPPPNN", "f32_refined", {}, "solve"),
    ((9, 12, 18), "DDNNDN", "f64", {}, "solve"),
    ((10, 12, 16), "NNPPNN", "f64", {"gauge": "pin"}, "adjoint"),
    ((9, 8, 12), "PPNNPP", "f64", {}, "solve"),             # periodic z
    ((9, 8, 12), "PPNNPP", "f32_refined", {}, "solve"),
    ((8, 12, 16), "DDNNNN", "f64", {}, "faces"),
    ((8, 12, 16), "DDNNNN", "f32_refined", {}, "faces"),
    ((16, 12, 8), "PPPPDD", "f64", {"zsolver": "cr"}, "solve"),
    ((16, 12, 8), "NNPPND", "f64", {"zsolver": "pcr"}, "solve"),
    ((8, 512, 512), "PPPPNN", "f64", {}, "solve"),           # exact-count kernel forms
    ((8, 512, 512), "PPPPNN", "f32_refined", {}, "solve"),
    ((7, 9, 6), "DDDDDD", "f64", {"batch": 3}, "solve"),
]


def _run(shape, bc, dtype, kw, mode, fill, rng_seed):
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import to_dev
    kw = dict(kw)
    batch = kw.pop("batch", 1)
    rng = np.random.default_rng(rng_seed)
    h = (1.0 / shape[2], 1.0 / shape[1], 1.0 / shape[0]) if shape[1] >= 512 else (0.7, 1.1, 0.9)
    plan = Plan(shape, bc, h, dtype=dtype, batch=batch, **kw)
    plan.workspace.fill_(fill)   # 0xFF bytes: NaN in every float and double
    tdt = torch.float32 if dtype == "f32" else torch.float64
    f = to_dev(rng.standard_normal((batch,) + shape), tdt)
    if mode == "adjoint":
        u = plan.adjoint(f)
    elif mode == "faces":
        faces = [None] * 6
        for i in range(6):
            if bc[i] != "P":
                faces[i] = to_dev(rng.standard_normal(plan.face_shape(i)), tdt)
        u = plan.solve(f, faces=faces)
    else:
        u = plan.solve(f)
    torch.cuda.synchronize()
    return u.cpu().numpy(), f.cpu().numpy(), h


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[1]}-{c[2]}-{c[4]}-{c[0]}")
def test_nan_and_zero_filled_workspace_agree(case):
    from gpu_util import banner
    shape, bc, dtype, kw, mode = case
    banner(f"workspace fill {case}")
    u_nan, f, h = _run(shape, bc, dtype, kw, mode, 255, 11)
    u_zero, _, _ = _run(shape, bc, dtype, kw, mode, 0, 11)
    assert np.all(np.isfinite(u_nan))
    assert np.array_equal(u_nan.view(np.uint8), u_zero.view(np.uint8))
    if mode == "solve" and dtype != "f32" and not kw and shape[1] < 512:
        from gpu_util import rel_max
        for b in range(f.shape[0]):
            assert rel_max(u_nan[b], oracle.solve(f[b], bc, h)) < 1e-12


def test_two_plans_share_one_workspace():
    """Alternating solves of two plans through one workspace pointer (C ABI):
    each call finds the other plan's tables there and uploads its own."""
    import torch
    from paper_1909_05423_amd import _lib
    from gpu_util import banner, to_dev, rel_max
    banner("two plans, one workspace")
    lib = _lib.load()
    specs = [((6, 8, 12), "PPPPNN", (1.0, 1.0, 1.0)), ((10, 12, 9), "DDNNDD", (0.5, 0.8, 1.3))]
    plans = []
    for (nz, ny, nx), bc, h in specs:
        p = ctypes.c_void_p()
        assert lib.pp_plan_create(nx, ny, nz, bc.encode(), (ctypes.c_double * 3)(*h), 0, 1, ctypes.byref(p)) == 0
        plans.append(p)
    try:
        nbytes = max(lib.pp_plan_workspace_bytes(p) for p in plans)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        rng = np.random.default_rng(31)
        fs = [rng.standard_normal(s) for s, _, _ in specs]
        fd = [to_dev(f) for f in fs]
        ud = [torch.empty_like(x) for x in fd]
        stream = torch.cuda.current_stream().cuda_stream
        for _ in range(3):
            for k, p in enumerate(plans):
                ud[k].fill_(float("nan"))
                st = lib.pp_solve(p, ctypes.c_void_p(fd[k].data_ptr()), ctypes.c_void_p(ud[k].data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(stream))
                assert st == 0
                torch.cuda.synchronize()
                (s, bc, h) = specs[k]
                assert rel_max(ud[k].cpu().numpy(), oracle.solve(fs[k], bc, h)) < 1e-12, (k, bc)
    finally:
        for p in plans:
            lib.pp_plan_destroy(p)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32_refined"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_source_reported_every_dtype(dtype, bad):
    """An Inf or NaN in f is reported as PP_ERR_NONFINITE: by the refined solve
    itself, by last_info for the plain solves."""
    import torch
    from paper_1909_05423_amd import Plan, _lib
    from gpu_util import to_dev
    f = np.random.default_rng(4).standard_normal((6, 8, 12))
    f[2, 3, 4] = bad
    plan = Plan((6, 8, 12), "PPPPNN", (1, 1, 1), dtype=dtype)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    with pytest.raises(_lib.PPError) as ei:
        plan.solve(to_dev(f, tdt))
        plan.last_info()
    assert ei.value.status == -8
    torch.cuda.synchronize()


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 22) + 16 * 37])
def test_stream_copy_copies(nbytes):
    """The bandwidth reference copy (pp_stream_copy) moves every byte, tails included."""
    import torch
    from paper_1909_05423_amd import _lib
    lib = _lib.load()
    a = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    st = lib.pp_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
