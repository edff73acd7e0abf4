"""pp_solve_noalloc (the solve that allocates nothing: the library's fixed
per-device workspace) against pp_solve, through the C ABI: two calls in a
row, the second with a smaller grid; every dtype."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [("f64", 0), ("f32", 1), ("f32_refined", 2)]


def _plan(lib, shape, bc, h, code):
    nz, ny, nx = shape
    p = ctypes.c_void_p()
    assert lib.pp_plan_create(nx, ny, nz, bc.encode(), (ctypes.c_double * 3)(*h), code, 1, ctypes.byref(p)) == 0
    return p


@pytest.mark.parametrize("dtype,code", CASES)
def test_noalloc_matches_pp_solve(dtype, code):
    import torch
    from paper_1909_05423_amd import _lib
    from gpu_util import banner, to_dev
    lib = _lib.load()
    tdt = torch.float32 if dtype == "f32" else torch.float64
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(101 + code)
    # second call: a smaller grid, other faces (the fixed buffer then holds the
    # first plan's larger contents and tables)
    for shape, bc in [((64, 96, 128), "PPPPNN"), ((9, 12, 18), "DDNNDN")]:
        banner(f"noalloc {dtype} {shape} {bc}")
        h = tuple(1.0 / n for n in shape[::-1])
        p = _plan(lib, shape, bc, h, code)
        try:
            assert lib.pp_plan_workspace_bytes(p) <= _lib.NOALLOC_SCRATCH_BYTES
            f = to_dev(rng.standard_normal(shape), tdt)
            ws = torch.empty(lib.pp_plan_workspace_bytes(p), dtype=torch.uint8, device="cuda")
            u_ref = torch.full_like(f, float("nan"))
            u_na = torch.full_like(f, float("nan"))
            assert lib.pp_solve(p, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u_ref.data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), stream) == 0
            assert lib.pp_solve_noalloc(p, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u_na.data_ptr()), stream) == 0
            torch.cuda.synchronize()
            a, b = u_na.cpu().numpy(), u_ref.cpu().numpy()
            assert np.all(np.isfinite(a))
            # same kernels, same inputs: the same bits
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), dtype
        finally:
            lib.pp_plan_destroy(p)
