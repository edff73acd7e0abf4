"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/ppsolve.h declares, and validates plans and arguments
before touching the GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppsolve.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1909_05423_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1909_05423_amd import build
        build.build()
    return _lib.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    from paper_1909_05423_amd import _lib
    names = _declared()
    assert set(names) == set(_lib.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n


def _create(lib, nx, ny, nz, bc, h=(1.0, 1.0, 1.0), dtype=0, batch=1):
    hh = (ctypes.c_double * 3)(*h)
    p = ctypes.c_void_p()
    st = lib.pp_plan_create(nx, ny, nz, bc.encode(), hh, dtype, batch, ctypes.byref(p))
    return st, p


@pytest.mark.parametrize("args,status", [
    ((8, 8, 8, "PPPPDD"), 0),
    ((384, 384, 16, "DDDDDD"), 0),
    ((1, 1, 1, "NNNNNN"), 0),
    ((6, 9, 5, "NNPPDN"), 0),
    ((8, 8, 8, "PDPPDD"), -2),     # mixed x faces
    ((8, 8, 8, "PPNDDD"), -2),     # mixed y faces
    ((8, 8, 8, "PPPPPP"), 0),      # periodic z (Sherman-Morrison)
    ((8, 8, 3, "DDNNPP"), 0),
    ((8, 8, 2, "PPPPPP"), -3),     # periodic z needs nz >= 3
    ((8, 8, 8, "PPPPPD"), -2),     # one periodic z face
    ((8, 8, 8, "PPPPXD"), -2),     # unknown face type
    ((10, 8, 8, "PPPPDD"), -3),    # prime factor 5
    ((8, 14, 8, "PPPPDD"), -3),    # prime factor 7
    ((4096, 8, 8, "PPPPDD"), -3),  # beyond the on-chip line limit
    ((0, 8, 8, "PPPPDD"), -1),
    ((8, 8, -1, "PPPPDD"), -1),
])
def test_plan_validation(lib, args, status):
    st, p = _create(lib, *args)
    assert st == status
    if st == 0:
        assert lib.pp_plan_workspace_bytes(p) > 0
        lib.pp_plan_destroy(p)


def test_plan_validation_spacing_batch_dtype(lib):
    assert _create(lib, 8, 8, 8, "PPPPDD", h=(1.0, 0.0, 1.0))[0] == -1
    assert _create(lib, 8, 8, 8, "PPPPDD", h=(1.0, float("nan"), 1.0))[0] == -1
    assert _create(lib, 8, 8, 8, "PPPPDD", batch=0)[0] == -1
    assert _create(lib, 8, 8, 8, "PPPPDD", dtype=7)[0] == -1


def test_workspace_sizes(lib):
    st, p64 = _create(lib, 512, 512, 512, "PPPPNN", dtype=0)
    assert st == 0
    st, p32 = _create(lib, 512, 512, 512, "PPPPNN", dtype=1)
    assert st == 0
    st, pir = _create(lib, 512, 512, 512, "PPPPNN", dtype=2)
    assert st == 0
    w64, w32, wir = (lib.pp_plan_workspace_bytes(p) for p in (p64, p32, pir))
    spectral64 = 256 * 512 * 512 * 16      # ceil(nx/2) complex columns per row
    assert spectral64 <= w64 < spectral64 * 1.2
    assert w32 < w64
    assert wir >= w32 + 512 ** 3 * 4       # the float residual buffer
    for p in (p64, p32, pir):
        lib.pp_plan_destroy(p)


def test_argument_errors_before_any_gpu_call(lib):
    st, p = _create(lib, 8, 8, 8, "PPPPDD")
    assert st == 0
    f = ctypes.c_void_p(0x100000)
    u = ctypes.c_void_p(0x200000)
    assert lib.pp_solve(p, f, u, None, None) == -5                     # no workspace
    assert lib.pp_solve(p, f, u, ctypes.c_void_p(0x300001), None) == -5  # misaligned
    assert lib.pp_solve(p, f, f, ctypes.c_void_p(0x400000), None) == -4  # u aliases f
    assert lib.pp_solve(p, f, ctypes.c_void_p(0x100000 + 8 * 100), ctypes.c_void_p(0x400000), None) == -4
    assert lib.pp_solve(p, None, u, ctypes.c_void_p(0x400000), None) == -1
    assert lib.pp_solve_adjoint(p, f, f, ctypes.c_void_p(0x400000), None) == -4
    assert lib.pp_plan_set_gauge(p, 5) == -1
    assert lib.pp_plan_set_refinement(p, -1.0, 3) == -1
    assert lib.pp_plan_set_refinement(p, 1e-12, -1) == -1
    it = ctypes.c_int(-1)
    assert lib.pp_plan_last_info(p, ctypes.byref(it), None, None) == 0
    assert it.value == 0
    lib.pp_plan_destroy(p)
    for code in range(-8, 1):
        assert lib.pp_status_string(code)


def test_face_argument_errors_before_any_gpu_call(lib):
    st, p = _create(lib, 8, 8, 8, "PPNNDN")
    assert st == 0
    f = ctypes.c_void_p(0x100000)
    u = ctypes.c_void_p(0x200000)
    ws = ctypes.c_void_p(0x400000)
    faces = (ctypes.c_void_p * 6)()
    faces[0] = 0x500000                                                      # a value on a periodic face
    assert lib.pp_solve_bc(p, f, faces, u, ws, None) == -1
    faces[0] = None
    faces[2] = 0x500004                                                      # misaligned
    assert lib.pp_solve_bc(p, f, faces, u, ws, None) == -1
    faces[2] = 0x200000 + 8 * 64                                             # inside u
    assert lib.pp_solve_bc(p, f, faces, u, ws, None) == -4
    faces[2] = 0x400000 + 256                                                # inside the workspace
    assert lib.pp_solve_bc(p, f, faces, u, ws, None) == -4
    lib.pp_plan_destroy(p)


def test_zsolver_option(lib):
    st, p = _create(lib, 8, 8, 8, "PPPPDD")
    assert st == 0
    assert lib.pp_plan_set_zsolver(p, 1) == 0
    assert lib.pp_plan_set_zsolver(p, 2) == 0
    assert lib.pp_plan_set_zsolver(p, 0) == 0
    assert lib.pp_plan_set_zsolver(p, 3) == -1
    assert lib.pp_plan_set_zsolver(p, -1) == -1
    lib.pp_plan_destroy(p)
    for solver in (1, 2):                                       # PCR, CR-P
        st, p = _create(lib, 8, 8, 8, "PPPPPP")
        assert st == 0 and lib.pp_plan_set_zsolver(p, solver) == -2     # periodic z: Thomas only
        lib.pp_plan_destroy(p)
        st, p = _create(lib, 8, 8, 4096, "PPPPDD")
        assert st == 0 and lib.pp_plan_set_zsolver(p, solver) == 0      # z lines up to 4096
        lib.pp_plan_destroy(p)
        st, p = _create(lib, 8, 8, 4097, "PPPPDD")
        assert st == 0 and lib.pp_plan_set_zsolver(p, solver) == -3     # z lines longer than 4096
        lib.pp_plan_destroy(p)
        st, p = _create(lib, 8, 1024, 8, "PPPPDD")
        assert st == 0 and lib.pp_plan_set_zsolver(p, solver) == -3     # y lines longer than 512
        lib.pp_plan_destroy(p)



def test_zsplit_option(lib):
    st, p = _create(lib, 8, 8, 16, "PPPPDD")
    assert st == 0
    for mode in (0, 1, 2, 0):
        assert lib.pp_plan_set_zsplit(p, mode) == 0
    assert lib.pp_plan_set_zsplit(p, 3) == -3     # 16 planes: no room for three segments
    assert lib.pp_plan_set_zsplit(p, 4) == -1
    assert lib.pp_plan_set_zsplit(p, -1) == -1
    lib.pp_plan_destroy(p)
    for nx, ny, nz, bc, want in [(8, 8, 16, "PPPPPP", -2),     # periodic z: one march
                                 (8, 8, 15, "PPPPDD", -3),     # fewer than two chunks of 8 planes
                                 (8, 2048, 32, "PPPPDD", -3),  # y lines over 1024: the general march
                                 (8, 384, 12, "PPPPDD", -3)]:  # double lines of 384: chunks of 8
        st, p = _create(lib, nx, ny, nz, bc)
        assert st == 0 and lib.pp_plan_set_zsplit(p, 2) == want, (nx, ny, nz, bc)
        assert lib.pp_plan_set_zsplit(p, 3) == want, (nx, ny, nz, bc)
        assert lib.pp_plan_set_zsplit(p, 1) == 0 and lib.pp_plan_set_zsplit(p, 0) == 0
        lib.pp_plan_destroy(p)
    # segments: few columns and z long enough for three of at least two
    # chunks; y lines up to 256 aim at 1024 workgroups, longer ones at 256
    for nx, ny, nz, dtype, want in [(16, 8, 48, 0, 0), (16, 8, 33, 0, 0), (16, 8, 32, 0, -3), (16, 8, 48, 2, -3),
                                    (512, 8, 4096, 0, 0), (1024, 8, 4096, 0, -3),
                                    (256, 256, 64, 0, 0), (256, 512, 64, 0, -3)]:
        st, p = _create(lib, nx, ny, nz, "PPPPDD", dtype=dtype)
        assert st == 0 and lib.pp_plan_set_zsplit(p, 3) == want, (nx, ny, nz, dtype)
        lib.pp_plan_destroy(p)


def test_noalloc_rejects_before_touching_the_gpu(lib):
    """pp_solve_noalloc: argument errors and the fixed-buffer limit are host checks."""
    from paper_1909_05423_amd import _lib
    st, p = _create(lib, 256, 256, 256, "PPPPNN", h=(1 / 256,) * 3, dtype=0)
    assert st == 0
    try:
        assert lib.pp_plan_workspace_bytes(p) > _lib.NOALLOC_SCRATCH_BYTES
        dummy = ctypes.c_void_p(256)
        assert lib.pp_solve_noalloc(p, dummy, ctypes.c_void_p(512), None) == -9
        assert lib.pp_solve_noalloc(p, None, dummy, None) == -1
        assert lib.pp_solve_noalloc(None, dummy, dummy, None) == -1
    finally:
        lib.pp_plan_destroy(p)
    assert b"no-alloc" in lib.pp_status_string(-9)


def test_noalloc_limit_matches_header():
    from paper_1909_05423_amd import _lib
    text = open(HEADER).read()
    m = re.search(r"#define PP_NOALLOC_SCRATCH_BYTES \((\d+)u \* 1024u \* 1024u\)", text)
    assert m and int(m.group(1)) * 1024 * 1024 == _lib.NOALLOC_SCRATCH_BYTES


def test_stream_copy_argument_errors(lib):
    """pp_stream_copy checks its arguments on the host (no GPU call for these)."""
    a, b = ctypes.c_void_p(4096), ctypes.c_void_p(1 << 20)
    assert lib.pp_stream_copy(None, b, 16, None) == -1
    assert lib.pp_stream_copy(a, None, 16, None) == -1
    assert lib.pp_stream_copy(a, b, 24, None) == -1                     # not a multiple of 16
    assert lib.pp_stream_copy(ctypes.c_void_p(4104), b, 16, None) == -1  # misaligned source
    assert lib.pp_stream_copy(a, ctypes.c_void_p(4096 + 16), 64, None) == -4   # overlap
    assert lib.pp_stream_copy(a, b, 0, None) == 0
