"""GPU parity for periodic z (cyclic z-systems through the Sherman-Morrison
splitting of the Thomas subsection) against the oracle, whose cyclic solve is
pinned to dense LU.  Tolerances as elsewhere: 1e-12 relative max-norm in double
and for the refined float solve, 1e-5 for the unrefined float solve.
"""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

XY = [x * 2 + y * 2 for x in "PND" for y in "PND"]
SHAPES = [(7, 12, 16), (5, 9, 6), (3, 1, 4), (3, 4, 3), (37, 36, 48), (20, 32, 27), (64, 8, 8)]


def _solve(f, bc, h, dtype="f64", gauge="mean", adjoint=False, faces=None):
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import to_dev
    f = np.asarray(f)
    plan = Plan(f.shape, bc, h, dtype=dtype, gauge=gauge)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    fd = to_dev(f.reshape((1,) + f.shape), tdt)
    if adjoint:
        u = plan.adjoint(fd)
    elif faces is not None:
        u = plan.solve(fd, faces=[None if g is None else to_dev(g.reshape(plan.face_shape(i)), tdt)
                                  for i, g in enumerate(faces)])
    else:
        u = plan.solve(fd)
    torch.cuda.synchronize()
    return u.double().cpu().numpy().reshape(f.shape), plan


@pytest.mark.parametrize("xy", XY)
def test_periodic_z_f64(xy):
    from gpu_util import banner, rel_max
    bc = xy + "PP"
    rng = np.random.default_rng(67 + sum(map(ord, bc)))
    for shape in SHAPES:
        banner(f"periodic z f64 {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape)
        u, _ = _solve(f, bc, h)
        assert rel_max(u, oracle.solve(f, bc, h, "mean")) < 1e-12, (bc, shape)


@pytest.mark.parametrize("bc", ["PPPPPP", "DDNNPP", "NNDDPP", "DDDDPP"])
def test_periodic_z_f32_and_refined(bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(71 + sum(map(ord, bc)))
    for shape in [(7, 12, 16), (37, 36, 48)]:
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape)
        banner(f"periodic z refined {bc} {shape}")
        u, plan = _solve(f, bc, h, dtype="f32_refined")
        assert rel_max(u, oracle.solve(f, bc, h, "mean")) < 1e-12, (bc, shape, plan.last_info())
        f32 = f.astype(np.float32).astype(np.float64)
        banner(f"periodic z f32 {bc} {shape}")
        u, _ = _solve(f32, bc, h, dtype="f32")
        assert rel_max(u, oracle.solve(f32, bc, h, "mean")) < 1e-5, (bc, shape)


@pytest.mark.parametrize("bc", ["PPPPPP", "NNNNPP", "PPNNPP"])
@pytest.mark.parametrize("gauge", ["mean", "pin", "pin_raw"])
def test_periodic_z_gauges_and_adjoint(bc, gauge):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(73)
    for shape in [(8, 12, 16), (5, 6, 9)]:
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape) + 0.3
        banner(f"periodic z gauge {gauge} {bc} {shape}")
        u, _ = _solve(f, bc, h, gauge=gauge)
        assert rel_max(u, oracle.solve(f, bc, h, gauge)) < 1e-12
        banner(f"periodic z adjoint {gauge} {bc} {shape}")
        v, _ = _solve(f, bc, h, gauge=gauge, adjoint=True)
        assert rel_max(v, oracle.solve_adjoint(f, bc, h, gauge)) < 1e-12


# the exact-count forms and the long-line form of the z march, on the unit cube
FULL_SHAPES = [(16, 512, 16), (8, 8, 512), (16, 512, 512), (9, 512, 12), (4, 1024, 4), (3, 2048, 2), (12, 384, 8),
               (7, 384, 6), (8, 1024, 4)]


@pytest.mark.parametrize("bc", ["PPPPPP", "DDNNPP", "NNPPPP"])
def test_periodic_z_full_and_long(bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(79 + sum(map(ord, bc)))
    for shape in FULL_SHAPES:
        h = tuple(1.0 / n for n in shape[::-1])
        f = rng.standard_normal(shape)
        uo = oracle.solve(f, bc, h, "mean")
        banner(f"periodic z full f64 {bc} {shape}")
        u, _ = _solve(f, bc, h)
        assert rel_max(u, uo) < 1e-12, ("f64", shape)
        banner(f"periodic z full refined {bc} {shape}")
        u, _ = _solve(f, bc, h, dtype="f32_refined")
        assert rel_max(u, uo) < 1e-12, ("refined", shape)


@pytest.mark.parametrize("bc", ["DDNNPP", "NNDDPP"])
def test_periodic_z_with_faces(bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(83)
    for shape in [(7, 12, 16), (20, 32, 27)]:
        nz, ny, nx = shape
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape)
        dims = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
        faces = [None if bc[i] == "P" else rng.standard_normal(dims[i]) for i in range(6)]
        banner(f"periodic z faces {bc} {shape}")
        u, _ = _solve(f, bc, h, faces=faces)
        assert rel_max(u, oracle.solve(f, bc, h, "mean", faces=faces)) < 1e-12


def test_periodic_z_closed_form_at_full_size():
    """A sum of eigenmodes of the all-periodic operator at 256^3 (no oracle
    needed): u = sum a_m phi_m / Lambda_m exactly, on sampled points."""
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import banner
    n = 256
    h = 1.0 / n
    rng = np.random.default_rng(89)
    c = (np.arange(n) + 0.5) * h
    modes = [(rng.integers(-6, 7), rng.integers(-6, 7), rng.integers(1, 7), rng.standard_normal(),
              rng.uniform(0, 2 * np.pi)) for _ in range(8)]
    lam = lambda k: -4.0 * np.sin(np.pi * k / n) ** 2 / h ** 2

    def field(coef):
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij", sparse=True)
        out = np.zeros((n, n, n))
        for kx, ky, kz, a, ph in modes:
            out += coef(kx, ky, kz) * a * np.cos(2 * np.pi * (kx * X + ky * Y + kz * Z) + ph)
        return out

    f = field(lambda kx, ky, kz: 1.0)
    uo = field(lambda kx, ky, kz: 1.0 / (lam(kx) + lam(ky) + lam(kz)))
    banner("periodic z closed form 256^3")
    plan = Plan((n, n, n), "PPPPPP", (h, h, h))
    u = plan.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.abs(u - uo).max() < 1e-12 * np.abs(uo).max()
