"""GPU parity for non-homogeneous face values (pp_solve_bc) against the oracle,
plus two checks that need no oracle: multilinear harmonic fields reproduced to
rounding, and second-order convergence with boundary data at larger sizes.

Tolerances as for the homogeneous solves: 1e-12 relative max-norm in double
and for the refined float solve, 1e-5 for the unrefined float solve.
"""

import numpy as np
import pytest

import oracle
from oracle import solver
from oracle.operator import boundary_lift

pytestmark = pytest.mark.gpu

FACE_BCS = [x * 2 + y * 2 + z for x in "PND" for y in "PND" for z in ("DD", "NN", "DN", "ND")]
SHAPES = [(7, 12, 16), (5, 9, 6), (3, 1, 4), (1, 4, 3), (20, 32, 27)]


def _face_dims(shape):
    nz, ny, nx = shape
    return [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2


def _random_faces(bc, shape, rng, batch=None, scale=1.0):
    lead = () if batch is None else (batch,)
    return [None if bc[i] == "P" else scale * rng.standard_normal(lead + d) for i, d in enumerate(_face_dims(shape))]


def _solve(f, bc, h, faces, dtype="f64", gauge="mean", batch=None):
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import to_dev
    f = np.asarray(f)
    if batch is None:
        batch = 1 if f.ndim == 3 else f.shape[0]
    shape = f.shape[-3:]
    plan = Plan(shape, bc, h, dtype=dtype, batch=batch, gauge=gauge)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    fd = to_dev(f.reshape((batch,) + shape), tdt)
    gd = [None if g is None else to_dev(np.asarray(g).reshape(plan.face_shape(i)), tdt) for i, g in enumerate(faces)]
    u = plan.solve(fd, faces=gd)
    torch.cuda.synchronize()
    return u.double().cpu().numpy().reshape(f.shape), plan


@pytest.mark.parametrize("bc", FACE_BCS)
def test_faces_f64_all_bcs(bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(41 + sum(map(ord, bc)))
    for shape in SHAPES:
        banner(f"faces f64 {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape)
        faces = _random_faces(bc, shape, rng)
        u, _ = _solve(f, bc, h, faces)
        uo = oracle.solve(f, bc, h, "mean", faces=faces)
        assert rel_max(u, uo) < 1e-12, (bc, shape)


@pytest.mark.parametrize("bc", ["DDNNDN", "NNDDND", "PPDDNN", "NNNNNN", "PPPPDD", "NNPPNN"])
def test_faces_refined_and_f32(bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(43 + sum(map(ord, bc)))
    for shape in [(8, 12, 16), (20, 32, 27)]:
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape)
        faces = _random_faces(bc, shape, rng)
        uo = oracle.solve(f, bc, h, "mean", faces=faces)
        banner(f"faces refined {bc} {shape}")
        u, plan = _solve(f, bc, h, faces, dtype="f32_refined")
        assert rel_max(u, uo) < 1e-12, (bc, shape, plan.last_info())
        f32 = f.astype(np.float32).astype(np.float64)
        g32 = [None if g is None else g.astype(np.float32).astype(np.float64) for g in faces]
        banner(f"faces f32 {bc} {shape}")
        u, _ = _solve(f32, bc, h, g32, dtype="f32")
        assert rel_max(u, oracle.solve(f32, bc, h, "mean", faces=g32)) < 1e-5, (bc, shape)


@pytest.mark.parametrize("bc", ["NNNNNN", "PPNNNN", "NNPPNN"])
@pytest.mark.parametrize("gauge", ["mean", "pin", "pin_raw"])
def test_faces_singular_gauges(bc, gauge):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(47)
    for shape in [(8, 12, 16), (5, 6, 9)]:
        banner(f"faces gauge {gauge} {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape) + 0.2
        faces = _random_faces(bc, shape, rng)
        u, plan = _solve(f, bc, h, faces, gauge=gauge)
        uo = oracle.solve(f, bc, h, gauge, faces=faces)
        assert rel_max(u, uo) < 1e-12
        _, means, _ = plan.last_info()
        lifted = f - boundary_lift(shape, bc, h, faces)
        expect = lifted.mean() if gauge != "pin_raw" else 0.0
        assert abs(means[0] - expect) < 1e-12 * max(1.0, np.abs(lifted).max())


def test_faces_batched():
    from gpu_util import rel_max
    rng = np.random.default_rng(53)
    for bc in ["DDNNDN", "PPPPNN"]:
        shape = (9, 12, 16)
        f = rng.standard_normal((3,) + shape)
        faces = _random_faces(bc, shape, rng, batch=3)
        h = (0.7, 1.1, 0.9)
        u, _ = _solve(f, bc, h, faces, batch=3)
        for b in range(3):
            fb = [None if g is None else g[b] for g in faces]
            assert rel_max(u[b], oracle.solve(f[b], bc, h, "mean", faces=fb)) < 1e-12


# exact-count kernel forms (x lines of 512 and 1024, y lines of 512) with faces,
# on the unit-cube spacing (see the note on long lines in test_gpu_parity.py)
FULL_SHAPES = [(8, 8, 512), (16, 512, 16), (8, 16, 1024), (16, 512, 512)]


@pytest.mark.parametrize("bc", ["DDNNDN", "PPPPNN", "NNDDDD"])
def test_faces_full_shapes(bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(59 + sum(map(ord, bc)))
    for shape in FULL_SHAPES:
        h = tuple(1.0 / n for n in shape[::-1])
        f = rng.standard_normal(shape)
        faces = _random_faces(bc, shape, rng)
        uo = oracle.solve(f, bc, h, "mean", faces=faces)
        banner(f"faces full f64 {bc} {shape}")
        u, _ = _solve(f, bc, h, faces)
        assert rel_max(u, uo) < 1e-12, ("f64", shape)
        banner(f"faces full refined {bc} {shape}")
        u, _ = _solve(f, bc, h, faces, dtype="f32_refined")
        assert rel_max(u, uo) < 1e-12, ("refined", shape)


def _multilinear(bc, rng):
    c = rng.standard_normal(8)
    vary = [bc[2 * d] != "P" for d in range(3)]
    terms = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1)]
    coef = [ci if all(vary[d] or not e[d] for d in range(3)) else 0.0 for ci, e in zip(c, terms)]
    return coef, terms


@pytest.mark.parametrize("bc", ["DDNNDN", "NNDDND", "DDDDDD", "NNNNNN", "PPDDNN"])
def test_faces_multilinear_exact_at_64(bc):
    """A multilinear field with consistent face data solves exactly (no oracle)."""
    from gpu_util import banner
    rng = np.random.default_rng(61)
    n = 64
    shape, h = (n, n, n), (1.0 / n,) * 3
    coef, terms = _multilinear(bc, rng)
    c = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")

    def u(x, y, z):
        return sum(ci * x ** e[0] * y ** e[1] * z ** e[2] for ci, e in zip(coef, terms)) + 0.0 * x

    def du(d, x, y, z):
        out = 0.0 * x
        for ci, e in zip(coef, terms):
            if e[d]:
                p = [x, y, z]
                term = ci
                for k in range(3):
                    if k != d:
                        term = term * p[k] ** e[k]
                out = out + term
        return out

    faces = []
    for i in range(6):
        d, side = i // 2, i % 2
        if bc[i] == "P":
            faces.append(None)
            continue
        pos = 0.0 if side == 0 else 1.0
        a, b = np.meshgrid(c, c, indexing="ij")
        pt = [(pos + 0 * a, b, a), (b, pos + 0 * a, a), (b, a, pos + 0 * a)][d]   # (x, y, z) on the face
        if bc[i] == "D":
            faces.append(u(*pt))
        else:
            faces.append((1.0 if side else -1.0) * du(d, *pt))
    banner(f"faces multilinear {bc} 64^3")
    uh, _ = _solve(np.zeros(shape), bc, h, faces)
    ustar = u(X, Y, Z)
    if solver.is_singular(bc):
        uh, ustar = uh - uh.mean(), ustar - ustar.mean()
    assert np.abs(uh - ustar).max() < 1e-11 * max(1.0, np.abs(ustar).max())


@pytest.mark.parametrize("bc", ["DDNNDN", "PPDDNN"])
def test_faces_second_order_up_to_256(bc):
    """Smooth solution with non-zero face values and fluxes on the unit cube:
    RMS error against the continuous solution drops 4x per halving of h up to
    256^3 (GPU only; the oracle pins the same convergence at 16-64)."""
    from gpu_util import banner
    kx = 2 * np.pi if bc[0] == "P" else 1.3
    ky = 2 * np.pi if bc[2] == "P" else 0.9
    kz = 0.7

    def u(x, y, z):
        return np.cos(kx * x + 0.4) * np.sin(ky * y + 0.3) * np.cosh(kz * z) + 0.5

    def grad(x, y, z):
        return (-kx * np.sin(kx * x + 0.4) * np.sin(ky * y + 0.3) * np.cosh(kz * z),
                ky * np.cos(kx * x + 0.4) * np.cos(ky * y + 0.3) * np.cosh(kz * z),
                kz * np.cos(kx * x + 0.4) * np.sin(ky * y + 0.3) * np.sinh(kz * z))

    errs = []
    for n in (64, 128, 256):
        c = (np.arange(n) + 0.5) / n
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        f = (kz * kz - kx * kx - ky * ky) * (u(X, Y, Z) - 0.5)
        a, b = np.meshgrid(c, c, indexing="ij")
        faces = []
        for i in range(6):
            d, side = i // 2, i % 2
            if bc[i] == "P":
                faces.append(None)
                continue
            pos = 0.0 if side == 0 else 1.0
            pt = [(pos + 0 * a, b, a), (b, pos + 0 * a, a), (b, a, pos + 0 * a)][d]
            faces.append(u(*pt) if bc[i] == "D" else (1.0 if side else -1.0) * grad(*pt)[d])
        banner(f"faces convergence {bc} {n}^3")
        uh, _ = _solve(f, bc, (1.0 / n,) * 3, faces)
        ustar = u(X, Y, Z)
        if solver.is_singular(bc):
            uh, ustar = uh - uh.mean(), ustar - ustar.mean()
        errs.append(np.sqrt(np.mean((uh - ustar) ** 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.05), (errs, orders)
