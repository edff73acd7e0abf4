"""GPU parity of the alternative z solvers (parallel cyclic reduction, and
cyclic reduction with a parallel backward phase; y transforms as separate
passes) against the oracle, whose z solve is the general Thomas algorithm
pinned to dense LU; and at full size against the backward-error bar.
Tolerances as for the default solver.
"""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BCS = [x * 2 + y * 2 + z for x in "PND" for y in "PND" for z in ("DD", "NN", "DN", "ND")]
SHAPES = [(7, 12, 16), (5, 9, 6), (3, 1, 4), (1, 4, 3), (2, 3, 1), (37, 36, 48), (20, 32, 27), (64, 8, 8),
          (6, 8, 8), (33, 8, 8)]
SOLVERS = ["pcr", "cr"]


def _solve(f, bc, h, dtype="f64", gauge="mean", adjoint=False, zsolver="pcr"):
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import to_dev
    f = np.asarray(f)
    plan = Plan(f.shape, bc, h, dtype=dtype, gauge=gauge, zsolver=zsolver)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    fd = to_dev(f.reshape((1,) + f.shape), tdt)
    u = plan.adjoint(fd) if adjoint else plan.solve(fd)
    torch.cuda.synchronize()
    return u.double().cpu().numpy().reshape(f.shape), plan


@pytest.mark.parametrize("zsolver", SOLVERS)
@pytest.mark.parametrize("bc", BCS)
def test_pcr_f64_all_bcs(bc, zsolver):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(97 + sum(map(ord, bc)))
    for shape in SHAPES:
        banner(f"{zsolver} f64 {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape)
        u, _ = _solve(f, bc, h, zsolver=zsolver)
        assert rel_max(u, oracle.solve(f, bc, h, "mean")) < 1e-12, (bc, shape)


@pytest.mark.parametrize("zsolver", SOLVERS)
@pytest.mark.parametrize("bc", ["PPPPNN", "DDNNDN", "NNDDND", "PPPPDD"])
def test_pcr_f32_refined_gauges_adjoint(bc, zsolver):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(101 + sum(map(ord, bc)))
    for shape in [(8, 12, 16), (37, 36, 48)]:
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal(shape) + 0.2
        banner(f"{zsolver} refined {bc} {shape}")
        u, _ = _solve(f, bc, h, dtype="f32_refined", zsolver=zsolver)
        assert rel_max(u, oracle.solve(f, bc, h, "mean")) < 1e-12
        f32 = f.astype(np.float32).astype(np.float64)
        banner(f"{zsolver} f32 {bc} {shape}")
        u, _ = _solve(f32, bc, h, dtype="f32", zsolver=zsolver)
        assert rel_max(u, oracle.solve(f32, bc, h, "mean")) < 1e-5
        for gauge in ["pin", "pin_raw"]:
            banner(f"{zsolver} {gauge} {bc} {shape}")
            u, _ = _solve(f, bc, h, gauge=gauge, zsolver=zsolver)
            assert rel_max(u, oracle.solve(f, bc, h, gauge)) < 1e-12
        banner(f"{zsolver} adjoint {bc} {shape}")
        v, _ = _solve(f, bc, h, adjoint=True, zsolver=zsolver)
        assert rel_max(v, oracle.solve_adjoint(f, bc, h, "mean")) < 1e-12


@pytest.mark.parametrize("zsolver", SOLVERS)
def test_pcr_full_size_backward_error_and_agreement(zsolver):
    """512^3 divergence workload: the PCR / CR-P solve meets the backward-error
    bar and agrees with the default (Thomas) solve."""
    import torch
    import workloads
    from paper_1909_05423_amd import Plan
    from gpu_util import banner
    wl = workloads.make("div_ppn")
    f = torch.from_numpy(wl["f"]).cuda()
    banner(f"{zsolver} 512^3 div_ppn")
    up = Plan(wl["shape"], wl["bc"], wl["h"], zsolver=zsolver).solve(f)
    ut = Plan(wl["shape"], wl["bc"], wl["h"]).solve(f)
    torch.cuda.synchronize()
    diff = float((up - ut).abs().max() / ut.abs().max())
    assert diff < 1e-12, diff
    u = up.cpu().numpy()[0]
    fh = wl["f"][0] - wl["f"][0].mean()
    eta = oracle.backward_error(fh, u, wl["bc"], wl["h"])
    assert eta < 1e-14, eta


@pytest.mark.parametrize("zsolver", SOLVERS)
def test_pcr_with_faces_and_batch(zsolver):
    """Face values and a batch of two through the alternative z solvers."""
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import banner, rel_max, to_dev
    rng = np.random.default_rng(103)
    for bc in ["DDNNDN", "PPPPNN"]:
        shape = (20, 32, 27)
        nz, ny, nx = shape
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal((2,) + shape)
        dims = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
        faces = [None if bc[i] == "P" else rng.standard_normal((2,) + dims[i]) for i in range(6)]
        banner(f"{zsolver} faces batch 2 {bc} {shape}")
        plan = Plan(shape, bc, h, batch=2, zsolver=zsolver)
        u = plan.solve(to_dev(f, torch.float64),
                       faces=[None if g is None else to_dev(g, torch.float64) for g in faces])
        torch.cuda.synchronize()
        u = u.cpu().numpy()
        for b in range(2):
            fb = [None if g is None else g[b] for g in faces]
            assert rel_max(u[b], oracle.solve(f[b], bc, h, "mean", faces=fb)) < 1e-12, (bc, b)


# The paper's comparison of the tridiagonal solvers runs 64 x 64 x nz grids
# with nz = 2^n - 1 (the sizes CR-P is stated for) up to 4095 (section
# "Comparison of Tridiagonal Solvers"); lines this long hold one real system
# per workgroup tile.  Every solver against the oracle element by element.
# Spacing h = 1/64 in every direction with a Dirichlet x direction: the
# operator's condition number stays near 5e3 (on the unit cube, hz = 1/nz
# makes it ~0.4 nz^2 = 7e6 at nz = 4095, where both the oracle's and any
# double-precision solve's rounding errors reach 1e-11).
@pytest.mark.parametrize("nz", [255, 511, 1023, 2047, 4095, 4096, 1000])
@pytest.mark.parametrize("bc", ["DDDDDD", "DDNNNN", "DDPPND"])
def test_paper_solver_sweep_shapes(nz, bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(nz + sum(map(ord, bc)))
    shape = (nz, 64, 64)
    h = (1 / 64, 1 / 64, 1 / 64)
    f = rng.standard_normal(shape)
    uo = oracle.solve(f, bc, h, "mean")
    for zsolver in ["thomas", "pcr", "cr"]:
        banner(f"sweep {zsolver} {bc} {shape}")
        u, _ = _solve(f, bc, h, zsolver=zsolver)
        err = rel_max(u, uo)
        assert err < 1e-12, (zsolver, err)
