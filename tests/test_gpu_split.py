"""GPU parity of the split Thomas march (section "Solution of the Resulting
Tridiagonal Matrices": each z-system eliminated from both ends toward a
meeting point, the two meeting rows solved, then substitution outward), forced
on through pp_plan_set_zsplit, against the CPU oracle and against the single
march on the same inputs.

Tolerances (relative max-norm against the oracle) as the other parity tests:
1e-12 in double and for the refined float solve, 1e-5 for the float solve;
split and single march agree to the same bounds (they differ only in the
order of rounding).
"""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_refined": 1e-12}


def _solve(f, bc, h, dtype, zsplit, gauge="mean", batch=1, adjoint=False):
    import torch
    from paper_1909_05423_amd import Plan
    from gpu_util import to_dev
    plan = Plan(f.shape[-3:], bc, h, dtype=dtype, batch=batch, gauge=gauge, zsplit=zsplit)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    fd = to_dev(f.reshape((batch,) + f.shape[-3:]), tdt)
    u = plan.adjoint(fd) if adjoint else plan.solve(fd)
    torch.cuda.synchronize()
    return u.double().cpu().numpy().reshape(f.shape), plan


def _input(rng, shape, dtype):
    f = rng.standard_normal(shape)
    return f.astype(np.float32).astype(np.float64) if dtype == "f32" else f


# (nz, ny, nx): whole halves (nz a multiple of 16), ragged halves, the
# shortest split column (two chunks), float lines of 384 (chunks of 6)
SHAPES = [(32, 12, 16), (37, 9, 6), (16, 8, 8), (61, 24, 27), (48, 384, 4)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32_refined"])
@pytest.mark.parametrize("bc", ["DDDDDD", "PPPPDN", "NNDDND", "PPNNDD", "DDPPNN"])
def test_split_vs_oracle_and_single_march(dtype, bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(sum(map(ord, bc + dtype)))
    for shape in SHAPES:
        banner(f"split {dtype} {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = _input(rng, shape, dtype)
        us, _ = _solve(f, bc, h, dtype, "on")
        u1, _ = _solve(f, bc, h, dtype, "off")
        uo = oracle.solve(f, bc, h, "mean")
        assert rel_max(us, uo) < TOL[dtype], (dtype, bc, shape)
        assert rel_max(us, u1) < TOL[dtype], (dtype, bc, shape)


@pytest.mark.parametrize("bc", ["PPPPNN", "NNNNNN", "NNPPNN"])
@pytest.mark.parametrize("gauge", ["mean", "pin", "pin_raw"])
@pytest.mark.parametrize("dtype", ["f64", "f32_refined"])
def test_split_singular_gauges_batch(bc, gauge, dtype):
    """The pinned zero-mode line (u_0 = 0 in the upper half) and the mean of
    the zero-mode solution, which the two halves add up, per batch entry."""
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(5)
    for shape in [(40, 12, 16), (33, 18, 9)]:
        banner(f"split gauge {dtype} {gauge} {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal((3,) + shape) + np.array([0.3, -1.0, 2.0])[:, None, None, None]
        us, plan = _solve(f, bc, h, dtype, "on", gauge=gauge, batch=3)
        _, means, _ = plan.last_info()
        for b in range(3):
            uo = oracle.solve(f[b], bc, h, gauge)
            assert rel_max(us[b], uo) < TOL[dtype], (b, gauge, bc, shape)
            expect = f[b].mean() if gauge != "pin_raw" else 0.0
            assert abs(means[b] - expect) < 1e-13 * max(1.0, abs(f[b]).max())


def test_split_many_columns_and_adjoint():
    """512 slots (more workgroups than compute units) and the adjoint solve."""
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(9)
    shape, bc = (20, 8, 1024), "DDNNDN"
    h = (1.0 / 1024, 1.0 / 8, 1.0 / 20)
    f = rng.standard_normal(shape)
    banner(f"split many columns {shape}")
    us, _ = _solve(f, bc, h, "f64", "on")
    assert rel_max(us, oracle.solve(f, bc, h, "mean")) < 1e-12
    ua, _ = _solve(f, bc, h, "f64", "on", adjoint=True)
    assert rel_max(ua, oracle.solve_adjoint(f, bc, h, "mean")) < 1e-12


# Segmented march (three or more segments per column; plans with few columns):
# (64, 12, 16) four whole segments, (100, 9, 6) seven with a ragged last one,
# (61, 24, 27) four, (48, 384, 4) three in double and four in float (the
# march of lines up to 512), (64, 256, 8) four (the exact-count form of the
# four-wavefront march of lines up to 256).
SEG_SHAPES = [(64, 12, 16), (100, 9, 6), (61, 24, 27), (48, 384, 4), (64, 256, 8)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", ["DDDDDD", "PPPPDN", "NNDDND", "PPNNDD", "DDPPNN"])
def test_segmented_vs_oracle_and_single_march(dtype, bc):
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(3 + sum(map(ord, bc + dtype)))
    for shape in SEG_SHAPES:
        banner(f"segmented {dtype} {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = _input(rng, shape, dtype)
        us, _ = _solve(f, bc, h, dtype, "seg")
        u1, _ = _solve(f, bc, h, dtype, "off")
        uo = oracle.solve(f, bc, h, "mean")
        assert rel_max(us, uo) < TOL[dtype], (dtype, bc, shape)
        assert rel_max(us, u1) < TOL[dtype], (dtype, bc, shape)


@pytest.mark.parametrize("bc", ["PPPPNN", "NNNNNN", "NNPPNN"])
@pytest.mark.parametrize("gauge", ["mean", "pin", "pin_raw"])
def test_segmented_singular_gauges_batch(bc, gauge):
    """The pinned zero-mode line in segment 0 and the zero-mode mean the
    segments add up, per batch entry."""
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(15)
    for shape in [(64, 12, 16), (70, 18, 9)]:
        banner(f"segmented gauge {gauge} {bc} {shape}")
        h = tuple(rng.uniform(0.5, 2.0, 3))
        f = rng.standard_normal((3,) + shape) + np.array([0.3, -1.0, 2.0])[:, None, None, None]
        us, plan = _solve(f, bc, h, "f64", "seg", gauge=gauge, batch=3)
        _, means, _ = plan.last_info()
        for b in range(3):
            uo = oracle.solve(f[b], bc, h, gauge)
            assert rel_max(us[b], uo) < 1e-12, (b, gauge, bc, shape)
            expect = f[b].mean() if gauge != "pin_raw" else 0.0
            assert abs(means[b] - expect) < 1e-13 * max(1.0, abs(f[b]).max())


def test_segmented_long_columns_and_adjoint():
    """The paper's solver-comparison shape family (few columns, long z), with
    Dirichlet x: no z-system close to singular."""
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(21)
    for shape in [(1023, 16, 16), (255, 64, 8)]:
        bc = "DDPPNN"
        h = (1.0 / 64, 1.0 / 64, 1.0 / 64)
        f = rng.standard_normal(shape)
        banner(f"segmented long {shape}")
        us, _ = _solve(f, bc, h, "f64", "seg")
        assert rel_max(us, oracle.solve(f, bc, h, "mean")) < 1e-12
        ua, _ = _solve(f, bc, h, "f64", "seg", adjoint=True)
        assert rel_max(ua, oracle.solve_adjoint(f, bc, h, "mean")) < 1e-12


def test_auto_keeps_near_singular_columns_whole():
    """Long columns under periodic x, y and Neumann z: splitting the zero
    mode's system would amplify rounding by about nz / 2, so the automatic
    layout keeps one march per column in double and meets the 1e-12 bar; the
    forced splits stay within the bound the header states (amplification
    times the unit roundoff).  Float plans keep the two-way split."""
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(23)
    shape, bc = (1023, 16, 16), "PPPPNN"
    h = (1.0 / 64, 1.0 / 64, 1.0 / 64)
    f = rng.standard_normal(shape)
    uo = oracle.solve(f, bc, h, "mean")
    banner(f"auto near-singular {shape}")
    u, _ = _solve(f, bc, h, "f64", "auto")
    assert rel_max(u, uo) < 1e-12
    for zs in ("on", "seg"):
        us, _ = _solve(f, bc, h, "f64", zs)
        assert rel_max(us, uo) < 512 * 2.2e-16 * 64, zs
    # float: the two-way split stays (float rounding dominates its meeting
    # rows), the segments go; same kernels as the forced split, so the same bits
    f32 = f.astype(np.float32).astype(np.float64)
    u32, _ = _solve(f32, bc, h, "f32", "auto")
    u32_on, _ = _solve(f32, bc, h, "f32", "on")
    assert np.array_equal(u32, u32_on)
    assert rel_max(u32, oracle.solve(f32, bc, h, "mean")) < 1e-5



def test_auto_segments_where_columns_alone_would_not_split():
    """Double lines up to 256 with 129-256 columns: the automatic layout takes
    the plan's segments (same kernels as the forced segmented march, so the
    same bits) and meets the 1e-12 bar."""
    from gpu_util import banner, rel_max
    rng = np.random.default_rng(27)
    shape, bc = (64, 16, 384), "DDNNNN"
    h = (1.0 / 384, 1.0 / 16, 1.0 / 64)
    f = rng.standard_normal(shape)
    banner(f"auto segments {shape}")
    u, _ = _solve(f, bc, h, "f64", "auto")
    us, _ = _solve(f, bc, h, "f64", "seg")
    assert np.array_equal(u, us)
    assert rel_max(u, oracle.solve(f, bc, h, "mean")) < 1e-12
