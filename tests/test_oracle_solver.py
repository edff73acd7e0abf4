"""Pins of the oracle solve and adjoint.

* brute force: dense LU of the assembled 7-point matrix (bordered when singular)
  on every supported boundary combination, sizes 1..8, all gauges;
* the literal adjoint against the transpose of the dense solution operator;
* closed-form discrete solutions for eigenmode sources;
* the paper's printed manufactured-solution errors (Tables tb3-tb7) and the
  second-order convergence they show;
* planted mistakes in the oracle are caught by these pins.
"""

import itertools
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import closed_form, solver
from oracle.dense import dense_operator, dense_solve
from oracle.operator import apply_laplacian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mms_tables.txt")

BCS = [x + x + y + y + z for x in "PND" for y in "PND" for z in ("DD", "NN", "DN", "ND", "PP")]
GAUGES = ["mean", "pin", "pin_raw"]


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("bc", BCS)
def test_against_dense_lu(bc):
    rng = np.random.default_rng(abs(hash(bc)) % 2**32)
    shapes = [(1, 1, 1), (2, 3, 1), (3, 1, 4), (4, 4, 3), (5, 6, 7), (8, 2, 8), (3, 8, 6)]
    for shape in shapes:
        h = tuple(rng.uniform(0.3, 2.0, 3))
        f = rng.standard_normal(shape)
        for gauge in GAUGES if solver.is_singular(bc) else ["mean"]:
            u = oracle.solve(f, bc, h, gauge)
            ud = dense_solve(f, bc, h, gauge)
            assert _rel(u, ud) < 1e-12, (bc, shape, gauge)


@pytest.mark.parametrize("bc", ["PPPPDD", "DDNNNN", "PPPPNN", "NNNNNN", "DDDDDD", "NNPPND", "PPPPPP"])
@pytest.mark.parametrize("gauge", GAUGES)
def test_adjoint_against_dense_transpose(bc, gauge):
    rng = np.random.default_rng(7)
    for shape in [(3, 4, 5), (2, 2, 6), (4, 3, 2)]:
        h = tuple(rng.uniform(0.5, 2.0, 3))
        G = dense_operator(shape, bc, h, gauge)
        g = rng.standard_normal(shape)
        v = oracle.solve_adjoint(g, bc, h, gauge)
        assert _rel(v.reshape(-1), G.T @ g.reshape(-1)) < 1e-12
        # the forward solve is the dense operator too
        f = rng.standard_normal(shape)
        assert _rel(oracle.solve(f, bc, h, gauge).reshape(-1), G @ f.reshape(-1)) < 1e-12


def test_mean_gauge_symmetric_pin_gauge_not():
    bc, h, shape = "PPPPNN", (1.0, 1.0, 1.0), (4, 3, 4)
    Gm = dense_operator(shape, bc, h, "mean")
    Gp = dense_operator(shape, bc, h, "pin")
    np.testing.assert_allclose(Gm, Gm.T, atol=1e-12)
    assert np.max(np.abs(Gp - Gp.T)) > 1e-3


def test_batched_solve_equals_loop():
    rng = np.random.default_rng(8)
    f = rng.standard_normal((3, 4, 5, 6))
    for bc in ["PPPPNN", "DDNNDD"]:
        ub = oracle.solve(f, bc, (1, 1, 1))
        for b in range(3):
            np.testing.assert_allclose(ub[b], oracle.solve(f[b], bc, (1, 1, 1)), atol=1e-13)


@given(bcx=st.sampled_from("PND"), bcy=st.sampled_from("PND"), bcz=st.sampled_from(["DD", "NN", "DN", "PP"]),
       nx=st.integers(1, 7), ny=st.integers(1, 7), nz=st.integers(1, 7),
       hx=st.floats(0.2, 3.0), hy=st.floats(0.2, 3.0), hz=st.floats(0.2, 3.0),
       seed=st.integers(0, 2**31), gauge=st.sampled_from(GAUGES))
@settings(max_examples=60, deadline=None)
def test_property_dense_linearity(bcx, bcy, bcz, nx, ny, nz, hx, hy, hz, seed, gauge):
    bc = bcx * 2 + bcy * 2 + bcz
    h = (hx, hy, hz)
    rng = np.random.default_rng(seed)
    f1 = rng.standard_normal((nz, ny, nx))
    f2 = rng.standard_normal((nz, ny, nx))
    u1 = oracle.solve(f1, bc, h, gauge)
    assert _rel(u1, dense_solve(f1, bc, h, gauge)) < 1e-11
    u12 = oracle.solve(2.0 * f1 - 3.0 * f2, bc, h, gauge)
    assert _rel(u12, 2.0 * u1 - 3.0 * oracle.solve(f2, bc, h, gauge)) < 1e-11


def test_residual_and_gauges_singular():
    rng = np.random.default_rng(9)
    bc, h = "PPPPNN", (0.1, 0.2, 0.3)
    f = rng.standard_normal((6, 5, 4)) + 0.7        # non-zero mean: incompatible
    fp = f - f.mean()
    um = oracle.solve(f, bc, h, "mean")
    up = oracle.solve(f, bc, h, "pin")
    assert abs(um.mean()) < 1e-14 * np.max(np.abs(um))
    assert abs(up[0].mean()) < 1e-14 * np.max(np.abs(up))
    np.testing.assert_allclose(um - up, np.full_like(um, (um - up).mean()), atol=1e-12)
    r = fp - apply_laplacian(um, bc, h)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(fp))
    # raw pin: all equations hold except a common constant absorbed by the plane z = 0
    ur = oracle.solve(f, bc, h, "pin_raw")
    r = f - apply_laplacian(ur, bc, h)
    np.testing.assert_allclose(r[1:], 0.0, atol=1e-11)
    np.testing.assert_allclose(r[0], np.full_like(r[0], r[0].mean()), atol=1e-11)


@pytest.mark.parametrize("name", ["mms_ppd", "noisy_dnn"])
def test_closed_form_manufactured(name):
    """T3: the discrete solution of f = -|w|^2 u* is u* |w|^2 / (-Lambda)."""
    import workloads
    wl = workloads.make(name, shape=(16, 12, 8))
    mode = wl["source_modes"][0]
    u = oracle.solve(-sum(w * w for w in mode["w"]) * wl["ustar"], wl["bc"], wl["h"])
    ratio = closed_form.manufactured_ratio(mode["w"], wl["h"])
    assert _rel(u, ratio * wl["ustar"]) < 1e-12


def test_closed_form_mms_ppd_ratio_value():
    # 32^3 unit cube, w = (2 pi, 2 pi, pi): u_h / u* for the default size of the periodic/Dirichlet case
    h = (1 / 32, 1 / 32, 1 / 32)
    assert abs(closed_form.manufactured_ratio((2 * np.pi, 2 * np.pi, np.pi), h) - 1.0029500125436) < 1e-12


@pytest.mark.parametrize("name,shape", [("modes_ppd", (8, 16, 12)), ("adjoint_ddd", (6, 8, 10))])
def test_closed_form_mode_sums(name, shape):
    """T6: a source that is a sum of discrete eigenmodes has an exact closed-form solution."""
    import workloads
    wl = workloads.make(name, shape=shape, batch=1)
    modes, amps = wl["modes"][0]
    u = oracle.solve(wl["f"][0], wl["bc"], wl["h"])
    uc = closed_form.solve_mode_sum(modes, amps, shape, wl["lengths"])
    assert _rel(u, uc) < 1e-12
    pts = [(0, 0, 0), (shape[0] - 1, 3, 5), (2, shape[1] - 1, shape[2] - 1)]
    at = closed_form.solve_mode_sum_at(modes, amps, shape, wl["lengths"], pts)
    np.testing.assert_allclose(at, [uc[p] for p in pts], atol=1e-12 * np.max(np.abs(uc)))


def _golden_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                rows.append((line[0], line[1], tuple(int(v) for v in line[2:5]), int(line[5]), float(line[6])))
    return rows


def _mms_error(bc, w, N):
    L = np.pi
    h = (L / N,) * 3
    c = (np.arange(N) + 0.5) * h[0]
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    factors = []
    for d, coord in ((0, X), (1, Y), (2, Z)):
        kind = bc[2 * d]
        factors.append({"P": np.exp(1j * w[d] * coord), "N": np.cos(w[d] * coord),
                        "D": np.sin(w[d] * coord)}[kind])
    ustar = factors[0] * factors[1] * factors[2]
    f = -sum(v * v for v in w) * ustar
    u = oracle.solve(f.real, bc, h)
    if np.iscomplexobj(ustar):
        u = u + 1j * oracle.solve(f.imag, bc, h)
    return float(np.sqrt(np.mean(np.abs(u - ustar) ** 2)))


@pytest.mark.parametrize("row", [r for r in _golden_rows() if r[3] == 128], ids=lambda r: r[0])
def test_paper_mms_tables_n128(row):
    table, bc, w, N, printed = row
    err = _mms_error(bc, w, N)
    # printed with six significant digits
    assert abs(err / printed - 1.0) < 1e-5, (table, err, printed)


@pytest.mark.slow
def test_paper_mms_order_of_accuracy():
    """tb4 at N = 128 and 256: observed order p = log(e2/e1)/log(h2/h1) -> 2.00."""
    rows = {r[3]: r for r in _golden_rows() if r[0] == "tb4"}
    e1 = _mms_error("NNNNDD", (1, 2, 3), 128)
    e2 = _mms_error("NNNNDD", (1, 2, 3), 256)
    assert abs(e2 / rows[256][4] - 1.0) < 1e-5
    p = np.log(e2 / e1) / np.log(0.5)
    assert abs(p - 2.0) < 2e-3


def test_convergence_order_closed_form_to_1024():
    """Second-order convergence of the discrete solution for the NN-NN-DD case, N = 16 .. 1024."""
    w = (1.0, 2.0, 3.0)
    errs = []
    Ns = [16, 32, 64, 128, 256, 512, 1024]
    for N in Ns:
        r = closed_form.manufactured_ratio(w, (np.pi / N,) * 3)
        errs.append(abs(r - 1.0))
    p = np.log(np.array(errs[1:]) / np.array(errs[:-1])) / np.log(0.5)
    assert np.all(np.abs(p - 2.0) < 2e-2)
    # the closed form's RMS error matches the paper at N = 1024 (tb4)
    rms_ustar = np.sqrt(0.5 * 0.5 * 0.5)   # mean of cos^2 cos^2 sin^2 over full periods
    assert abs(errs[-1] * rms_ustar / 1.94121e-6 - 1.0) < 1e-4


# --- planted mistakes: the pins above must catch them -------------------------------------

def _plant(monkeypatch, target, attr, replacement):
    monkeypatch.setattr(target, attr, replacement)


def test_planted_wrong_eigenvalue_is_caught(monkeypatch):
    from oracle import eigen
    orig = eigen.eigenvalues

    def wrong(kind, n, h):
        lam = orig(kind, n, h)
        return lam * (1.0 + 1e-3) if kind == "D" else lam
    monkeypatch.setattr(solver, "eigenvalues", wrong)
    f = np.random.default_rng(1).standard_normal((4, 5, 6))
    assert _rel(oracle.solve(f, "DDNNNN", (1, 1, 1)), dense_solve(f, "DDNNNN", (1, 1, 1))) > 1e-6


def test_planted_wrong_end_row_is_caught(monkeypatch):
    orig = solver._z_coefficients

    def wrong(lam, nz, bc, hz):
        a, b, c = orig(lam, nz, bc, hz)
        b = b.copy()
        b[..., 0] -= 1.0 / (hz * hz)       # quadratic-ghost style end row instead of the linear one
        return a, b, c
    monkeypatch.setattr(solver, "_z_coefficients", wrong)
    f = np.random.default_rng(2).standard_normal((4, 5, 6))
    assert _rel(oracle.solve(f, "PPPPDD", (1, 1, 1)), dense_solve(f, "PPPPDD", (1, 1, 1))) > 1e-6


def test_planted_transposed_transform_is_caught(monkeypatch):
    from oracle import transforms
    orig = transforms.forward_matrix
    monkeypatch.setattr(transforms, "forward_matrix", lambda k, n: orig(k, n).T)
    f = np.random.default_rng(3).standard_normal((4, 5, 6))
    assert _rel(oracle.solve(f, "NNDDDD", (1, 1, 1)), dense_solve(f, "NNDDDD", (1, 1, 1))) > 1e-6


def test_planted_dropped_projection_is_caught(monkeypatch):
    f = np.random.default_rng(4).standard_normal((4, 5, 6)) + 1.0
    monkeypatch.setattr(solver, "_mean", lambda v: 0.0 * v.mean(axis=(-3, -2, -1), keepdims=True))
    assert _rel(oracle.solve(f, "PPPPNN", (1, 1, 1)), dense_solve(f, "PPPPNN", (1, 1, 1))) > 1e-6


def test_bc_validation():
    for bad in ["PPPPD", "PDPPDD", "PPNDDD", "XXPPDD", "PPPPPD"]:
        with pytest.raises(ValueError):
            oracle.solve(np.zeros((2, 2, 2)), bad, (1, 1, 1))
    with pytest.raises(ValueError):
        oracle.solve(np.zeros((2, 2, 2)), "PPPPDD", (1, 0, 1))
