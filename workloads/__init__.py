"""Seeded synthetic inputs for the Poisson solve (shared by the tests, the bench
and the oracle checks).

This module only draws random numbers and evaluates source fields on the grid;
it holds none of the solver's arithmetic (no transforms, no eigenvalues, no
tridiagonal solves).  All fields are float64, C-ordered (B, nz, ny, nx) with x
fastest, on cell centres x_i = (i + 1/2) h of a box of side lengths L.

Workloads (sizes are the defaults; every recipe also takes a smaller shape for
fast parity tests):

mms_ppd        32^3, periodic x,y / Dirichlet z, unit cube.
               u* = sin(2 pi x) sin(2 pi y) sin(pi z), f = -9 pi^2 u*.
noisy_dnn      256^3, Dirichlet x / Neumann y / Neumann z, unit cube.
               u* = sin(pi x) cos(2 pi y) cos(3 pi z), f = -14 pi^2 u* + e with
               e i.i.d. N(0, 0.01) (standard deviation 0.1), then the mean of f
               is subtracted.
div_ppn        512^3, periodic x,y / Neumann z, unit cube.  A staggered velocity
               field with i.i.d. N(0, 1) components on the cell faces (periodic
               in x and y, zero normal velocity on the two z walls);
               f = discrete divergence (face differences / h).  sum(f) = 0 up
               to rounding.
modes_ppd      1024 x 1024 x 512 (nx, ny, nz), periodic x,y / Dirichlet z, unit
               cube.  64 modes a cos(2 pi (kx x + ky y) + phi) sin(pi kz z),
               a ~ N(0,1), kx, ky uniform in [-8, 8], kz uniform in [1, 8],
               phi ~ U[0, 2 pi).
adjoint_ddd    384^3 x batch 4, Dirichlet everywhere, unit cube.  For each batch
               entry a source and a target field, each a sum of 64 modes
               a sin(pi kx x) sin(pi ky y) sin(pi kz z), k uniform in [1, 8],
               a ~ N(0,1).

Mode lists are returned with every mode-built field so that exact solutions
can be formed independently of the solver.
"""

import numpy as np

TWO_PI = 2.0 * np.pi
HALF_PI = 0.5 * np.pi

WORKLOADS = {
    "mms_ppd": dict(shape=(32, 32, 32), bc="PPPPDD", batch=1, seed=1),
    "noisy_dnn": dict(shape=(256, 256, 256), bc="DDNNNN", batch=1, seed=2),
    "div_ppn": dict(shape=(512, 512, 512), bc="PPPPNN", batch=1, seed=3),
    "modes_ppd": dict(shape=(512, 1024, 1024), bc="PPPPDD", batch=1, seed=4),
    "adjoint_ddd": dict(shape=(384, 384, 384), bc="DDDDDD", batch=4, seed=50),
}


def _centres(n, length=1.0):
    return (np.arange(n) + 0.5) * (length / n)


def _factor(w, phase, coord):
    return np.cos(w * coord + phase)


def _eval_modes(modes, amps, shape, lengths=(1.0, 1.0, 1.0)):
    """sum_m amps[m] * mode_m on the grid, as one (nz x 2M) @ (2M x ny*nx) product."""
    nz, ny, nx = shape
    x = _centres(nx, lengths[0])
    y = _centres(ny, lengths[1])
    z = _centres(nz, lengths[2])
    zcols, xyrows = [], []
    for m, a in zip(modes, amps):
        wx, wy, wz = m["w"]
        if m["form"] == "sep":
            px, py, pz = m["phase"]
            zcols.append(a * _factor(wz, pz, z))
            xyrows.append(np.outer(_factor(wy, py, y), _factor(wx, px, x)).reshape(-1))
        else:  # xywave: cos(wx x + wy y + p) = cos(wx x) cos(wy y + p) - sin(wx x) sin(wy y + p)
            pxy, pz = m["phase"]
            zf = a * _factor(wz, pz, z)
            zcols += [zf, -zf]
            xyrows.append(np.outer(np.cos(wy * y + pxy), np.cos(wx * x)).reshape(-1))
            xyrows.append(np.outer(np.sin(wy * y + pxy), np.sin(wx * x)).reshape(-1))
    Z = np.stack(zcols, axis=1)
    XY = np.stack(xyrows, axis=0)
    return (Z @ XY).reshape(shape)


def _sep_sine_modes(rng, count, kmax=8):
    k = rng.integers(1, kmax + 1, size=(count, 3))
    a = rng.standard_normal(count)
    modes = [dict(form="sep", w=(np.pi * kx, np.pi * ky, np.pi * kz),
                  phase=(-HALF_PI, -HALF_PI, -HALF_PI)) for kx, ky, kz in k]
    return modes, a


def make(name, shape=None, batch=None, seed=None):
    """Build workload `name`; returns a dict with f of shape (B, nz, ny, nx) and metadata."""
    spec = dict(WORKLOADS[name])
    shape = tuple(shape) if shape is not None else spec["shape"]
    batch = batch if batch is not None else spec["batch"]
    seed = seed if seed is not None else spec["seed"]
    nz, ny, nx = shape
    lengths = (1.0, 1.0, 1.0)
    h = (lengths[0] / nx, lengths[1] / ny, lengths[2] / nz)
    out = dict(name=name, shape=shape, bc=spec["bc"], batch=batch, h=h, lengths=lengths, seed=seed)

    if name == "mms_ppd":
        mode = dict(form="sep", w=(TWO_PI, TWO_PI, np.pi), phase=(-HALF_PI, -HALF_PI, -HALF_PI))
        ustar = _eval_modes([mode], [1.0], shape)
        w2 = sum(w * w for w in mode["w"])
        f = -w2 * ustar
        out.update(f=np.broadcast_to(f, (batch,) + shape).copy(), ustar=ustar,
                   source_modes=[mode], source_amps=[-w2])
    elif name == "noisy_dnn":
        mode = dict(form="sep", w=(np.pi, TWO_PI, 3 * np.pi), phase=(-HALF_PI, 0.0, 0.0))
        ustar = _eval_modes([mode], [1.0], shape)
        w2 = sum(w * w for w in mode["w"])
        rng = np.random.default_rng(seed)
        fs = []
        for _ in range(batch):
            f = -w2 * ustar + 0.1 * rng.standard_normal(shape)
            fs.append(f - f.mean())
        out.update(f=np.stack(fs), ustar=ustar, source_modes=[mode], source_amps=[-w2])
    elif name == "div_ppn":
        rng = np.random.default_rng(seed)
        fs = []
        for _ in range(batch):
            vx = rng.standard_normal(shape)
            vy = rng.standard_normal(shape)
            vz = np.zeros((nz + 1, ny, nx))
            vz[1:nz] = rng.standard_normal((nz - 1, ny, nx))
            f = (np.roll(vx, -1, axis=2) - vx) / h[0]
            f += (np.roll(vy, -1, axis=1) - vy) / h[1]
            f += (vz[1:] - vz[:-1]) / h[2]
            fs.append(f)
            del vx, vy, vz
        out.update(f=np.stack(fs))
    elif name == "modes_ppd":
        rng = np.random.default_rng(seed)
        fs, mlist = [], []
        for _ in range(batch):
            kx = rng.integers(-8, 9, size=64)
            ky = rng.integers(-8, 9, size=64)
            kz = rng.integers(1, 9, size=64)
            a = rng.standard_normal(64)
            phi = rng.uniform(0.0, TWO_PI, size=64)
            modes = [dict(form="xywave", w=(TWO_PI * i, TWO_PI * j, np.pi * k), phase=(p, -HALF_PI))
                     for i, j, k, p in zip(kx, ky, kz, phi)]
            fs.append(_eval_modes(modes, a, shape))
            mlist.append((modes, a))
        out.update(f=np.stack(fs), modes=mlist)
    elif name == "adjoint_ddd":
        fs, ts, mlist, tlist = [], [], [], []
        for b in range(batch):
            modes, a = _sep_sine_modes(np.random.default_rng(seed + 2 * b), 64)
            tmodes, ta = _sep_sine_modes(np.random.default_rng(seed + 2 * b + 1), 64)
            fs.append(_eval_modes(modes, a, shape))
            ts.append(_eval_modes(tmodes, ta, shape))
            mlist.append((modes, a))
            tlist.append((tmodes, ta))
        out.update(f=np.stack(fs), target=np.stack(ts), modes=mlist, target_modes=tlist)
    else:
        raise KeyError(name)
    return out


def random_field(shape, seed, batch=1):
    """Plain i.i.d. N(0,1) source (used for tiny parity cases of any boundary combination)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch,) + tuple(shape))
