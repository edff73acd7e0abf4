"""The paper's printed manufactured-solution errors reproduced by the GPU
solver at full size (section "Verification and Validation" -> "Order of
Accuracy", Tables tb3-tb7): N = 512 and 1024 cells per direction on [0, pi]^3,
source f = -|w|^2 u* (the continuous Laplacian sampled at cell centres), RMS
error of the f64 solve against u*, compared with the printed six-digit values
of tests/golden/mms_tables.txt (readings there); the observed order between
N = 512 and 1024 is 2.

Fields are formed on the GPU (separable products) so nothing of size N^3
passes through host memory.
"""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mms_tables.txt")


def _rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                rows.append((line[0], line[1], tuple(int(v) for v in line[2:5]), int(line[5]), float(line[6])))
    return rows


def _gpu_mms_error(bc, w, N):
    import torch
    from paper_1909_05423_amd import Plan
    L = np.pi
    h = L / N
    c = (torch.arange(N, dtype=torch.float64, device="cuda") + 0.5) * h
    fac = []
    for d in range(3):
        kind = bc[2 * d]
        if kind == "P":
            fac.append((torch.cos(w[d] * c), torch.sin(w[d] * c)))   # exp(i w x) as (re, im)
        elif kind == "N":
            fac.append((torch.cos(w[d] * c), None))
        else:
            fac.append((torch.sin(w[d] * c), None))

    def cmul(a, b):   # complex 1-D factors as (re, im or None)
        if a[1] is None and b[1] is None:
            return (a[0] * b[0], None)
        ar, ai = a
        br, bi = b
        if ai is None:
            return (ar * br, ar * bi)
        if bi is None:
            return (ar * br, ai * br)
        return (ar * br - ai * bi, ar * bi + ai * br)

    # u* = fx(x) fy(y) fz(z) on the (z, y, x) grid, as real and imaginary parts
    fx, fy, fz = fac
    parts = []
    for comp in (0, 1):
        def outer(zf, yf, xf):
            return zf[:, None, None] * yf[None, :, None] * xf[None, None, :]
        # expand the complex product of three factors into real tensors
        terms = []
        for zi, zt in enumerate([fz[0], fz[1]]):
            for yi, yt in enumerate([fy[0], fy[1]]):
                for xi, xt in enumerate([fx[0], fx[1]]):
                    if zt is None or yt is None or xt is None:
                        continue
                    k = zi + yi + xi   # power of i
                    sign = [1, 1, -1, -1][k]
                    if (k % 2) != comp:
                        continue
                    terms.append((sign, zt, yt, xt))
        if not terms:
            parts.append(None)
            continue
        u = None
        for sign, zt, yt, xt in terms:
            t = outer(zt, yt, xt)
            u = sign * t if u is None else u + sign * t
        parts.append(u)
    w2 = float(sum(v * v for v in w))
    plan = Plan((N, N, N), bc, (h, h, h), dtype="f64")
    sq = 0.0
    for ustar in parts:
        if ustar is None:
            continue
        f = (-w2 * ustar).contiguous()
        u = plan.solve(f)
        sq += float(((u - ustar) ** 2).sum())
        del f, u
    del parts, plan
    torch.cuda.empty_cache()
    return float(np.sqrt(sq / N ** 3))


@pytest.mark.parametrize("table", ["tb3", "tb4", "tb5", "tb6", "tb7"])
def test_paper_mms_tables_512_and_1024(table):
    from gpu_util import banner
    rows = {r[3]: r for r in _rows() if r[0] == table}
    errs = {}
    for N in (512, 1024):
        _, bc, w, _, printed = rows[N]
        banner(f"MMS {table} {bc} w={w} N={N}")
        errs[N] = _gpu_mms_error(bc, w, N)
        banner(f"   rms error {errs[N]:.6e}, printed {printed:.6e}")
        assert abs(errs[N] / printed - 1.0) < 1e-5, (table, N, errs[N], printed)
    p = np.log(errs[1024] / errs[512]) / np.log(0.5)
    assert abs(p - 2.0) < 2e-3, p
