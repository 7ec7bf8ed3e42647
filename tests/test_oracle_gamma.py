"""Pins of the gamma-index oracle (Sec. 3.1 agreement test) against closed
forms: identical doses, a uniformly scaled field (no spatial term can help),
and a shifted linear ramp, for which the 3-D lattice search reduces to a 1-D
minimisation along the ramp and trilinear interpolation is exact."""
import math

import numpy as np
import pytest

from oracle import gamma as G


def _grid(n=(9, 10, 11)):
    nz, ny, nx = n
    return np.zeros((nz, ny, nx))


def test_identical_doses_give_zero():
    rng = np.random.default_rng(1)
    ref = rng.uniform(0.5, 2.0, (6, 7, 8)).astype(np.float32)
    g, nr, npass = G.gamma_index(ref, ref, (0.2, 0.25, 0.3), 0.02, 0.2, 0.6)
    assert nr == np.count_nonzero(ref > 0.6) and npass == nr
    assert np.all(g[ref > 0.6] == 0.0) and np.all(g[ref <= 0.6] == -1.0)


@pytest.mark.parametrize("eps", [0.005, -0.015, 0.03, 0.5])
def test_uniform_field_scaled(eps):
    ref = np.full((5, 6, 7), 2.0, np.float32)
    ev = (ref * (1 + eps)).astype(np.float32)
    tol = 0.04
    g, nr, npass = G.gamma_index(ref, ev, (0.4, 0.4, 0.4), tol, 0.2, 0.0, gamma_cap=2.0)
    want = min(2.0, abs(float(ev[0, 0, 0]) - 2.0) / tol)
    assert np.allclose(g, want, rtol=1e-12, atol=0)
    assert npass == (nr if want < 1 else 0)


@pytest.mark.parametrize("shift_cm,slope,dx", [(0.1, 0.5, 0.1), (0.15, 2.0, 0.05),
                                                (0.3, 0.05, 0.1), (0.05, 10.0, 0.1)])
def test_shifted_linear_ramp_closed_form(shift_cm, slope, dx):
    """D_ref = slope x, D_eval(x) = slope (x - shift): gamma^2(r) =
    min_i a (shift - h i)^2 + b (h i)^2, a = slope^2/dD^2, b = 1/dr^2, for
    voxels far enough from the clamped border; it never falls below the
    continuous minimum shift^2 a b / (a + b)."""
    n = 40
    dD, dr, cap, s = 0.02, 0.2, 2.0, 5
    x = (np.arange(n) + 0.5) * dx
    ref = np.broadcast_to(slope * x + 1.0, (3, 4, n)).astype(np.float32)
    ev = np.broadcast_to(slope * (x - shift_cm) + 1.0, (3, 4, n)).astype(np.float32)
    g, _, _ = G.gamma_index(ref, ev, (dx, 0.1, 0.1), dD, dr, -1.0, cap, s)
    a, b, h = slope ** 2 / dD ** 2, 1.0 / dr ** 2, dr / s
    # float32 storage of the doses perturbs them by ~1e-7 relative
    amp = slope * x.max() + 1.0
    i = np.arange(-int(cap * s), int(cap * s) + 1)
    g2 = np.min(a * (shift_cm - h * i) ** 2 + b * (h * i) ** 2)
    want = math.sqrt(min(g2, cap * cap))
    margin = int(math.ceil((cap * dr + shift_cm) / dx)) + 1
    inner = g[:, :, margin:n - margin]
    assert inner.size > 0
    assert np.allclose(inner, want, rtol=0, atol=2e-5 * amp / dD)
    cont = shift_cm * math.sqrt(a * b / (a + b))
    assert want >= min(cap, cont) - 1e-12


def test_region_and_cap():
    ref = np.zeros((4, 4, 4), np.float32)
    ref[1:3, 1:3, 1:3] = 1.0
    ev = ref * 100.0
    g, nr, npass = G.gamma_index(ref, ev, (0.5, 0.5, 0.5), 0.01, 0.2, 0.5, gamma_cap=1.5)
    assert nr == 8 and npass == 0
    assert np.all(g[ref > 0.5] == 1.5) and np.all(g[ref <= 0.5] == -1.0)


def test_lattice_is_a_ball():
    L = G.lattice(0.2, 2.0, 5)
    r2 = (L ** 2).sum(1)
    # r_3(100) = 30 representations of 100 as a sum of three squares
    assert r2.max() <= 100 and (r2 == 100).sum() == 30
    # the count of integer points in a ball of radius 10 (OEIS A000605)
    assert len(L) == 4169
