"""Host report tools (Fig. 6 profiles): interpolation and beam geometry
against closed forms, on analytic dose fields (no GPU)."""
import numpy as np

from paper_1109_3266_amd import dose_report as R
from synth import workloads as W


def _grid_coords(g):
    x = g["ox"] + (np.arange(g["nx"]) + 0.5) * g["dx"]
    y = g["oy"] + (np.arange(g["ny"]) + 0.5) * g["dy"]
    z = g["oz"] + (np.arange(g["nz"]) + 0.5) * g["dz"]
    return np.meshgrid(z, y, x, indexing="ij")


def test_trilinear_sample_exact_on_linear_fields():
    g = dict(nx=7, ny=5, nz=4, dx=0.3, dy=0.5, dz=0.7, ox=-1.0, oy=2.0, oz=0.5)
    Z, Y, X = _grid_coords(g)
    f = 2.0 * X - 3.0 * Y + 0.5 * Z + 1.0
    rng = np.random.default_rng(3)
    lo = np.array([g["ox"] + g["dx"] / 2, g["oy"] + g["dy"] / 2, g["oz"] + g["dz"] / 2])
    hi = lo + np.array([(g["nx"] - 1) * g["dx"], (g["ny"] - 1) * g["dy"], (g["nz"] - 1) * g["dz"]])
    p = lo + rng.random((200, 3)) * (hi - lo)
    want = 2.0 * p[:, 0] - 3.0 * p[:, 1] + 0.5 * p[:, 2] + 1.0
    assert np.allclose(R.sample(f, g, p), want, rtol=0, atol=1e-12)
    # outside the centres the value is clamped to the nearest face
    q = np.array([[lo[0] - 5, lo[1], lo[2]]])
    assert np.allclose(R.sample(f, g, q), 2.0 * lo[0] - 3.0 * lo[1] + 0.5 * lo[2] + 1.0)


def test_fig6_profiles_of_an_analytic_beam():
    """Water box geometry: beam along -y entering at y = +10 cm; a dose
    exp(-mu d) * (1 + x^2/100) gives an exponential depth curve and a
    symmetric lateral profile along the bow-tie direction only."""
    wl = W.water_box_bowtie(scale=2)
    g, geo = wl.grid, wl.geometry
    src, axis, ea, eb = R.beam_frame(geo)
    assert np.allclose(axis, [0, -1, 0]) and np.allclose(ea, [1, 0, 0])
    assert np.allclose(R.entry_depth_point(g, src, axis), [0, 10, 0])
    Z, Y, X = _grid_coords(g)
    mu = 0.2
    dose = np.exp(-mu * (10.0 - Y)) * (1.0 + X * X / 100.0)
    out = R.fig6_profiles(dose, np.zeros_like(dose), g, geo, depth_cm=3.0)
    d, v, s = out["depth"]
    inner = (d > 1.0) & (d < 19.0)
    ratio = v[inner][1:] / v[inner][:-1]
    step = d[1] - d[0]
    assert np.allclose(ratio, np.exp(-mu * step), rtol=1e-9)
    t, va, _ = out["lateral_a"]
    tb, vb, _ = out["lateral_b"]
    m = np.abs(t) < 9.0
    assert np.allclose(va[m], va[m][::-1], rtol=1e-9)          # symmetric in x
    assert np.ptp(vb[np.abs(tb) < 9.0]) < 1e-9                  # flat along z
    assert va[m].max() > 1.5 * va[m].min()
