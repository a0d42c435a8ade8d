"""The seeded input generators (no method arithmetic): the thin-inclusion
fields and the Dirichlet left/right boundary data."""
import numpy as np

from paper_2606_08883_amd import workloads as wl
from paper_2606_08883_amd.configs import WORKLOADS


def test_inclusions_are_seeded_thin_and_of_the_stated_contrast():
    for kind, values in (("high", {1.0, 1e4}), ("low", {1.0, 1e-4}), ("both", {1.0, 1e4, 1e-4})):
        K = wl.inclusions_K(160, 160, kind, 11)
        assert np.array_equal(K, wl.inclusions_K(160, 160, kind, 11))
        assert not np.array_equal(K, wl.inclusions_K(160, 160, kind, 12))
        assert set(np.unique(K)) == values
        frac = np.mean(K != 1.0)
        assert 0.01 < frac < 0.2  # thin: a few percent of the cells
    Kb = wl.inclusions_K(160, 160, "both", 11)
    assert Kb.max() / Kb.min() == 1e8
    # 24 segments one cell thick and at most 0.45 of the side long per kind
    for kind in ("high", "low"):
        assert np.count_nonzero(wl.inclusions_K(160, 160, kind, 11) != 1.0) <= 24 * 72


def test_dirichlet_left_right_data():
    f, g = wl.dirichlet_left_right(40, 30)
    assert f.shape == (1200,) and not f.any()
    assert np.array_equal(g[:30], np.ones(30)) and not g[30:].any()
    w = WORKLOADS["incl-low"]
    assert w.bc == (1, 1, 0, 0) and w.field == "incl-low"
    f2, g2 = w.boundary_data()
    assert g2.shape == (2 * w.ny + 2 * w.nx,)


def test_mixture_spans_the_contrast_with_channel_facies():
    K = wl.mixture_K(256, 256, 5, 6)
    assert abs(K.max() - 1.0) < 1e-15 and abs(K.max() / K.min() / 1e8 - 1.0) < 1e-9
    chi = wl.gaussian_field(256, 256, 160.0, 24.0, 5) > 0.0
    # the facies still separate the field: channel cells are on average
    # about the facies contrast (1e4, stretched) more permeable
    ratio = np.exp(np.log(K[chi.ravel()]).mean() - np.log(K[~chi.ravel()]).mean())
    assert 1e3 < ratio < 1e6
    assert 0.3 < chi.mean() < 0.7


def test_gaussian_field3_is_seeded_unit_variance_and_correlated():
    g = wl.gaussian_field3(48, 40, 32, 4.0, 7)
    assert g.shape == (32, 40, 48)
    assert np.array_equal(g, wl.gaussian_field3(48, 40, 32, 4.0, 7))
    assert abs(g.std() - 1.0) < 0.2 and abs(g.mean()) < 0.3
    # covariance exp(-r^2 / ell^2) along every axis at lag 2: exp(-1/4)
    for ax in range(3):
        a = np.moveaxis(g, ax, 0)
        c = np.mean(a[2:] * a[:-2]) / np.mean(a * a)
        assert abs(c - np.exp(-0.25)) < 0.1
    K = wl.lognormal_K3(16, 12, 8, 2.0, 3.0, 5)
    assert K.shape == (16 * 12 * 8,) and np.all(K > 0)
    b = wl.corner_sources3(4, 3, 2)
    assert b[0] == 1.0 and b[23] == -1.0 and np.count_nonzero(b) == 2


def test_cube_workload():
    from paper_2606_08883_amd.configs import WORKLOADS3
    w = WORKLOADS3["cube"]
    assert (w.nx, w.ny, w.nz, w.s) == (96, 96, 96, 8) and not any(w.bc)
    cfg = w.binding_config()
    assert (cfg.sx, cfg.oversample, cfg.degree, cfg.sweeps) == (8, 2, 1, 1)
    assert w.permeability().shape == (w.cells,)
