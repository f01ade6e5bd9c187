"""Host-side logic of the far-sidelobe surrogate (no GPU): the sample ordering
and the split of the TOD into main disc + annulus pickup that the network
learns, checked with the oracle."""
import numpy as np

import oracle
from synth import beams as B
from synth import sky as SK

from paper_1908_05662_amd.surrogate import _hilbert_index, detector_coef, network_flops_per_sample, spatial_order

D2R = np.pi / 180


def test_hilbert_curve_is_a_unit_step_walk():
    for n in (2, 4, 16):
        xs, ys = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        d = _hilbert_index(n, xs.ravel(), ys.ravel())
        assert sorted(d.tolist()) == list(range(n * n))
        o = np.argsort(d)
        steps = np.abs(np.diff(xs.ravel()[o])) + np.abs(np.diff(ys.ravel()[o]))
        assert (steps == 1).all()


def test_spatial_order_is_a_permutation_with_local_neighbours():
    rng = np.random.default_rng(0)
    n = 200_000
    th, ph = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n)
    o = spatial_order(th, ph)
    assert np.array_equal(np.sort(o), np.arange(n))
    p = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)[o]
    # consecutive samples are close: the median angular step is a few mean spacings
    step = np.arccos(np.clip((p[1:] * p[:-1]).sum(1), -1, 1))
    spacing = np.sqrt(4 * np.pi / n)
    assert np.median(step) < 3 * spacing
    # and a group of 64 stays compact (median within 10, 95% within 20 spacings of its mean)
    g = p[: (n // 64) * 64].reshape(-1, 64, 3)
    c = g.mean(1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    rad = np.arccos(np.clip((g * c[:, None, :]).sum(2), -1, 1)).max(1)
    assert np.median(rad) < 10 * spacing and np.quantile(rad, 0.95) < 20 * spacing


def test_tod_splits_into_main_disc_and_annulus_pickup():
    """For an ideal beamsor, d(rho <= R) = d(rho <= r) + sum_c coef_c P_c(r < rho <= R),
    with P the Stokes pickup in the zeta = 0 frame -- the decomposition the
    network is trained on (oracle only)."""
    nside = 16
    I, Q, U = SK.make_sky(nside, 3 * nside - 1, 2.0, seed=11)
    T, u, v, rho, sig = B.tangent_grid(81, 25 * D2R)
    g = B.elliptical_gaussian(rho, sig, 3 * D2R) + B.ring_lobe(rho, 12 * D2R, 3 * D2R, 0.05)
    M = B.ideal_beamsor(g, T).dense()
    rng = np.random.default_rng(4)
    th, ph, ps = np.arccos(rng.uniform(-1, 1, 7)), rng.uniform(0, 2 * np.pi, 7), rng.uniform(0, 2 * np.pi, 7)
    for zeta, eps, s in [(0.0, 0.0, 1.0), (0.7, 0.1, 1.3), (-1.2, -0.05, 0.8)]:
        args = (nside, I, Q, U, M, T, zeta, eps, s)
        full = oracle.tod(*args, 0.0, 20 * D2R, 0, 1e-3, th, ph, ps)
        main = oracle.tod(*args, 0.0, 6 * D2R, 0, 1e-3, th, ph, ps)
        P = oracle.tod(nside, I, Q, U, M, T, 0.0, eps, s, 6 * D2R, 20 * D2R, 0, 1e-3, th, ph, ps, oracle.OUT_STOKES)
        c = detector_coef(zeta, eps, s)
        split = main + P @ np.array(c)
        assert np.abs(split - full).max() <= 1e-12 * np.abs(full).max()


def test_network_flop_count():
    assert network_flops_per_sample(256, 4) == 2 * (5 * 256 + 3 * 256 * 256 + 256 * 3) == 397312
