"""The paper's ideal whole-sky CMB validation (Sec. 6.2) with every step on the GPU:
convolution of an E-only polarised sky with a 1.5 deg Gaussian beam at every
nside-128 pixel centre for psi = 0, 45, 90 deg (one detector, zeta = 0), binned
maps, then the spectra of those maps divided by the beam transfer function and
compared with the spectra of the input maps.  Also the two variants the paper
runs next: pointings offset randomly from the pixel centres (spurious B from
intra-pixel gradients) and offsets symmetric about the centres (that B
suppressed by orders of magnitude), and a temperature-only sky (no T to P).

The sky follows a CMB-like recipe of our own (no Boltzmann code here) at
nside 256 instead of 512; the quantities compared are the paper's."""
import numpy as np
import pytest

from oracle import spectra as S
from synth import beams as B
from synth import scans as SC
from synth import sky as SK
from synth import workloads as W

from gpu_helpers import say

pytestmark = pytest.mark.gpu
D2R = np.pi / 180.0
NSIDE_SKY, LMAX_SKY = 256, 767
NSIDE_MAP, LMAX = 128, 383
FWHM = 1.5 * D2R
L_LO, L_HI = 2, 200
ITER = 3                      # Jacobi steps of the spectrum estimator (the usual anafast default)


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture(scope="module")
def setup(torch):
    from paper_1908_05662_amd.api import Convolver, Spectra

    conv = Convolver(0)
    cl = SK.cmb_like_cl(LMAX_SKY)
    (I, Q, U), _ = SK.make_teb_sky(NSIDE_SKY, LMAX_SKY, cl, seed=W.SEED_BASE + 62)
    conv.set_sky(NSIDE_SKY, *(torch.from_numpy(m).cuda() for m in (I, Q, U)), dtype=torch.float64)
    T, u, v, rho, sig = B.tangent_grid(201, 5.0 * D2R)
    g = B.elliptical_gaussian(rho, sig, FWHM)
    bs = B.ideal_beamsor(g, T)
    conv.set_beamsor(0, bs.dense(), bs.half_span_tan, 0.0, 1.0, dtype=torch.float64)
    conv.set_detector(0, 0.0, 0.0, 5.0 * D2R, W.NORM_PER_SAMPLE, 1.0)
    sp_in = Spectra(conv, NSIDE_SKY, LMAX)
    cl_in = sp_in.anafast(*(torch.from_numpy(m).cuda() for m in (I, Q, U)), iterations=ITER).cpu().numpy()
    yield conv, (I, Q, U), cl_in
    torch.cuda.synchronize()
    conv.close()


def _observe(conv, torch, sky, th, ph, psi, nside_sky=NSIDE_SKY):
    from paper_1908_05662_amd.api import MapMaker, Spectra

    conv.set_sky(nside_sky, *(torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in sky), dtype=torch.float64)
    conv.set_pointing(0, *(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (th, ph, psi)))
    tod = conv.convolve(0)
    maps, rc = MapMaker(conv, NSIDE_MAP).add(th, ph, psi, tod, 0.0, 0.0, 1.0).solve()
    assert float(rc.min()) > 0.1                    # every pixel seen at three angles
    return Spectra(conv, NSIDE_MAP, LMAX).anafast(maps[0], maps[1], maps[2], iterations=ITER).cpu().numpy()


def _beam_corrected(cl):
    bT = S.gauss_beam_window(FWHM, LMAX)
    bP = S.gauss_beam_window(FWHM, LMAX, spin=2)
    out = cl.copy()
    out[0] /= bT * bT
    out[1] /= bP * bP
    out[2] /= bP * bP
    out[3] /= bT * bP
    return out


def _offset_scan(rng, symmetric):
    """Offsets uniform in +-half a pixel size in theta and in phi sin(theta), redrawn
    (seeded) until the offset pointing, and for the symmetric scan its mirror about
    the centre as well, stays inside the pixel: the maps then keep every pixel's
    three angles and the offsets act only inside pixels."""
    import oracle

    th, ph, psi = SC.pixel_centre_scan(NSIDE_MAP)
    pix = oracle.ang2pix(NSIDE_MAP, th, ph)
    size = np.sqrt(4 * np.pi / (12 * NSIDE_MAP ** 2))          # pixel size (rad)
    dth = np.zeros_like(th)
    dph = np.zeros_like(th)
    todo = np.arange(th.size)
    while todo.size:
        dth[todo] = rng.uniform(-0.5, 0.5, todo.size) * size
        dph[todo] = rng.uniform(-0.5, 0.5, todo.size) * size / np.sin(th[todo])
        out = oracle.ang2pix(NSIDE_MAP, th[todo] + dth[todo], ph[todo] + dph[todo]) != pix[todo]
        if symmetric:
            out |= oracle.ang2pix(NSIDE_MAP, th[todo] - dth[todo], ph[todo] - dph[todo]) != pix[todo]
        todo = todo[out]
    if symmetric:
        return (np.concatenate([th + dth, th - dth]), np.concatenate([ph + dph, ph - dph]),
                np.concatenate([psi, psi]))
    return th + dth, ph + dph, psi


def test_ideal_cmb_pixel_centres(setup, torch):
    conv, sky, cl_in = setup
    say("case: ideal CMB, pixel centres, E-only sky nside 256 -> maps nside 128")
    th, ph, psi = SC.pixel_centre_scan(NSIDE_MAP)
    cl = _beam_corrected(_observe(conv, torch, sky, th, ph, psi))
    ls = slice(L_LO, L_HI + 1)
    rt = np.abs(cl[0, ls] / cl_in[0, ls] - 1.0)
    re = np.abs(cl[1, ls] / cl_in[1, ls] - 1.0)
    leak = cl[2, ls] / cl_in[1, ls]
    say(f"  TT residual median {np.median(rt):.2e} max {rt.max():.2e}; EE median {np.median(re):.2e} "
        f"max {re.max():.2e}; BB / EE_in max {leak.max():.2e}")
    assert np.median(rt) < 1e-2 and np.median(re) < 1e-2
    assert leak.max() < 1e-4                        # no E to B leakage


def test_no_temperature_to_polarisation(setup, torch):
    conv, sky, _ = setup
    say("case: temperature-only sky through the same chain")
    th, ph, psi = SC.pixel_centre_scan(NSIDE_MAP)
    z = np.zeros_like(sky[0])
    cl = _observe(conv, torch, (sky[0], z, z), th, ph, psi)
    ls = slice(L_LO, L_HI + 1)
    tp = max((cl[1, ls] / cl[0, ls]).max(), (cl[2, ls] / cl[0, ls]).max())
    say(f"  max (EE, BB) / TT = {tp:.2e}")
    assert tp < 1e-6


def test_random_versus_symmetric_offsets(setup, torch):
    conv, sky, cl_in = setup
    say("case: pointings offset from pixel centres, random and symmetric")
    rng = np.random.default_rng(7)
    cl_r = _observe(conv, torch, sky, *_offset_scan(rng, False))
    rng = np.random.default_rng(7)
    cl_s = _observe(conv, torch, sky, *_offset_scan(rng, True))
    ls = slice(50, L_HI + 1)
    bb_r, bb_s = cl_r[2, ls].mean(), cl_s[2, ls].mean()
    ee = cl_in[1, ls].mean()
    say(f"  mean BB over l 50..200: random {bb_r:.3e}, symmetric {bb_s:.3e} (ratio {bb_r / bb_s:.1f}); "
        f"random BB / EE_in {bb_r / ee:.2e}")
    assert bb_r > 1e-6 * ee                         # a spurious B appears with random offsets
    assert bb_s < 1e-2 * bb_r                       # symmetric offsets suppress it


def test_ideal_cmb_paper_configuration(torch):
    """The same pixel-centre run in the paper's own configuration: sky at nside 512
    and the 1.5 deg Gaussian given as an nside-2048 HEALPix beam map (resampled by
    the library onto a 201^2 grid over +-5 deg)."""
    from paper_1908_05662_amd.api import Convolver, Spectra

    say("case: ideal CMB, paper configuration (sky nside 512, beam map nside 2048)")
    nside_sky, lmax_sky = 512, 1535
    conv = Convolver(0)
    try:
        cl = SK.cmb_like_cl(lmax_sky)
        sky, _ = SK.make_teb_sky(nside_sky, lmax_sky, cl, seed=W.SEED_BASE + 63)
        conv.set_sky(nside_sky, *(torch.from_numpy(m).cuda() for m in sky), dtype=torch.float64)
        bmap = B.healpix_beam_map(2048, FWHM, rho_max_rad=6.0 * D2R)
        conv.set_beam_healpix_scalar(0, 2048, 201, np.tan(5.0 * D2R), bmap, 0.5, 0.5, 0.0, 1.0, dtype=torch.float64)
        conv.set_detector(0, 0.0, 0.0, 5.0 * D2R, W.NORM_PER_SAMPLE, 1.0)
        cl_in = Spectra(conv, nside_sky, LMAX).anafast(*(torch.from_numpy(m).cuda() for m in sky),
                                                       iterations=ITER).cpu().numpy()
        th, ph, psi = SC.pixel_centre_scan(NSIDE_MAP)
        out = _beam_corrected(_observe(conv, torch, sky, th, ph, psi, nside_sky=nside_sky))
    finally:
        torch.cuda.synchronize()
        conv.close()
    ls = slice(L_LO, L_HI + 1)
    rt = np.abs(out[0, ls] / cl_in[0, ls] - 1.0)
    re = np.abs(out[1, ls] / cl_in[1, ls] - 1.0)
    leak = out[2, ls] / cl_in[1, ls]
    say(f"  TT residual median {np.median(rt):.2e} max {rt.max():.2e}; EE median {np.median(re):.2e} "
        f"max {re.max():.2e}; BB / EE_in max {leak.max():.2e}")
    assert np.median(rt) < 1e-2 and np.median(re) < 1e-2
    assert leak.max() < 1e-4


def _pair_leakage(torch, T_sky, dx=0.0, ell=0.0):
    """A detector pair (zeta = 0 and -90 deg) at every nside-128 pixel centre and
    psi = 0, 45, 90 deg on a temperature-only sky; the second detector's beam is
    offset by dx (radians, along its theta') and/or elongated (ellipticity ell).
    Both are binned into one set of maps; returns mean (EE + BB) / TT over l 50..200."""
    from paper_1908_05662_amd.api import Convolver, MapMaker, Spectra

    conv = Convolver(0)
    try:
        z = np.zeros_like(T_sky)
        conv.set_sky(NSIDE_SKY, *(torch.from_numpy(m).cuda() for m in (T_sky, z, z)), dtype=torch.float64)
        Tg, u, v, rho, sig = B.tangent_grid(201, 5.0 * D2R)
        th, ph, psi = SC.pixel_centre_scan(NSIDE_MAP)
        th1, ph1, psi1 = SC.offset_pointing(th, ph, psi, dx, 0.0)
        pts = [(th, ph, psi), (th1, ph1, psi1)]
        zetas = [0.0, -np.pi / 2]
        for k in range(2):
            g = B.elliptical_gaussian(rho, sig, FWHM, ell if k else 0.0, 0.3)
            bs = B.ideal_beamsor(g, Tg)
            conv.set_beamsor(k, bs.dense(), bs.half_span_tan, 0.0, 1.0, dtype=torch.float64)
            conv.set_detector(k, zetas[k], 0.0, 5.0 * D2R, W.NORM_PER_SAMPLE, 1.0)
            conv.set_pointing(k, *(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in pts[k]))
        tod = conv.convolve(-1)
        n = th.size
        mm = MapMaker(conv, NSIDE_MAP)
        for k in range(2):
            mm.add(*pts[k], tod[k * n:(k + 1) * n], zetas[k], 0.0, 1.0)
        maps, rc = mm.solve()
        assert float(rc.min()) > 0.1
        cl = Spectra(conv, NSIDE_MAP, LMAX).anafast(maps[0], maps[1], maps[2], iterations=ITER).cpu().numpy()
    finally:
        torch.cuda.synchronize()
        conv.close()
    ls = slice(50, L_HI + 1)
    return float(((cl[1, ls] + cl[2, ls]) / cl[0, ls]).mean())


def test_pair_mismatch_leakage(setup, torch):
    """Sec. 7's systematics on synthetic inputs: a matched detector pair leaks no
    temperature into polarisation; a pointing offset or an elongated beam on one
    detector of the pair does, and the leaked power grows as the square of the
    mismatch (the difference beam is first order in it)."""
    _, sky, _ = setup
    say("case: detector-pair mismatch on a temperature-only sky")
    base = _pair_leakage(torch, sky[0])
    d1 = _pair_leakage(torch, sky[0], dx=0.01 * D2R)
    d2 = _pair_leakage(torch, sky[0], dx=0.02 * D2R)
    e1 = _pair_leakage(torch, sky[0], ell=0.02)
    e2 = _pair_leakage(torch, sky[0], ell=0.04)
    say(f"  (EE + BB) / TT, l 50..200: matched {base:.2e}; pointing 0.01 deg {d1:.2e}, 0.02 deg {d2:.2e} "
        f"(ratio {d2 / d1:.2f}); ellipticity 0.02 {e1:.2e}, 0.04 {e2:.2e} (ratio {e2 / e1:.2f})")
    assert base < 1e-6
    assert d1 > 10 * base and e1 > 10 * base
    assert 3.0 < d2 / d1 < 5.0 and 3.0 < e2 / e1 < 5.0
