"""GPU harmonic analysis and power spectra against the FP64 oracle (through the C ABI).

Parity: a_lm and spectra element by element at sizes the oracle finishes in
seconds (several ring lengths with odd factors, lmax below, at and above
3 nside - 1), and at the benchmark size (nside 1024, lmax 3071) on sampled m
columns, which the oracle computes one by one.  FP64 on both sides: the
tolerance is 1e-12 of the largest |a_lm| (sums of ~1e4 terms of FP64 products)."""
import numpy as np
import pytest

from oracle import spectra as S

from gpu_helpers import say

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture(scope="module")
def conv(torch):
    from paper_1908_05662_amd.api import Convolver

    c = Convolver(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _maps(nside, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(3, 12 * nside * nside))


def _gpu_alm(torch, conv, nside, lmax, maps, pol=True):
    from paper_1908_05662_amd.api import Spectra

    sp = Spectra(conv, nside, lmax, pol=pol)
    dev = [torch.from_numpy(m).cuda() for m in maps]
    out = sp.map2alm(*(dev if pol else dev[:1]))
    torch.cuda.synchronize()
    return sp, [None if a is None else a.cpu().numpy() for a in out]


@pytest.mark.parametrize("nside,lmax", [(1, 2), (4, 11), (16, 47), (32, 128), (64, 191), (64, 100)])
def test_alm_parity(torch, conv, nside, lmax):
    say(f"case: map2alm parity nside {nside} lmax {lmax}")
    maps = _maps(nside, nside + lmax)
    _, (gT, gE, gB) = _gpu_alm(torch, conv, nside, lmax, maps)
    oT, oE, oB = S.map2alm(*maps, S.healpix_rings(nside), lmax)
    for name, g, o in (("T", gT, oT), ("E", gE, oE), ("B", gB, oB)):
        err = np.abs(g - o).max() / np.abs(o).max()
        say(f"  a^{name}: max |gpu - oracle| / max |a| = {err:.2e}")
        assert err < TOL


def test_spectra_parity(torch, conv):
    nside, lmax = 32, 95
    say(f"case: anafast parity nside {nside} lmax {lmax}")
    from paper_1908_05662_amd.api import Spectra

    maps = _maps(nside, 5)
    sp = Spectra(conv, nside, lmax)
    cl = sp.anafast(*(torch.from_numpy(m).cuda() for m in maps)).cpu().numpy()
    want = S.anafast(nside, lmax, *maps)
    for k, name in enumerate(S.SPECTRA):
        err = np.abs(cl[k] - want[k]).max() / np.abs(want[:3]).max()
        say(f"  {name}: {err:.2e}")
        assert err < TOL
    # alm2cl on the buffers of the last analysis reproduces the TE column
    te = sp.alm2cl(sp.alm[0], sp.alm[1]).cpu().numpy()
    assert np.abs(te - want[3]).max() < TOL * np.abs(want[:3]).max()


def test_temperature_only(torch, conv):
    nside, lmax = 16, 40
    say(f"case: temperature-only analysis nside {nside} lmax {lmax}")
    from paper_1908_05662_amd.api import Spectra

    maps = _maps(nside, 9)
    sp, (gT, gE, gB) = _gpu_alm(torch, conv, nside, lmax, maps[:1], pol=False)
    assert gE is None and gB is None
    oT, _, _ = S.map2alm(maps[0], None, None, S.healpix_rings(nside), lmax)
    assert np.abs(gT - oT).max() < TOL * np.abs(oT).max()
    cl = sp.anafast(torch.from_numpy(maps[0]).cuda()).cpu().numpy()
    assert cl.shape == (1, lmax + 1)
    assert np.abs(cl[0] - S.alm2cl(oT, oT, lmax)).max() < TOL * np.abs(cl).max()


def test_bad_arguments(torch, conv):
    from paper_1908_05662_amd.api import Spectra

    with pytest.raises(ValueError):
        Spectra(conv, 24, 10)              # not a power of two
    with pytest.raises(ValueError):
        Spectra(conv, 2048, 10)            # above the largest nside
    with pytest.raises(ValueError):
        Spectra(conv, 8, 33)               # lmax above 4 nside
    sp = Spectra(conv, 8, 10)
    T = torch.zeros(12 * 64, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        sp.map2alm(T, T, None)             # Q without U
    with pytest.raises(ValueError):
        sp.map2alm(T[:100])                # wrong size
    from paper_1908_05662_amd import _lib as L

    lib = conv._lib
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    rc = lib.pisco_map2alm(conv._h, 8, 10, 0, T.data_ptr(), None, None, sp.alm[0].data_ptr(), None, None,
                           small.data_ptr(), small.numel(), None)
    assert rc == L.EINVAL and b"workspace" in lib.pisco_last_error(conv._h)
    rc = lib.pisco_map2alm(conv._h, 8, 10, 17, T.data_ptr(), None, None, sp.alm[0].data_ptr(), None, None,
                           sp.workspace.data_ptr(), sp.workspace.numel(), None)
    assert rc == L.EINVAL and b"iterations" in lib.pisco_last_error(conv._h)
    with pytest.raises(ValueError):
        sp.alm2map(sp.alm[0], sp.alm[1], None)  # a^E without a^B


def test_full_size_sampled_columns(torch, conv):
    """nside 1024, lmax 3071 (the benchmark analysis) in one launch pair; the
    oracle computes the columns m = 0, 1, 17, 1024, 2900, 3071 for every l."""
    nside, lmax = 1024, 3071
    say(f"case: map2alm full size nside {nside} lmax {lmax}, sampled m columns")
    maps = _maps(nside, 11)
    _, (gT, gE, gB) = _gpu_alm(torch, conv, nside, lmax, maps)
    ms = [0, 1, 17, 1024, 2900, 3071]
    oT, oE, oB = S.map2alm(*maps, S.healpix_rings(nside), lmax, ms=ms)
    for m in ms:
        k = S.alm_index(lmax, np.arange(m, lmax + 1), m)
        for name, g, o in (("T", gT, oT), ("E", gE, oE), ("B", gB, oB)):
            scale = np.abs(o[k]).max()
            err = np.abs(g[k] - o[k]).max() / scale
            say(f"  m {m} a^{name}: {err:.2e} (max |a| {scale:.2e})")
            assert err < TOL
    assert np.all(np.isfinite(gT)) and np.all(np.isfinite(gE)) and np.all(np.isfinite(gB))


@pytest.mark.parametrize("nside,lmax", [(1, 3), (8, 23), (32, 95), (64, 191), (16, 64)])
def test_alm2map_parity(torch, conv, nside, lmax):
    from paper_1908_05662_amd.api import Spectra

    say(f"case: alm2map parity nside {nside} lmax {lmax}")
    rng = np.random.default_rng(100 + nside)
    n = S.alm_size(lmax)
    al = []
    for f in range(3):
        a = rng.normal(size=n) + 1j * rng.normal(size=n)
        a[S.alm_index(lmax, np.arange(lmax + 1), 0)] = a[S.alm_index(lmax, np.arange(lmax + 1), 0)].real
        al.append(a)
    sp = Spectra(conv, nside, lmax)
    got = sp.alm2map(*(torch.from_numpy(a).cuda() for a in al))
    torch.cuda.synchronize()
    want = S.alm2map(*al, S.healpix_rings(nside), lmax)
    for name, g, w in zip("TQU", got, want):
        err = np.abs(g.cpu().numpy() - w).max() / np.abs(w).max()
        say(f"  {name}: {err:.2e}")
        assert err < TOL
    Tonly = sp.alm2map(torch.from_numpy(al[0]).cuda())
    assert Tonly[1] is None and np.abs(Tonly[0].cpu().numpy() - want[0]).max() < TOL * np.abs(want[0]).max()


def test_iterated_analysis_parity_and_convergence(torch, conv):
    """Three Jacobi steps on the GPU equal the oracle's, and shrink the quadrature
    error of a band-limited field by orders of magnitude."""
    from paper_1908_05662_amd.api import Spectra

    nside, lmax = 16, 20
    say(f"case: iterated map2alm nside {nside} lmax {lmax}")
    rng = np.random.default_rng(5)
    n = S.alm_size(lmax)
    truth = []
    for f in range(3):
        a = rng.normal(size=n) + 1j * rng.normal(size=n)
        a[S.alm_index(lmax, np.arange(lmax + 1), 0)] = a[S.alm_index(lmax, np.arange(lmax + 1), 0)].real
        if f:
            a[S.alm_index(lmax, np.array([0, 1, 1]), np.array([0, 0, 1]))] = 0.0
        truth.append(a)
    R = S.healpix_rings(nside)
    maps = S.alm2map(*truth, R, lmax)
    sp = Spectra(conv, nside, lmax)
    dev = [torch.from_numpy(m).cuda() for m in maps]
    errs = []
    for it in (0, 3):
        got = [a.cpu().numpy() for a in sp.map2alm(*dev, iterations=it)]
        want = S.map2alm_iter(*maps, R, lmax, it)
        for g, w in zip(got, want):
            assert np.abs(g - w).max() < TOL * np.abs(w).max()
        errs.append(max(np.abs(g - t).max() for g, t in zip(got, truth)) / np.abs(truth[0]).max())
    say(f"  error against the input a_lm: {errs[0]:.2e} (one pass), {errs[1]:.2e} (3 iterations)")
    assert errs[1] < 1e-3 * errs[0]
