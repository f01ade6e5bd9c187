"""Circular polarisation (V) and a rotating half-wave plate on the GPU, against
the oracle (which carries both through its literal 4x4 Mueller chain)."""
import numpy as np
import pytest

import oracle
from synth import beams as B
from synth import workloads as W

from gpu_helpers import rel_err, say

pytestmark = pytest.mark.gpu
D2R = np.pi / 180
F64_TOL = 1e-12
F32_TOL = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture()
def conv(torch):
    from paper_1908_05662_amd.api import Convolver

    c = Convolver(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _beams(scalar_v):
    """(n, n, 4, 4) Mueller fields on a 121^2 grid over +-2 deg: a full one
    (Q<->U and V->T, V->Q leakage, elliptical) and, if scalar_v, a one-grid
    one whose V column is proportional to the main beam."""
    T, u, v, rho, sig = B.tangent_grid(121, 2.0 * D2R)
    g = B.elliptical_gaussian(rho, sig, 0.6 * D2R, 0.08, 0.4)
    full = B.with_qu_leakage(B.ideal_beamsor(g, T), g, 0.02).dense().copy()
    full[:, :, 0, 3] = 0.03 * B.elliptical_gaussian(rho, sig, 0.7 * D2R, 0.0, 0.0)   # V -> T, another shape
    full[:, :, 1, 3] = 0.01 * g                                                       # V -> Q
    one = B.ideal_beamsor(g, T).dense().copy()
    if scalar_v:
        one[:, :, 0, 3] = 0.05 * g
    return T, full, one


def _scan(n):
    w = W.c2(n_samples=n)
    d = w.detectors[0]
    return w, d.theta, d.phi, d.psi


def _load(conv, torch, w, dtype, M, T, zeta, eps, s, th, ph, ps, hwp, V, scalar_ok, det=0, rmax=1.8 * D2R,
          norm=W.NORM_PER_SAMPLE, scale=1.0):
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    kind = conv.set_beamsor(det, M, T, eps, s, dtype=tdt, allow_scalar=scalar_ok)
    conv.set_detector(det, zeta, 0.0, rmax, norm, scale)
    conv.set_pointing(det, *(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (th, ph, ps)))
    conv.set_hwp(det, None if hwp is None else torch.from_numpy(np.ascontiguousarray(hwp)).cuda())
    return kind


def _oracle(w, dtype, M, T, zeta, eps, s, th, ph, ps, hwp, V, mode=oracle.OUT_TOD, rmax=1.8 * D2R,
            norm=W.NORM_PER_SAMPLE, scale=1.0):
    r = (lambda x: np.asarray(x, dtype=dtype).astype(np.float64))
    M = r(M) if dtype == np.float32 else M
    return oracle.tod(w.nside, *(r(m) for m in w.sky), M, T, zeta, eps, s, 0.0, rmax, norm, scale, th, ph, ps, mode,
                      V=None if V is None else r(V), hwp=hwp)


@pytest.mark.parametrize("dtype,tol,algo", [(np.float64, F64_TOL, 0), (np.float32, F32_TOL, 0),
                                            (np.float32, F32_TOL, 1), (np.float32, F32_TOL, 2)])
@pytest.mark.parametrize("beam", ["full", "scalar"])
@pytest.mark.parametrize("plate", [False, True])
def test_v_and_plate_parity(conv, torch, dtype, tol, algo, beam, plate):
    """CES scan (coherent tiles) of the nside-512 sky plus a V map; a plate
    spinning at 2 Hz at 100 samples/s when `plate`; sampled outputs vs the oracle."""
    say(f"case: V/plate {np.dtype(dtype).name} algo {algo} beam {beam} plate {plate}")
    n = 20_000
    w, th, ph, ps = _scan(n)
    rng = np.random.default_rng(31)
    V = 0.05 * rng.standard_normal(w.sky[0].size)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    conv.set_sky(w.nside, *(torch.from_numpy(np.asarray(m, dtype=dtype)).cuda() for m in w.sky), dtype=tdt,
                 V=torch.from_numpy(V.astype(dtype)).cuda())
    conv.set_launch(algorithm=algo)
    T, full, one = _beams(scalar_v=True)
    M = full if beam == "full" else one
    hwp = (2 * np.pi * 2.0 / 100.0) * np.arange(n) + 0.3 if plate else None
    kind = _load(conv, torch, w, dtype, M, T, 0.35, 0.03, 1.2, th, ph, ps, hwp, V, scalar_ok=(beam == "scalar"))
    assert kind == beam
    idx = np.linspace(0, n - 1, 60).astype(int)
    for mode in (oracle.OUT_TOD, oracle.OUT_STOKES):
        got = conv.convolve(0, out_mode=mode).cpu().numpy()
        want = _oracle(w, dtype, M, T, 0.35, 0.03, 1.2, th[idx], ph[idx], ps[idx],
                       None if hwp is None else hwp[idx], V, mode)
        e = rel_err(got[idx], want)
        say(f"  mode {mode}: max rel err {e:.3e}")
        assert e <= tol


def test_plate_is_visible_and_periodic(conv, torch):
    """The plate changes the TOD, and phi -> phi + pi/2 leaves it unchanged (FP32 tile path)."""
    say("case: plate period on the GPU")
    n = 8192
    w, th, ph, ps = _scan(n)
    conv.set_sky(w.nside, *(torch.from_numpy(np.asarray(m, dtype=np.float32)).cuda() for m in w.sky))
    T, full, one = _beams(scalar_v=False)
    hw = np.linspace(0.0, 6.0, n)
    _load(conv, torch, w, np.float32, full, T, 0.1, 0.0, 1.0, th, ph, ps, None, None, scalar_ok=False)
    plain = conv.convolve(0).cpu().numpy()
    conv.set_hwp(0, hw)
    a = conv.convolve(0).cpu().numpy()
    conv.set_hwp(0, hw + np.pi / 2)
    b = conv.convolve(0).cpu().numpy()
    assert rel_err(a, b) <= 2e-6
    assert rel_err(a, plain) > 1e-3


def test_batched_launch_mixes_plate_and_plain_detectors(conv, torch):
    """One batched launch with a plate on detector 1 only; each detector's slice
    equals its own single-detector launch and the oracle."""
    from paper_1908_05662_amd import PiscoError

    say("case: batched launch, plate on one detector")
    n = 6000
    w, th, ph, ps = _scan(n)
    conv.set_sky(w.nside, *(torch.from_numpy(np.asarray(m, dtype=np.float32)).cuda() for m in w.sky))
    T, full, one = _beams(scalar_v=False)
    hw = np.linspace(0.0, 9.0, n)
    for k in range(3):
        _load(conv, torch, w, np.float32, one, T, 0.2 * k, 0.01, 1.0, th, ph, ps, hw if k == 1 else None, None,
              scalar_ok=True, det=k)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        allv = conv.convolve(-1, stream=stream).clone()
    stream.synchronize()
    allv = allv.cpu().numpy()
    idx = np.linspace(0, n - 1, 30).astype(int)
    for k in range(3):
        single = conv.convolve(k).cpu().numpy()
        assert rel_err(allv[k * n:(k + 1) * n], single) <= 2e-6
        want = _oracle(w, np.float32, one, T, 0.2 * k, 0.01, 1.0, th[idx], ph[idx], ps[idx],
                       hw[idx] if k == 1 else None, None)
        assert rel_err(single[idx], want) <= F32_TOL
    # a plate stream of the wrong length is an error at convolve time
    conv.set_hwp(2, hw[:100])
    with pytest.raises(PiscoError):
        conv.convolve(2)


def test_v_column_lds_slice_on_every_tile_shape(conv, torch):
    """A full beam with a V column stages one more float per record and wave;
    the largest tile shape (8 waves x 256 records) still fits the 160 KiB of a
    compute unit with it, and every shape gives the default shape's result."""
    say("case: V-column LDS slice vs launch shape")
    n = 4096
    w, th, ph, ps = _scan(n)
    rng = np.random.default_rng(5)
    V = 0.05 * rng.standard_normal(w.sky[0].size)
    conv.set_sky(w.nside, *(torch.from_numpy(np.asarray(m, dtype=np.float32)).cuda() for m in w.sky),
                 V=torch.from_numpy(V.astype(np.float32)).cuda())
    T, full, one = _beams(scalar_v=False)
    _load(conv, torch, w, np.float32, full, T, 0.3, 0.02, 1.0, th, ph, ps, None, V, scalar_ok=False)
    conv.set_launch(algorithm=1)
    ref = conv.convolve(0).cpu().numpy()
    for wpg, ch in [(8, 256), (8, 128), (4, 64), (1, 256)]:
        conv.set_launch(waves_per_group=wpg, chunk=ch)
        assert rel_err(conv.convolve(0).cpu().numpy(), ref) <= 2e-6, (wpg, ch)
    idx = np.linspace(0, n - 1, 16).astype(int)
    want = _oracle(w, np.float32, full, T, 0.3, 0.02, 1.0, th[idx], ph[idx], ps[idx], None, V)
    assert rel_err(ref[idx], want) <= F32_TOL
