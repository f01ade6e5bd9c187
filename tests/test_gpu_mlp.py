"""GPU kernels of the far-sidelobe network against the FP64 reference (through the C ABI)."""
import numpy as np
import pytest

from oracle import mlp as ref

from gpu_helpers import say

pytestmark = pytest.mark.gpu
WIDTH, HIDDEN = 256, 4


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture()
def net(torch):
    from paper_1908_05662_amd.api import Convolver, Mlp

    conv = Convolver(0)
    m = Mlp(conv, WIDTH, HIDDEN, max_batch=1024, seed=7)
    yield conv, m
    torch.cuda.synchronize()
    m.close()
    conv.close()


def _inputs(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    psi = rng.uniform(0, 2 * np.pi, n)
    return np.concatenate([v, np.sin(psi)[:, None], np.cos(psi)[:, None]], 1).astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - b) / max(np.linalg.norm(b), 1e-300))


def test_forward_matches_reference(net, torch):
    conv, m = net
    say("case: mlp forward, n = 1000 and 3000 (ragged, several passes)")
    rng = np.random.default_rng(0)
    p = m.get_params().numpy().astype(np.float64)
    for n in (1000, 3000):
        x = _inputs(rng, n)
        y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
        want, _ = ref.forward(p, x.astype(np.float64), WIDTH, HIDDEN)
        e = _rel(y, want)
        say(f"  n {n}: relative error {e:.3e}")
        assert e < 1e-2  # BF16 activations between layers, FP32 accumulation


def test_gradient_matches_reference_and_is_deterministic(net, torch):
    conv, m = net
    say("case: mlp gradient, n = 512")
    rng = np.random.default_rng(1)
    x = _inputs(rng, 512)
    t = rng.normal(size=(512, 3)).astype(np.float32)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss, g = m.gradient(xt, tt)
    loss2, g2 = m.gradient(xt, tt)
    assert torch.equal(g, g2) and torch.equal(loss, loss2)
    p = m.get_params().numpy().astype(np.float64)
    lw, gw = ref.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64), WIDTH, HIDDEN)
    assert abs(loss.item() - lw) < 1e-2 * lw
    g = g.cpu().numpy()
    lay, _ = ref.layout(WIDTH, HIDDEN)
    for l, (wo, r, c, bo) in enumerate(lay):
        ew = _rel(g[wo:wo + r * c], gw[wo:wo + r * c])
        eb = _rel(g[bo:bo + r], gw[bo:bo + r])
        say(f"  map {l}: weight grad rel err {ew:.3e}, bias grad rel err {eb:.3e}")
        assert ew < 3e-2 and eb < 3e-2


def test_adam_step_matches_reference(net, torch):
    conv, m = net
    say("case: mlp adam steps")
    rng = np.random.default_rng(2)
    x = torch.from_numpy(_inputs(rng, 256)).cuda()
    t = torch.from_numpy(rng.normal(size=(256, 3)).astype(np.float32)).cuda()
    p = m.get_params().numpy().astype(np.float64)
    mm = np.zeros_like(p)
    vv = np.zeros_like(p)
    for step in (1, 2, 3):
        _, g = m.gradient(x, t)
        m.train_step(x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)
        p, mm, vv = ref.adam_step(p, mm, vv, g.cpu().numpy().astype(np.float64), step, 1e-3, 0.9, 0.999, 1e-8)
        got = m.get_params().numpy().astype(np.float64)
        err = np.abs(got - p).max()
        say(f"  step {step}: max |param - reference| {err:.3e}")
        assert err < 2e-6


def test_training_reduces_loss(net, torch):
    conv, m = net
    say("case: mlp training on a smooth field")
    rng = np.random.default_rng(3)
    x = _inputs(rng, 8192)
    tgt = np.stack([np.sin(2 * x[:, 0]) * x[:, 2], x[:, 1] * x[:, 4] - x[:, 0] * x[:, 3],
                    np.cos(3 * x[:, 2]) * x[:, 3]], 1).astype(np.float32)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    first = None
    for it in range(300):
        b = (it * 1024) % 8192
        loss = m.train_step(xt[b:b + 1024], tt[b:b + 1024], lr=2e-3).item()
        first = loss if first is None else first
    say(f"  loss {first:.4e} -> {loss:.4e}")
    assert loss < 0.05 * first


def test_features_and_apply(net, torch):
    conv, m = net
    say("case: sidelobe features and TOD epilogue")
    from synth import workloads as W
    from gpu_helpers import load_workload

    w = W.c1(n_samples=777)
    load_workload(conv, w, np.float32)
    d = w.detectors[0]
    x = m.features(0).cpu().numpy()
    st = np.sin(d.theta)
    want = np.stack([st * np.cos(d.phi), st * np.sin(d.phi), np.cos(d.theta), np.sin(d.psi), np.cos(d.psi)], 1)
    assert np.abs(x - want).max() < 1e-6
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    tod = torch.linspace(-1, 1, 777, dtype=torch.float32, device="cuda")
    base = tod.cpu().numpy().astype(np.float64)
    mean, std, coef = [0.1, -0.2, 0.3], [2.0, 0.5, 1.5], [0.7, -1.1, 0.4]
    m.apply(0, mean, std, coef, tod)
    want = base + sum(coef[c] * (np.float32(mean[c]) + np.float64(np.float32(std[c])) * y[:, c]) for c in range(3))
    # the fused epilogue runs the network itself: its outputs equal forward()'s bit for bit, so the TOD can
    # differ only by the rounding of the double epilogue to float (one ulp); a changed network output would
    # move it by far more
    got = tod.cpu().numpy()
    ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got - want) <= ulp)
