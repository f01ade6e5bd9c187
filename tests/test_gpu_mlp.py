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


# Element-wise bounds.  The device holds the hidden activations (and, in the
# backward pass, the hidden layers' pre-activation gradients) in BF16 and
# accumulates in FP32; the reference (oracle/mlp.py) keeps FP64 throughout
# with the same BF16 weights.  Each stored value carries a rounding error of at
# most half a BF16 ulp, h(v) = 2^(floor(log2 |v|) - 8); modelled as independent
# and uniform (variance h^2 / 3), they move an output by a zero-mean sum whose
# standard deviation follows from the output's first-order sensitivity to each
# stored value:  sigma^2 = sum_stored (d out / d v)^2 h(v)^2 / 3.  A sum of
# hundreds of such terms is close to Gaussian, so |device - reference| stays
# within K_SIGMA sigma for every one of the ~10^4 compared entries (a tail of
# 8 sigma has probability ~1e-15 per entry); FP32 accumulation adds at most
# GAMMA_K = K u / (1 - K u) (u = 2^-24) of the sum of absolute products.  For
# a weight gradient, a sum over the batch of (dL/dz) x (activation), both
# factors carry the variance of everything that rounded before them: a stored
# activation its own rounding plus that of the layers below it carried up by
# the chain rule, dL/dz the output's forward variance carried down, plus each
# hidden layer's rounding of its stored gradient.  A wrong row or column moves
# an entry by about its own size, 30 or more sigma here.
K_SIGMA = 8.0
U32 = 2.0 ** -24


def _gamma(k):
    return k * U32 / (1 - k * U32)


def _half_ulp_bf16(v):
    a = np.maximum(np.abs(v), 1e-30)
    return np.exp2(np.floor(np.log2(a)) - 8)


def _forward_bound(p, x):
    """Reference outputs, their per-entry tolerance (see above) and the rounding
    variance of each output."""
    y, (zs, acts, Ws) = ref.forward(p, x, WIDTH, HIDDEN)
    lay, _ = ref.layout(WIDTH, HIDDEN)
    bL = p[lay[HIDDEN][3]:lay[HIDDEN][3] + 3]
    tol = _gamma(WIDTH + 1) * (np.abs(acts[HIDDEN]) @ np.abs(Ws[HIDDEN]).T + np.abs(bL))
    # J = d y_i / d a^(l) for every sample, from the output layer down
    J = np.broadcast_to(Ws[HIDDEN], (x.shape[0], 3, WIDTH)).copy()
    var = np.zeros_like(y)
    for l in range(HIDDEN - 1, -1, -1):
        var += ((J * _half_ulp_bf16(acts[l + 1])[:, None, :]) ** 2).sum(2) / 3.0
        if l > 0:
            J = (J * ref.silu_grad(zs[l])[:, None, :]) @ Ws[l]
    return y, tol + K_SIGMA * np.sqrt(var), var


def _activation_variance(p, x):
    """Rounding variance of every stored activation: its own BF16 rounding
    plus the variance of its pre-activation, carried up from the layers
    below (the input is exact)."""
    _, (zs, acts, Ws) = ref.forward(p, x, WIDTH, HIDDEN)
    var = [np.zeros_like(acts[0])]
    for l in range(HIDDEN):
        vz = var[l] @ (Ws[l] ** 2).T
        var.append(ref.silu_grad(zs[l]) ** 2 * vz + _half_ulp_bf16(acts[l + 1]) ** 2 / 3.0)
    return var


def test_forward_matches_reference(net, torch):
    conv, m = net
    say("case: mlp forward element-wise vs the FP64 reference, n = 1000 and 3000 (several passes)")
    rng = np.random.default_rng(0)
    p = m.get_params().numpy().astype(np.float64)
    for n in (1000, 3000):
        x = _inputs(rng, n)
        y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
        want, tol, _ = _forward_bound(p, x.astype(np.float64))
        ratio = np.abs(y - want) / tol
        say(f"  n {n}: max |dy| / bound {ratio.max():.3f}, median bound / |y| {np.median(tol / np.abs(want)):.2e}, "
            f"L2 rel err {_rel(y, want):.2e}")
        assert np.all(ratio <= 1.0)


def test_gradient_matches_reference_and_is_deterministic(net, torch):
    """Weight and bias gradients entry by entry.  The variance of each entry
    sums, over the batch, the variance of the stored activation it multiplies
    (its own rounding and what it inherits from the layers below) and the
    variance of the back-propagated gradient dL/dz it multiplies; the latter
    starts from the output residual (which inherits the forward pass's output
    variance) and is carried down the layers by the chain rule, each hidden
    layer adding the rounding of its own stored gradient."""
    conv, m = net
    say("case: mlp gradient element-wise vs the FP64 reference, n = 512")
    rng = np.random.default_rng(1)
    n = 512
    x = _inputs(rng, n)
    t = rng.normal(size=(n, 3)).astype(np.float32)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss, g = m.gradient(xt, tt)
    loss2, g2 = m.gradient(xt, tt)
    assert torch.equal(g, g2) and torch.equal(loss, loss2)
    p = m.get_params().numpy().astype(np.float64)
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    lw, gw = ref.loss_and_grad(p, x64, t64, WIDTH, HIDDEN)
    assert abs(loss.item() - lw) <= 1e-2 * lw
    y, (zs, acts, Ws) = ref.forward(p, x64, WIDTH, HIDDEN)
    _, _, var_y = _forward_bound(p, x64)
    var_a = _activation_variance(p, x64)
    dz = 2.0 * (y - t64) / y.size            # dL/dy: FP32 on the device, not stored
    vdz = (2.0 / y.size) ** 2 * var_y        # inherited from the forward outputs
    g = g.cpu().numpy().astype(np.float64)
    lay, _ = ref.layout(WIDTH, HIDDEN)
    worst = []
    for l in range(HIDDEN, -1, -1):
        wo, r, c, bo = lay[l]
        a = acts[l]
        va = var_a[l]   # zero for map 0, which multiplies the exact input
        var_w = vdz.T @ (a * a) + (dz * dz).T @ va
        wt = _gamma(n) * (np.abs(dz).T @ np.abs(a)) + K_SIGMA * np.sqrt(var_w)
        bt = _gamma(n) * np.abs(dz).sum(0) + K_SIGMA * np.sqrt(vdz.sum(0))
        rw = np.abs(g[wo:wo + r * c].reshape(r, c) - gw[wo:wo + r * c].reshape(r, c)) / wt
        rb = np.abs(g[bo:bo + r] - gw[bo:bo + r]) / bt
        say(f"  map {l}: max |dg| / bound weights {rw.max():.3f}, biases {rb.max():.3f}; "
            f"L2 rel err {_rel(g[wo:wo + r * c], gw[wo:wo + r * c]):.2e}")
        worst.append(max(rw.max(), rb.max()))
        if l > 0:
            sg = ref.silu_grad(zs[l - 1])
            dz_next = (dz @ Ws[l]) * sg
            vdz = (vdz @ (Ws[l] ** 2)) * sg ** 2 + _half_ulp_bf16(dz_next) ** 2 / 3.0
            dz = dz_next
    assert max(worst) <= 1.0


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


@pytest.mark.parametrize("width, hidden", [(64, 2), (192, 3), (384, 3), (512, 4)])
def test_apply_equals_forward_all_instances(torch, width, hidden):
    """The fused epilogue is instantiated per width (64-row workgroups below 256, 128-row
    ones from 256 up): at each shape it runs the same network as forward(), so the TOD
    differs from the host sum over forward()'s outputs only by the final rounding (one ulp),
    over a stream whose length is not a multiple of either row count."""
    from paper_1908_05662_amd.api import Convolver, Mlp
    from synth import workloads as W
    from gpu_helpers import load_workload

    say(f"case: fused epilogue against forward(), width {width}, {hidden} hidden layers")
    conv = Convolver(0)
    m = Mlp(conv, width, hidden, max_batch=64, seed=11 + width)
    try:
        w = W.c1(n_samples=1000)
        load_workload(conv, w, np.float32)
        x = m.features(0)
        y = m.forward(x).cpu().numpy().astype(np.float64)
        tod = torch.linspace(-1, 1, 1000, dtype=torch.float32, device="cuda")
        base = tod.cpu().numpy().astype(np.float64)
        mean, std, coef = [0.05, 0.1, -0.3], [1.5, 0.25, 0.75], [-0.6, 0.9, 1.3]
        m.apply(0, mean, std, coef, tod)
        want = base + sum(coef[c] * (np.float32(mean[c]) + np.float64(np.float32(std[c])) * y[:, c])
                          for c in range(3))
        got = tod.cpu().numpy()
        ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - want) <= ulp)
    finally:
        torch.cuda.synchronize()
        m.close()
        conv.close()
