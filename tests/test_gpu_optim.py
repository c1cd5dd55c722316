"""Adam over the map parameters on the GPU (gsl_adam_step,
gsl_window_optimize) against the oracle's Adam and activations."""
import numpy as np
import pytest
import torch

import scenegen as S

from gpuutil import context, ops

pytestmark = pytest.mark.gpu


def _rand_state(N, seed):
    rng = np.random.default_rng(seed)
    raw = rng.normal(size=(14, N)).astype(np.float32)
    raw[3:6] = rng.uniform(-4, -1, (3, N))  # log-scale
    return raw


def _gaussians(O, N):
    z = lambda *s: torch.zeros(*s, dtype=torch.float32, device="cuda")
    return O.Gaussians(z(3, N), z(3, N), z(4, N), z(N), z(3, N))


def _act_np(g):
    return {k: getattr(g, k).cpu().numpy().astype(np.float64).reshape(-1, g.N) for k in
            ("mean", "scale", "quat", "opacity", "color")}


def test_adam_activate_matches_oracle(oracle):
    O = ops()
    ctx = context()
    N = 3000
    raw = _rand_state(N, 1)
    st = O.AdamState(torch.from_numpy(raw).cuda())
    g = _gaussians(O, N)
    O.adam_activate(ctx, st, g)
    torch.cuda.synchronize()
    want = oracle.activate(raw)
    got = _act_np(g)
    for k in want:
        np.testing.assert_allclose(got[k], want[k], rtol=2e-6, atol=1e-7, err_msg=k)


@pytest.mark.parametrize("sh_degree", [0, 2])
def test_adam_init_matches_oracle(oracle, sh_degree):
    """gsl_adam_init: raw rows = the oracle's inverse activation of the
    activated parameters (log-scale, opacity logit, the rest as they are),
    moments and step count zero; at a row stride above N (a window kept at a
    fixed capacity) the padding columns are left alone."""
    O = ops()
    ctx = context()
    N, ld = 2999, 3072
    rng = np.random.default_rng(11)
    act = {"mean": rng.normal(size=(3, N)), "scale": np.exp(rng.uniform(-5, 0, (3, N))),
           "quat": rng.normal(size=(4, N)), "opacity": rng.uniform(1e-3, 1 - 1e-3, (1, N)),
           "color": rng.uniform(0, 1, (3, N))}
    K = (sh_degree + 1) ** 2 - 1
    if K:
        act["sh"] = rng.normal(0, 0.3, (3 * K, N))
    act = {k: a.astype(np.float32) for k, a in act.items()}
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = O.Gaussians(t(act["mean"]), t(act["scale"]), t(act["quat"]), t(act["opacity"][0]), t(act["color"]),
                    t(act["sh"]) if K else None)
    rows = 14 + 3 * K
    block = torch.full((3 * rows, ld), 7.0, dtype=torch.float32, device="cuda")
    st = O.AdamState(block[:rows], block[rows:2 * rows], block[2 * rows:], n=N)
    st.d_step.fill_(5)
    gs, ss = g.struct(), st.struct()
    import ctypes as C
    from paper_2501_08672_amd import _abi as A
    A.check(A.lib().gsl_adam_init(ctx.h, C.byref(gs), C.byref(ss), None))
    torch.cuda.synchronize()
    want = oracle.deactivate({k: a.astype(np.float64) for k, a in act.items()})
    b = block.cpu().numpy()
    # float32 log of float32 inputs: a few ulp of the result
    np.testing.assert_allclose(b[:rows, :N], want, rtol=1e-6, atol=2e-7)
    assert np.all(b[rows:, :N] == 0.0)
    assert np.all(b[:, N:] == 7.0)
    assert int(st.d_step.item()) == 0
    # round trip through the activation
    g2 = O.Gaussians(*(torch.empty_like(x) for x in (g.mean, g.scale, g.quat, g.opacity, g.color)),
                     torch.empty_like(g.sh) if K else None)
    O.adam_activate(ctx, st, g2)
    torch.cuda.synchronize()
    for k in ("mean", "scale", "quat", "opacity", "color") + (("sh",) if K else ()):
        np.testing.assert_allclose(getattr(g2, k).cpu().numpy().reshape(-1, N), act[k].reshape(-1, N), rtol=2e-6,
                                   atol=1e-7, err_msg=k)


def test_adam_steps_match_oracle(oracle):
    """Three steps with changing gradients: raw values, moments and the
    activated outputs follow the oracle (float32 against float64)."""
    O = ops()
    ctx = context()
    N = 5000
    rng = np.random.default_rng(2)
    raw = _rand_state(N, 3)
    st = O.AdamState(torch.from_numpy(raw).cuda())
    g = _gaussians(O, N)
    grads = O.Grads(N, 1, "cuda")
    lr = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)
    hp = O.adam_hparams(lr=lr, eps=1e-8)
    x, m, v = raw.astype(np.float64), np.zeros((14, N)), np.zeros((14, N))
    # the oracle gets the hyper-parameters the device receives (float32 values)
    f32 = lambda a: np.float32(a).astype(np.float64)
    lr_rows = np.repeat(f32(np.array(lr)), [3, 3, 4, 1, 3])
    b1, b2, eps = f32(0.9), f32(0.999), f32(1e-8)
    for t in range(1, 4):
        g_act = {"mean": rng.normal(size=(3, N)), "scale": rng.normal(size=(3, N)), "quat": rng.normal(size=(4, N)),
                 "opacity": rng.normal(size=(1, N)), "color": rng.normal(size=(3, N))}
        for k, arr in g_act.items():
            getattr(grads, k).copy_(torch.from_numpy(arr.astype(np.float32).reshape(getattr(grads, k).shape)))
        g_act = {k: a.astype(np.float32).astype(np.float64) for k, a in g_act.items()}
        O.adam_step(ctx, st, hp, grads, g)
        x, m, v = oracle.adam_step(x, m, v, oracle.raw_gradient(x, g_act), t, lr_rows, beta1=b1, beta2=b2, eps=eps)
    torch.cuda.synchronize()
    assert int(st.d_step.item()) == 3
    np.testing.assert_allclose(st.m.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(st.v.cpu().numpy(), v, rtol=1e-5, atol=1e-9)
    # raw values of magnitude up to ~4 are stored in float32: ~5e-7 absolute
    np.testing.assert_allclose(st.raw.cpu().numpy(), x, rtol=1e-5, atol=1e-6)
    want = oracle.activate(x)
    got = _act_np(g)
    for k in want:
        np.testing.assert_allclose(got[k], want[k], rtol=2e-5, atol=1e-6, err_msg=k)


def _optim_setup(O, ctx, seed=5):
    sc = S.config1()
    tgt = S.jitter_means(sc, 0.02, seed)
    tgt.cams = sc.cams
    cs = O.CameraSet(sc.cams)
    o = O.opts(16)
    gt = O.Gaussians.from_scene(tgt)
    pt = O.project(ctx, gt, cs, o)
    bt = O.bin_sort(ctx, cs, gt.N, o, pt)
    target, _, _ = O.render_fwd(ctx, cs, gt.N, o, pt, bt)
    g = O.Gaussians.from_scene(sc)
    st = O.AdamState.from_gaussians(ctx, g)
    O.adam_activate(ctx, st, g)
    win = O.Window(ctx, g, cs, o, target.clone(), loss="l1", headroom=1.5)
    return win, st


def test_window_optimize_graph_matches_eager_steps():
    """gsl_window_optimize (one graph of iterations) against the same
    iterations as separate eager window and Adam steps."""
    O = ops()
    ctx = context()
    hp = O.adam_hparams(lr=(1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3), eps=1e-8)
    win_a, st_a = _optim_setup(O, ctx)
    win_b, st_b = _optim_setup(O, ctx)
    losses = win_a.optimize(st_a, hp, iters=4, use_graph=True).clone()
    eager = []
    for _ in range(4):
        win_b.step(use_graph=False)
        eager.append(float(win_b.d_loss.item()))
        O.adam_step(ctx, st_b, hp, win_b.grads, win_b.g)
    torch.cuda.synchronize()
    assert win_a.status() == 0 and win_b.status() == 0
    np.testing.assert_allclose(losses.cpu().numpy(), eager, rtol=1e-4)
    a, b = st_a.raw.cpu().numpy(), st_b.raw.cpu().numpy()
    # float32 atomics order the 2D-gradient sums differently run to run, and
    # Adam normalises the step, so a gradient near zero can step either way:
    # nearly all parameters agree to far below the learning rates
    bad = np.abs(a - b) > 2e-4
    assert bad.mean() < 2e-3, (bad.sum(), bad.size)
    assert int(st_a.d_step.item()) == 4 and int(st_b.d_step.item()) == 4


def test_window_optimize_reduces_loss_and_replays():
    """Ten iterations lower the L1 loss against the jittered target, and a
    second call (a replay of the recorded graph) continues from there."""
    O = ops()
    ctx = context()
    win, st = _optim_setup(O, ctx, seed=6)
    hp = O.adam_hparams(lr=(2e-3, 5e-3, 1e-3, 5e-2, 2.5e-3))
    l1 = win.optimize(st, hp, iters=10).clone()
    l2 = win.optimize(st, hp, iters=10).clone()
    torch.cuda.synchronize()
    assert win.status() == 0
    l1, l2 = l1.cpu().numpy(), l2.cpu().numpy()
    assert l1[-1] < 0.9 * l1[0], l1
    assert l2[-1] < l1[-1], (l1, l2)
    assert int(st.d_step.item()) == 20
