"""Pins of the surrogate MLP oracle: library routines (torch's float64
autograd, Adam and bfloat16 conversion) and finite differences, so that a
dropped term, a transposed operand or a wrong sign in the oracle fails."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from paper_2407_02363_amd import inputs


def rand_params(seed, scale=0.2):
    g = inputs.rng(seed)
    return [(g.normal(0, scale, (o, i)), g.normal(0, 0.05, o)) for i, o in M.LAYERS]


def test_bf16_rounding_matches_torch():
    g = inputs.rng(0)
    x = np.concatenate([g.normal(0, 10, 5000), g.normal(0, 1e-3, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3.0e38, -2.5e-38]])
    # exact ties at bf16 precision: 1 + 2^-8 rounds to even (1.0), 1 + 3*2^-8 up
    x = np.concatenate([x, [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8)]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_encode_order_and_closed_form():
    x = M.encode(np.zeros((1, 7)), rounding=False)
    assert np.array_equal(x[0], np.tile([0.0, 1.0], 7))
    q = np.array([[np.pi / 2, 0, 0, 0, 0, 0, -np.pi / 2]])
    x = M.encode(q, rounding=False)
    assert np.allclose(x[0, :2], [1, 0]) and np.allclose(x[0, 12:], [-1, 0])


def torch_net(params):
    return [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
            for W, b in params]


def torch_forward(tp, x):
    h = torch.tensor(x)
    for li, (W, b) in enumerate(tp):
        h = torch.nn.functional.linear(h, W, b)
        if li < len(tp) - 1:
            h = torch.relu(h)
    return h


def test_forward_and_backward_match_torch_autograd():
    params = rand_params(1)
    q = inputs.random_joint_states(64, 2)
    t = inputs.rng(3).uniform(0, 30, (64, 12))
    y, acts = M.forward(params, q, rounding=False)
    tp = torch_net(params)
    ty = torch_forward(tp, M.encode(q, rounding=False))
    assert np.allclose(y, ty.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss, dy = M.loss_and_dy(y, t, rounding=False)
    tl = torch.mean((ty - torch.tensor(t)) ** 2)
    assert abs(loss - tl.item()) < 1e-9 * max(1.0, abs(loss))
    tl.backward()
    grads = M.backward(params, acts, dy, rounding=False)
    for (dW, db), (W, b) in zip(grads, tp):
        assert np.allclose(dW, W.grad.numpy(), rtol=1e-10, atol=1e-12)
        assert np.allclose(db, b.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_backward_matches_finite_differences():
    params = rand_params(4, scale=0.3)
    q = inputs.random_joint_states(8, 5)
    t = inputs.rng(6).uniform(0, 5, (8, 12))
    y, acts = M.forward(params, q, rounding=False)
    _, dy = M.loss_and_dy(y, t, rounding=False)
    grads = M.backward(params, acts, dy, rounding=False)
    g = inputs.rng(7)
    h = 1e-6
    for li in range(4):
        for _ in range(6):
            for which in (0, 1):
                arr = params[li][which]
                idx = tuple(int(g.integers(0, s)) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = M.loss_and_dy(M.forward(params, q, rounding=False)[0], t, rounding=False)[0]
                arr[idx] = old - h
                lm = M.loss_and_dy(M.forward(params, q, rounding=False)[0], t, rounding=False)[0]
                arr[idx] = old
                num = (lp - lm) / (2 * h)
                ana = grads[li][which][idx]
                assert abs(num - ana) <= 1e-4 * max(1e-3, abs(ana)) + 1e-7, (li, which, idx)


def test_adam_matches_torch():
    g = inputs.rng(8)
    w = [g.normal(0, 1, (5, 3)), g.normal(0, 1, 4)]
    tw = [torch.tensor(a.copy(), requires_grad=True) for a in w]
    opt = torch.optim.Adam(tw, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(a) for a in w]
    v = [np.zeros_like(a) for a in w]
    for step in range(1, 6):
        grads = [g.normal(0, 1, a.shape) for a in w]
        for t_, gr in zip(tw, grads):
            t_.grad = torch.tensor(gr)
        opt.step()
        w, m, v = M.adam(w, grads, m, v, step)
        for a, t_ in zip(w, tw):
            assert np.allclose(a, t_.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_rounded_forward_close_to_exact():
    """The bf16 plan perturbs outputs by about the bf16 relative precision."""
    params = [(M.bf16(W), M.f32(b)) for W, b in rand_params(9, scale=0.1)]
    q = inputs.random_joint_states(256, 10)
    y_r, _ = M.forward(params, q, rounding=True)
    y_e, _ = M.forward(params, q, rounding=False)
    scale = np.abs(y_e).max()
    assert np.abs(y_r - y_e).max() < 0.05 * scale
    assert not np.array_equal(y_r, y_e)


def test_fallback_rule():
    pred = np.array([[10.0] * 12, [10.0] * 11 + [4.0]])
    r = np.full(12, 0.02)
    # clearance 10 * 0.01 - 0.02 = 0.08 m vs margin 0.05 + 1 voxel error
    need = M.needs_exact(pred, r, 0.01, 0.05, 1.0)
    assert need.tolist() == [False, True]
    assert M.needs_exact(pred, r, 0.01, 0.05, 2.0).tolist() == [False, True]
    assert M.needs_exact(pred, r, 0.01, 0.05, 3.5).tolist() == [True, True]


def test_fallback_rule_per_sphere_and_nan():
    pred = np.full((3, 12), 10.0)
    pred[1, 5] = 7.0          # clearance 0.07 - 0.02 = 0.05 m
    pred[2, 0] = np.nan
    r = np.full(12, 0.02)
    eps = np.zeros(12)
    # sphere 5 has clearance 0.05 m: inside margin + its bound only once
    # its bound is positive; the other spheres' bounds do not matter for it
    assert M.needs_exact(pred, r, 0.01, 0.04, eps).tolist() == [False, False, True]
    eps[5] = 1.5              # 0.05 < 0.04 + 0.015
    assert M.needs_exact(pred, r, 0.01, 0.04, eps).tolist() == [False, True, True]
    eps[:] = 0.0
    eps[3] = 5.0              # sphere 3: 0.08 < 0.04 + 0.05 in every state
    assert M.needs_exact(pred, r, 0.01, 0.04, eps).tolist() == [True, True, True]


def test_calibrate_by_hand():
    tgt = np.zeros((3, 12))
    pred = np.zeros((3, 12))
    tgt[:, 0], pred[:, 0] = [1.0, 2.0, 30.0], [1.5, 1.0, 45.0]   # row 2 above the clip: ignored
    tgt[:, 1], pred[:, 1] = [5.0, 5.0, 5.0], [9.0, 4.0, 6.0]     # largest overestimate 4
    tgt[:, 2], pred[:, 2] = [3.0, 3.0, 3.0], [1.0, 2.0, 3.0]     # only underestimates: 0
    pred[0, 3] = np.nan                                           # a NaN prediction: unbounded
    e = M.calibrate(pred, tgt, 24.0)
    assert e.dtype == np.float32
    assert e[0] == np.float32(0.5) and e[1] == 4.0 and e[2] == 0.0 and np.isinf(e[3])
    assert (e[4:] == 0.0).all()
    # without a clip the far row counts too
    assert M.calibrate(pred, tgt, 0.0)[0] == 15.0


def test_loss_with_clip_by_hand():
    y = np.zeros((1, 12))
    t = np.zeros((1, 12))
    y[0, 4], t[0, 4] = 30.0, 40.0
    loss, dy = M.loss_and_dy(y, t, rounding=False, clip=24.0)
    assert loss == 36.0 / 12 and dy[0, 4] == 1.0 and (np.delete(dy, 4) == 0).all()
    loss_nc, _ = M.loss_and_dy(y, t, rounding=False)
    assert loss_nc == 100.0 / 12
    # a clip above every target changes nothing
    assert M.loss_and_dy(y, t, rounding=False, clip=50.0)[0] == loss_nc
