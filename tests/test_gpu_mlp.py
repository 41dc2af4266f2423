"""The learned self-distance surrogate on the GPU against the CPU oracle.

Forward, backward and Adam are compared with oracle/mlp_ref.py under the
same bf16 precision plan; the device accumulates in float32 (the oracle in
float64), so a bf16 result may differ by one unit in the last place where
the float32 sum lands near a rounding boundary, and float32 results by
float32 rounding.  Tolerances below follow from that.  The labels come from
the exact self-map EDT and must match the oracle's transform bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from paper_2407_02363_amd import inputs, mlp
from paper_2407_02363_amd.surrogate import Surrogate
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu


def ws_views(ws, batch):
    """Activations saved by sdf_mlp_forward, at the library's workspace
    offsets (256-byte aligned regions in the documented order)."""
    P = (batch + 63) // 64 * 64
    sizes = [("x", P * 32 * 2), ("h1", P * 256 * 2), ("h2", P * 256 * 2), ("h3", P * 256 * 2),
             ("y", P * 32 * 4)]
    out, off = {}, 0
    raw = ws.cpu().numpy()
    for name, nbytes in sizes:
        buf = raw[off:off + nbytes]
        if name == "y":
            out[name] = buf.view(np.float32).reshape(P, 32).astype(np.float64)
        else:
            cols = 32 if name == "x" else 256
            out[name] = (buf.view(np.uint16).astype(np.uint32) << 16).view(np.float32).reshape(P, cols).astype(np.float64)
        off += (nbytes + 255) // 256 * 256
    return out


def device_params(s: Surrogate):
    """The parameters as the kernels see them: bf16 weights, f32 biases."""
    w16 = s.w16.float().cpu().numpy().astype(np.float64)
    master = s.master.cpu().numpy()
    out = []
    for (wo, bo, rows, cols), (ro, ci) in zip(mlp.LAYOUT, mlp.REAL):
        W = w16[wo:wo + rows * cols].reshape(rows, cols)[:ro, :ci]
        out.append((W, master[bo:bo + ro].astype(np.float64)))
    return out


def perturbed_surrogate(seed):
    s = Surrogate(dev(), seed=seed, batch=512)
    g = inputs.rng(seed + 100)
    p = s.master.cpu().numpy()
    for _, bo, rows, _ in mlp.LAYOUT:
        p[bo:bo + rows] = g.normal(0, 0.1, rows)
    # keep the padded output rows at zero
    p[mlp.B4 + 12:mlp.B4 + 32] = 0
    s.master.copy_(torch.from_numpy(p))
    mlp.sdf_mlp_pack(s.master, s.w16)
    return s


def test_pack_is_round_to_nearest_even():
    s = Surrogate(dev(), seed=1, batch=64)
    torch.cuda.synchronize()
    ref = M.bf16(s.master.cpu().numpy().astype(np.float64))
    assert np.array_equal(s.w16.float().cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("batch", [1, 300, 512])
def test_forward_matches_oracle(batch):
    s = perturbed_surrogate(2)
    q_np = inputs.random_joint_states(batch, 3).astype(np.float32)
    q = torch.from_numpy(q_np).to(dev())
    y = torch.empty((batch, 12), dtype=torch.float32, device=dev())
    say(f"[mlp] forward batch={batch}")
    mlp.sdf_mlp_forward(s.w16, s.master, q, y, s.ws)
    torch.cuda.synchronize()
    params = device_params(s)
    acts = ws_views(s.ws, batch)
    # inputs: bf16(sin / cos); the device's sinf may sit one bf16 step away
    # from the float64 value only at rounding boundaries
    x_ref = M.encode(q_np.astype(np.float64))
    assert np.mean(acts["x"][:batch, :14] == x_ref) > 0.999
    assert np.abs(acts["x"][:batch, :14] - x_ref).max() <= 2 ** -8
    assert (acts["x"][:batch, 14:] == 0).all()
    # every layer from the device's own inputs: bf16 outputs equal the
    # oracle's or are one bf16 step away
    ins = [acts["x"][:batch, :14], acts["h1"][:batch], acts["h2"][:batch], acts["h3"][:batch]]
    outs = [acts["h1"][:batch], acts["h2"][:batch], acts["h3"][:batch], acts["y"][:batch, :12]]
    for li, (W, b) in enumerate(params):
        z = M.f32(ins[li] @ W.T + b)
        # float32 summation of n products: error <= (n + 2) 2^-24 sum |terms|
        acc = (np.abs(ins[li]) @ np.abs(W).T + np.abs(b)) * (W.shape[1] + 2) * 2.0 ** -24
        got = outs[li]
        if li < 3:
            ref = M.bf16(np.maximum(z, 0))
            # plus one bf16 step of the result when the sums straddle a boundary
            allowed = 2.0 ** -7 * np.maximum(np.abs(ref), np.abs(got)) + 2 * acc
            assert (np.abs(got - ref) <= allowed).all(), (li, np.abs(got - ref).max())
            assert np.mean(got == ref) > 0.995, li
        else:
            assert (np.abs(got - z) <= 2 * acc + 1e-30).all(), (li, np.abs(got - z).max())
    assert np.array_equal(y.cpu().numpy(), acts["y"][:batch, :12].astype(np.float32))
    # end to end from q: small relative to the output scale
    y_ref, _ = M.forward(params, q_np.astype(np.float64))
    scale = np.abs(y_ref).max() + 1e-6
    assert np.abs(y.cpu().numpy() - y_ref).max() < 0.02 * scale


def test_backward_matches_oracle():
    batch = 320
    s = perturbed_surrogate(4)
    q_np = inputs.random_joint_states(batch, 5).astype(np.float32)
    t_np = inputs.rng(6).uniform(0, 20, (batch, 12)).astype(np.float32)
    q = torch.from_numpy(q_np).to(dev())
    t = torch.from_numpy(t_np).to(dev())
    y = torch.empty((batch, 12), dtype=torch.float32, device=dev())
    mlp.sdf_mlp_forward(s.w16, s.master, q, y, s.ws)
    mlp.sdf_mlp_backward(s.w16, t, s.grad, s.loss, s.ws)
    torch.cuda.synchronize()
    say("[mlp] backward")
    params = device_params(s)
    acts = ws_views(s.ws, batch)
    a = [acts["x"][:batch, :14], acts["h1"][:batch], acts["h2"][:batch], acts["h3"][:batch]]
    yd = y.cpu().numpy().astype(np.float64)
    loss, dy = M.loss_and_dy(yd, t_np.astype(np.float64))
    assert abs(float(s.loss.item()) - loss) <= 1e-5 * loss
    grads = M.backward(params, a, dy)
    g = s.grad.cpu().numpy()
    for li, ((wo, bo, rows, cols), (ro, ci)) in enumerate(zip(mlp.LAYOUT, mlp.REAL)):
        dW = g[wo:wo + rows * cols].reshape(rows, cols)
        db = g[bo:bo + rows]
        rdW, rdb = grads[li]
        # padding gradients are exactly zero
        assert (dW[ro:, :] == 0).all() and (dW[:, ci:] == 0).all() and (db[ro:] == 0).all()
        err = np.abs(dW[:ro, :ci] - rdW).max()
        assert err <= 2e-3 * np.abs(rdW).max() + 1e-7, (li, err, np.abs(rdW).max())
        assert np.abs(db[:ro] - rdb).max() <= 2e-3 * np.abs(rdb).max() + 1e-7, li
    # same inputs, same bits: the reductions have a fixed order
    g1 = s.grad.clone()
    mlp.sdf_mlp_forward(s.w16, s.master, q, y, s.ws)
    mlp.sdf_mlp_backward(s.w16, t, s.grad, s.loss, s.ws)
    torch.cuda.synchronize()
    assert torch.equal(g1, s.grad)


def test_adam_matches_oracle():
    s = Surrogate(dev(), seed=7, batch=64)
    g = inputs.rng(8)
    w = s.master.cpu().numpy().astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in range(1, 4):
        gr = g.normal(0, 1, w.shape).astype(np.float32)
        s.grad.copy_(torch.from_numpy(gr))
        mlp.sdf_mlp_adam(s.master, s.w16, s.m, s.v, s.grad, step, 1e-3)
        (w,), (m,), (v,) = M.adam([w], [gr.astype(np.float64)], [m], [v], step)
    torch.cuda.synchronize()
    got = s.master.cpu().numpy().astype(np.float64)
    assert np.abs(got - w).max() < 1e-6
    assert np.array_equal(s.w16.float().cpu().numpy().astype(np.float64), M.bf16(got))


def test_fallback_kernel_matches_rule():
    """The kernel's yes/no per state equals the oracle's rule evaluated in
    the same float32 order, for per-sphere bounds, including NaN rows."""
    g = inputs.rng(9)
    n = 5000
    y_np = g.uniform(0, 25, (n, 12)).astype(np.float32)
    y_np[17, 3] = np.nan
    radii = g.uniform(0.02, 0.05, 12).astype(np.float32)
    eps = g.uniform(0.0, 3.0, 12).astype(np.float32)
    voxel, margin = 0.01, 0.05
    s = Surrogate(dev(), seed=0, batch=64)
    need, count = s.fallback(torch.from_numpy(y_np).to(dev()), torch.from_numpy(radii).to(dev()),
                             voxel, margin, torch.from_numpy(eps).to(dev()))
    torch.cuda.synchronize()
    ref = M.needs_exact(y_np, radii, voxel, margin, eps)
    got = need.cpu().numpy().astype(bool)
    assert np.array_equal(got, ref) and got[17]
    assert 0 < got.sum() < n and int(count.item()) == int(got.sum())


def test_calibrate_matches_oracle():
    g = inputs.rng(10)
    n = 3000
    t_np = g.uniform(0, 40, (n, 12)).astype(np.float32)
    p_np = (t_np + g.normal(0, 1.5, (n, 12))).astype(np.float32)
    p_np[5, 7] = np.nan
    t = torch.from_numpy(t_np).to(dev())
    p = torch.from_numpy(p_np).to(dev())
    eps = torch.full((12,), -1.0, dtype=torch.float32, device=dev())
    for clip in (24.0, 0.0):
        mlp.sdf_mlp_calibrate(p, t, clip, eps)
        torch.cuda.synchronize()
        ref = M.calibrate(p_np, t_np, clip)
        assert np.array_equal(eps.cpu().numpy(), ref), clip
        assert np.isinf(ref[7]) and (ref[np.arange(12) != 7] > 0).all()


def test_gather_and_clip_match_plain():
    """A minibatch named by row indices, with clipped targets, gives the same
    bits as the gathered rows and pre-clipped targets passed directly."""
    rows, batch, clip = 1000, 448, 12.0
    s = perturbed_surrogate(14)
    q_np = inputs.random_joint_states(rows, 15).astype(np.float32)
    t_np = inputs.rng(16).uniform(0, 20, (rows, 12)).astype(np.float32)
    idx_np = inputs.rng(17).permutation(rows)[:batch].astype(np.int32)
    q, t = torch.from_numpy(q_np).to(dev()), torch.from_numpy(t_np).to(dev())
    idx = torch.from_numpy(idx_np).to(dev())
    y1 = torch.empty((batch, 12), dtype=torch.float32, device=dev())
    mlp.sdf_mlp_forward(s.w16, s.master, q, y1, s.ws, idx=idx)
    mlp.sdf_mlp_backward(s.w16, t, s.grad, s.loss, s.ws, idx=idx, clip_vox=clip)
    torch.cuda.synchronize()
    g1, l1 = s.grad.clone(), s.loss.clone()
    qg = torch.from_numpy(q_np[idx_np]).to(dev())
    tg = torch.from_numpy(np.minimum(t_np[idx_np], np.float32(clip))).to(dev())
    y2 = torch.empty((batch, 12), dtype=torch.float32, device=dev())
    mlp.sdf_mlp_forward(s.w16, s.master, qg, y2, s.ws)
    mlp.sdf_mlp_backward(s.w16, tg, s.grad, s.loss, s.ws)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(g1, s.grad) and torch.equal(l1, s.loss)
    # an index outside q poisons only its own row
    bad = idx.clone()
    bad[3] = rows
    mlp.sdf_mlp_forward(s.w16, s.master, q, y1, s.ws, idx=bad)
    torch.cuda.synchronize()
    yb = y1.cpu().numpy()
    assert np.isnan(yb[3]).all() and np.array_equal(np.delete(yb, 3, 0), np.delete(y2.cpu().numpy(), 3, 0))


@pytest.mark.parametrize("edt_mode", ["many", "batched"])
def test_labeler_matches_oracle(oracle_lib, edt_mode):
    from paper_2407_02363_amd.selfmap import SelfMapLabeler
    st = inputs.self_map_setup()
    lab = SelfMapLabeler(st, chunk=8, device=dev(), edt_mode=edt_mode)
    qs = inputs.random_joint_states(13, 11)   # one full chunk and a partial one
    say("[mlp] labels")
    got = lab.labels(qs).cpu().numpy()
    g = st.grid
    for k, q in enumerate(qs):
        occ = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_links(g, occ, st.link_pts, st.link_off, st.robot.poses12(q), st.mask)
        d2, site = oracle_lib.edt(occ)
        c = inputs.sphere_centres(st.robot, q, st.sphere_links, st.sphere_local)
        ref = oracle_lib.query_spheres(g, d2, site, c, st.sphere_radii).view(np.float32)[:, 6]
        assert np.array_equal(got[k], ref), k


def test_training_is_deterministic_and_learns():
    from paper_2407_02363_amd.selfmap import SelfMapLabeler
    st = inputs.self_map_setup()
    lab = SelfMapLabeler(st, chunk=48, device=dev())
    qs = inputs.random_joint_states(4096 * 2, 12)
    y = lab.labels(qs)
    q = torch.from_numpy(qs.astype(np.float32)).to(dev())
    runs = []
    for rep in range(2):
        s = Surrogate(dev(), seed=13, batch=4096)
        hist = s.train(q, y, epochs=12, lr=2e-3, seed=1)
        say(f"[mlp] run {rep} loss {hist[0]:.3f} -> {hist[-1]:.3f}")
        runs.append((hist, s.master.clone()))
    assert runs[0][0] == runs[1][0] and torch.equal(runs[0][1], runs[1][1])
    assert runs[0][0][-1] < 0.2 * runs[0][0][0]


def test_surrogate_gain_with_zero_misses():
    """Trained on exact-EDT labels, with its error bound calibrated per sphere
    on held-out states, the surrogate plus fallback rule never calls a state
    safe that the exact transform puts inside the margin, and skips the exact
    transform for a real share of the look-ahead states."""
    from paper_2407_02363_amd.selfmap import SelfMapLabeler
    st = inputs.self_map_setup()
    lab = SelfMapLabeler(st, chunk=48, device=dev())
    q_tr = inputs.random_joint_states(131072, 21)
    q_va = inputs.random_joint_states(16384, 22)
    q_te = inputs.random_joint_states(16384, 23)
    say("[mlp] labelling 164k states")
    y_tr, y_va, y_te = lab.labels(q_tr), lab.labels(q_va), lab.labels(q_te)
    s = Surrogate(dev(), seed=3, batch=4096, clip_vox=24.0)
    margin = 0.05
    # a sphere inside the margin has an exact distance below the clip, so the
    # calibration rows cover it
    assert (margin + st.sphere_radii.max()) / st.grid.voxel < s.clip_vox
    t = lambda a: torch.from_numpy(a.astype(np.float32)).to(dev())
    hist = s.train(t(q_tr), y_tr, epochs=40, lr=2e-3, seed=2, lr_final=2e-5)
    eps = s.calibrate(t(q_va), y_va).cpu().numpy()
    assert np.isfinite(eps).all() and (eps > 0).all(), eps
    p_te = s.predict(t(q_te))
    radii = torch.from_numpy(st.sphere_radii).to(dev())
    need, count = s.fallback(p_te, radii, st.grid.voxel, margin)
    torch.cuda.synchronize()
    need = need.cpu().numpy().astype(bool)
    exact_clear = y_te.cpu().numpy().astype(np.float64) * st.grid.voxel - st.sphere_radii[None, :]
    truly_near = (exact_clear < margin).any(1)
    misses = int((truly_near & ~need).sum())
    skipped = 1.0 - need.mean()
    say(f"[mlp] loss {hist[0]:.2f}->{hist[-1]:.3f}, eps {np.round(eps, 2)} vox, "
        f"fallback {need.mean():.3f}, truly near {truly_near.mean():.3f}, misses {misses}")
    assert misses == 0
    assert skipped > 0.15


def test_select_keeps_bits():
    """sdf_mlp_select copies the exact record word of every flagged state and
    the prediction of every other state, bit for bit, reading the records in
    place through their strides (and in place over y)."""
    g = inputs.rng(30)
    b = 37
    y_np = g.normal(0, 10, (b, 12)).astype(np.float32)
    rec_np = g.integers(-2**31, 2**31 - 1, (b, 12, 16), dtype=np.int64).astype(np.int32)
    need_np = (g.random(b) < 0.5).astype(np.int32) * g.integers(1, 9, b).astype(np.int32)
    y = torch.from_numpy(y_np).to(dev())
    rec = torch.from_numpy(rec_np).to(dev())
    need = torch.from_numpy(need_np).to(dev())
    out = torch.full((b, 12), -1.0, dtype=torch.float32, device=dev())
    exact = rec[:, :, 6].view(torch.float32)
    mlp.sdf_mlp_select(y, need, exact, out)
    torch.cuda.synchronize()
    ref = np.where(need_np[:, None] != 0, rec_np[:, :, 6], y_np.view(np.int32))
    assert np.array_equal(out.cpu().numpy().view(np.int32), ref)
    mlp.sdf_mlp_select(y, need, exact, y)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().view(np.int32), ref)
    assert 0 < (need_np != 0).sum() < b


def test_assisted_lookahead_graph(oracle_lib):
    """The look-ahead batch with no host round trip (one graph: forward,
    fallback flags, gated exact transform, select): the flags follow the
    oracle's rule on the predictions, every flagged state gets the oracle's
    exact distances, every other state its prediction, over several
    replays whose flags differ (so switched-off slots hold stale maps)."""
    from paper_2407_02363_amd.selfmap import SelfMapLabeler
    from paper_2407_02363_amd.surrogate import AssistedLookahead
    st = inputs.self_map_setup()
    g = st.grid
    S, chunks = 16, 3
    sur = perturbed_surrogate(31)
    sur.eps.fill_(0.5)
    radii = torch.from_numpy(st.sphere_radii).to(dev())
    lab = SelfMapLabeler(st, chunk=S, device=dev(), use_graph=False)
    qs = inputs.random_joint_states(chunks * S, 32)
    poses, cen = lab.stage(qs)
    q = torch.from_numpy(qs.astype(np.float32)).to(dev())
    ws = mlp.new_workspace(S, dev())
    preds = []
    for k in range(chunks):
        y = torch.empty((S, 12), dtype=torch.float32, device=dev())
        mlp.sdf_mlp_forward(sur.w16, sur.master, q[k * S:(k + 1) * S], y, ws)
        preds.append(y.cpu().numpy())
    pred = np.concatenate(preds)
    eps_np = sur.eps.cpu().numpy()
    slack = (pred.astype(np.float64) * g.voxel - st.sphere_radii[None] - eps_np[None] * g.voxel).min(1)
    margin = float(np.median(slack))
    assist = AssistedLookahead(sur, lab, radii, g.voxel, margin)
    flagged = 0
    for k in range(chunks):
        sl = slice(k * S, (k + 1) * S)
        say(f"[assisted] chunk {k}")
        out = assist.run(q[sl], poses[sl], cen[sl]).cpu().numpy()
        need = assist.need.cpu().numpy().astype(bool)
        ref_need = M.needs_exact(pred[sl], st.sphere_radii, g.voxel, margin, eps_np)
        assert np.array_equal(need, ref_need), k
        assert np.array_equal(out[~need].view(np.int32), pred[sl][~need].view(np.int32)), k
        for j in np.flatnonzero(need):
            qj = qs[k * S + j]
            occ = np.zeros(g.shape, np.uint8)
            oracle_lib.insert_links(g, occ, st.link_pts, st.link_off, st.robot.poses12(qj), st.mask)
            d2, site = oracle_lib.edt(occ)
            c = inputs.sphere_centres(st.robot, qj, st.sphere_links, st.sphere_local)
            ref = oracle_lib.query_spheres(g, d2, site, c, st.sphere_radii).view(np.float32)[:, 6]
            assert np.array_equal(out[j].view(np.int32), ref.view(np.int32)), (k, j)
        flagged += int(need.sum())
    assert 0 < flagged < chunks * S


@pytest.mark.parametrize("batch", [1, 16, 100, 4096])
def test_infer_equals_forward(batch):
    """The one-launch inference kernel gives the forward pass's predictions
    bit for bit (same products in the same order, same epilogues), NaN rows
    included."""
    s = perturbed_surrogate(40)
    q_np = inputs.random_joint_states(batch, 41).astype(np.float32)
    if batch > 3:
        q_np[3, 2] = np.nan
    q = torch.from_numpy(q_np).to(dev())
    ws = mlp.new_workspace(batch, dev())
    y_fwd = torch.empty((batch, 12), dtype=torch.float32, device=dev())
    y_inf = torch.full((batch, 12), -1.0, dtype=torch.float32, device=dev())
    mlp.sdf_mlp_forward(s.w16, s.master, q, y_fwd, ws)
    mlp.sdf_mlp_infer(s.w16, s.master, q, y_inf)
    torch.cuda.synchronize()
    a, b = y_fwd.cpu().numpy(), y_inf.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    if batch > 3:
        assert np.isnan(b[3]).all() and not np.isnan(np.delete(b, 3, 0)).any()
    # the fused fallback rule decides as sdf_mlp_fallback does on the same y
    r_np = inputs.rng(42).uniform(0.02, 0.05, 12).astype(np.float32)
    e_np = inputs.rng(43).uniform(0.0, 3.0, 12).astype(np.float32)
    radii, eps = torch.from_numpy(r_np).to(dev()), torch.from_numpy(e_np).to(dev())
    # a margin that leaves about half of the states on each side of the rule
    fin = a[np.isfinite(a).all(1)].astype(np.float64)
    margin = float(np.median((fin * 0.01 - r_np - e_np * 0.01).min(1)))
    need_f = torch.full((batch,), 7, dtype=torch.int32, device=dev())
    count = torch.zeros(1, dtype=torch.int32, device=dev())
    need_i = torch.full((batch,), 7, dtype=torch.int32, device=dev())
    mlp.sdf_mlp_fallback(y_fwd, radii, eps, 0.01, margin, need_f, count)
    mlp.sdf_mlp_infer(s.w16, s.master, q, y_inf, radii, eps, 0.01, margin, need_i)
    torch.cuda.synchronize()
    assert torch.equal(need_f, need_i)
    assert np.array_equal(y_inf.cpu().numpy().view(np.uint32), a.view(np.uint32))
    n_need = int(need_i.sum().item())
    assert int(count.item()) == n_need and (batch < 16 or 0 < n_need < batch)
