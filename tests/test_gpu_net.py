"""Proposal network on the GPU against the FP64 net oracle.

Tolerances follow from the device arithmetic: the trunk stores activations,
weights and the back-propagated ReLU-masked gradients in bfloat16 (the oracle
rounds at the same points with bf16_trunk=True), every sum accumulates in
FP32.  Left over are FP32-vs-FP64 accumulation differences (relative ~1e-6)
and, where such a difference moves a value across a bfloat16 rounding
boundary, one bfloat16 unit (2^-8 relative) on a small fraction of the
elements.  Parameter gradients are sums of many same-signed-magnitude
terms and are compared norm-relative to 3e-3.  The input gradient is a sum
of 576 terms of both signs per element that largely cancel, so a one-unit
difference of the rounded masked gradient G0 shows up relative to the size
of the terms, not of the sum: it is bounded elementwise by 2^-6 (four
bfloat16 units, for the flips and the upstream differences) times the same
sum taken over absolute values, sum |W0| |G0|.  Outputs rounded to bfloat16
by the kernel itself are compared to 2^-8 relative.
"""

import numpy as np
import pytest

from oracle import net as onet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def pn(torch):
    import paper_2503_20875_amd as cm
    from paper_2503_20875_amd import proposal
    cm._abi.load()
    return proposal


def bf16_exact(rng, shape, lo=-1.0, hi=1.0):
    return onet.bf16(rng.uniform(lo, hi, shape))


def to_dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").to(dtype)


def rel_norm(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def test_mfma_probe_layout(torch, pn):
    """One MFMA on small integers (exact in FP32) equals A @ B."""
    rng = np.random.default_rng(1)
    A = rng.integers(-8, 9, (16, 32)).astype(np.float64)
    B = rng.integers(-8, 9, (32, 16)).astype(np.float64)
    print("[net] mfma probe", flush=True)
    C = pn.mfma_probe(to_dev(torch, A, torch.bfloat16), to_dev(torch, B, torch.bfloat16))
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.float64), A @ B)


def packed_w(W):
    """[64][cin][9] -> [64][k32] with k = tap * cin + ci (the test's own
    restatement of the documented layout)."""
    o, cin, taps = W.shape
    k32 = (taps * cin + 31) // 32 * 32
    out = np.zeros((o, k32))
    out[:, :taps * cin] = W.transpose(0, 2, 1).reshape(o, taps * cin)
    return out


@pytest.mark.parametrize("cin,L,B", [(16, 300, 2), (64, 131, 3), (16, 1, 1), (64, 64, 1), (64, 1100, 2), (16, 1029, 1)])
def test_conv_forward(torch, pn, cin, L, B):
    rng = np.random.default_rng(cin + L)
    x = bf16_exact(rng, (B, cin, L), 0.0, 1.0)
    W = onet.bf16(rng.normal(0, np.sqrt(2.0 / (9 * cin)), (64, cin, 9)))
    b = rng.normal(0, 0.1, 64).astype(np.float32).astype(np.float64)
    ref = np.maximum(onet.conv1d(x, W, b), 0.0).transpose(0, 2, 1)  # [B][L][64]
    print(f"[net] conv fwd cin={cin} L={L} B={B}", flush=True)
    y = pn.conv1d_fwd(to_dev(torch, x.transpose(0, 2, 1), torch.bfloat16), to_dev(torch, packed_w(W), torch.bfloat16),
                      to_dev(torch, b, torch.float32))
    torch.cuda.synchronize()
    got = y.float().cpu().numpy().astype(np.float64)
    scale = max(np.abs(ref).max(), 1e-30)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * scale)


@pytest.mark.parametrize("cin,L,B", [(16, 300, 2), (64, 517, 2), (64, 5, 1), (64, 1100, 1), (16, 1029, 2)])
def test_conv_backward(torch, pn, cin, L, B):
    rng = np.random.default_rng(7 * cin + L)
    x = bf16_exact(rng, (B, cin, L), 0.0, 1.0)
    W = onet.bf16(rng.normal(0, np.sqrt(2.0 / (9 * cin)), (64, cin, 9)))
    b = rng.normal(0, 0.1, 64)
    y = onet.bf16(np.maximum(onet.conv1d(x, W, b), 0.0))  # post-ReLU output as the device stores it
    dy = bf16_exact(rng, (B, 64, L))
    G = dy * (y > 0)
    gx, gW, gb = onet.conv1d_backward(x, W, G)
    print(f"[net] conv bwd cin={cin} L={L} B={B}", flush=True)
    dx, dw, db = pn.conv1d_bwd(to_dev(torch, dy.transpose(0, 2, 1), torch.float32),
                               to_dev(torch, y.transpose(0, 2, 1), torch.bfloat16),
                               to_dev(torch, x.transpose(0, 2, 1), torch.bfloat16),
                               to_dev(torch, packed_w(W), torch.bfloat16))
    torch.cuda.synchronize()
    k32 = (9 * cin + 31) // 32 * 32
    dw = dw.cpu().numpy().astype(np.float64)
    assert np.all(dw[:, 9 * cin:] == 0.0) and dw.shape == (64, k32)
    dw = dw[:, :9 * cin].reshape(64, 9, cin).transpose(0, 2, 1)
    for got, ref in ((dx.cpu().numpy().transpose(0, 2, 1), gx), (dw, gW), (db.cpu().numpy(), gb)):
        scale = max(np.abs(ref).max(), 1e-30)
        assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref) + 1e-5 * scale)


def test_conv_backward_partial_sums_at_training_size(torch, pn):
    """The weight gradient through the partial-sum workspace, where several
    256-position chunks share a workgroup (cin 16, 32 x 4 096 positions: two
    chunks per workgroup), against the oracle and against the atomic path;
    two calls give the same bits."""
    cin, L, B = 16, 4096, 32
    assert pn.bwd_partial_floats(cin, L, B) == (L // 512) * B * (64 * 160 + 64)
    rng = np.random.default_rng(4096)
    x = bf16_exact(rng, (B, cin, L), 0.0, 1.0)
    W = onet.bf16(rng.normal(0, np.sqrt(2.0 / (9 * cin)), (64, cin, 9)))
    y = onet.bf16(np.maximum(onet.conv1d(x, W, rng.normal(0, 0.1, 64)), 0.0))
    dy = bf16_exact(rng, (B, 64, L))
    _, gW, gb = onet.conv1d_backward(x, W, dy * (y > 0))
    print(f"[net] conv bwd partial sums cin={cin} L={L} B={B}", flush=True)
    args = (to_dev(torch, dy.transpose(0, 2, 1), torch.float32), to_dev(torch, y.transpose(0, 2, 1), torch.bfloat16),
            to_dev(torch, x.transpose(0, 2, 1), torch.bfloat16), to_dev(torch, packed_w(W), torch.bfloat16))
    _, dw1, db1 = pn.conv1d_bwd(*args, dx_out=False)
    _, dw2, db2 = pn.conv1d_bwd(*args, dx_out=False)
    _, dwa, dba = pn.conv1d_bwd(*args, partial=False, dx_out=False)
    torch.cuda.synchronize()
    assert torch.equal(dw1, dw2) and torch.equal(db1, db2)
    got_w = dw1.cpu().numpy().astype(np.float64)
    assert np.all(got_w[:, 9 * cin:] == 0.0)
    got_w = got_w[:, :9 * cin].reshape(64, 9, cin).transpose(0, 2, 1)
    got_a = dwa.cpu().numpy().astype(np.float64)[:, :9 * cin].reshape(64, 9, cin).transpose(0, 2, 1)
    for got, ref in ((got_w, gW), (got_a, gW), (db1.cpu().numpy(), gb), (dba.cpu().numpy(), gb)):
        scale = max(np.abs(ref).max(), 1e-30)
        assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref) + 1e-5 * scale)


def test_conv_backward_rejects_a_short_workspace(torch, pn):
    from paper_2503_20875_amd import _abi
    cin, L, B = 64, 512, 2
    need = pn.bwd_partial_floats(cin, L, B)
    t = lambda *shape, dt=torch.bfloat16: torch.zeros(shape, dtype=dt, device="cuda")  # noqa: E731
    dy, y, x, w = t(B, L, 64, dt=torch.float32), t(B, L, 64), t(B, L, cin), t(64, 576)
    g, wt, part = t(B, L, 64), t(64 * 9 * cin), t(need - 4, dt=torch.float32)
    dw, db = t(64, 576, dt=torch.float32), t(64, dt=torch.float32)
    rc = _abi.load().cetra_conv1d_bwd(None, dy.data_ptr(), y.data_ptr(), x.data_ptr(), cin, L, B, w.data_ptr(), 576,
                                      g.data_ptr(), wt.data_ptr(), part.data_ptr(), need - 4, None, dw.data_ptr(),
                                      db.data_ptr())
    assert rc != 0


def net_case(seed=0, B=2, L=700, n_win=16):
    """Parameters (FP32-exact), a bfloat16-exact input, log windows over
    0.1-5 d on 0.02-d bins and one positive window per example."""
    rng = np.random.default_rng(seed)
    p = onet.init_params(c_in=16, width=64, n_layers=5, n_event=8, hidden=64, seed=seed)
    for k in p:
        if k.startswith("b") or k in ("p", "u"):
            p[k] = rng.normal(0, 0.05, p[k].shape)
    for k in p:  # FP32-exact parameters (the device masters are FP32)
        p[k] = p[k].astype(np.float32).astype(np.float64)
    x = bf16_exact(rng, (B, 16, L), 0.0, 1.0)
    q, edges = onet.windows_for(n_win, 0.1, 5.0)
    q = q.astype(np.float32).astype(np.float64)
    y = np.zeros((B, n_win))
    for b in range(B):
        y[b, rng.integers(n_win)] = 1.0
    return p, x, q, edges, y


@pytest.mark.parametrize("seed", [0, 4])
def test_network_forward_backward(torch, pn, seed):
    """The whole network (trunk, projection, fold pooling at 4 trial periods
    per window, head, loss) forward and backward against the oracle."""
    p, x, q, edges, y = net_case(seed)
    win = pn.Windows.log_spaced(len(q), 0.1, 5.0, 0.02)
    assert np.allclose(win.edges, edges, rtol=1e-15) and np.allclose(win.q, q)
    trials = win.trials(4)
    assert np.allclose(trials, onet.fold_trials(edges, 4, 0.02), rtol=1e-15, atol=0)
    z_ref, cache = onet.forward(p, x, q, trials, keep=True, bf16_trunk=True)
    # the backward follows each window's winning phase: the case is usable
    # only if every winner beats the runner-up by far more than the FP32
    # summation error of the device, so both sides pick the same phase
    g1, _, g2 = onet.fold_pool(cache["e"], trials, runner_up=True)
    assert np.all(g1 - g2 > 1e-4 * np.maximum(np.abs(g1), 1.0)), "test case has near-tied fold maxima"
    loss_ref, gz = onet.bce_loss(z_ref, y, pos_weight=4.0)
    g_ref = onet.backward(p, cache, gz)
    model = pn.ProposalNet(n_event=8, hidden=64, n_trial=4)
    model.load_arrays(p)
    print(f"[net] forward/backward seed={seed} B={x.shape[0]} L={x.shape[2]} W={len(q)}", flush=True)
    z = model.forward(to_dev(torch, x.transpose(0, 2, 1), torch.bfloat16), win)
    loss, dx = model.backward(to_dev(torch, y, torch.float32), pos_weight=4.0, want_dx=True)
    torch.cuda.synchronize()
    assert np.all(np.abs(z.cpu().numpy() - z_ref) <= 3e-3 * max(1.0, np.abs(z_ref).max()))
    assert abs(float(loss.item()) - loss_ref) <= 3e-3 * abs(loss_ref)
    g = model.grad_arrays()
    for name, ref in g_ref.items():
        if name == "x":
            continue
        assert rel_norm(g[name], ref) < 3e-3, (name, rel_norm(g[name], ref))
    gx = dx.cpu().numpy().transpose(0, 2, 1).astype(np.float64)
    mag = onet.conv1d_backward(x, np.abs(onet.bf16(p["W0"])), np.abs(cache["G0"]))[0]
    assert np.all(np.abs(gx - g_ref["x"]) <= 2.0 ** -6 * mag + 1e-12), \
        float(np.max(np.abs(gx - g_ref["x"]) / (mag + 1e-30)))


def _winner_score32(e, trials, arg_ref, b, w, c):
    """FP32 score of the oracle's winning (trial, phase): the exact sum of
    the integer-valued events at its transit positions, and its count."""
    s_, ph = arg_ref[b, w, c]
    L = e.shape[2]
    R = onet.fold_step(trials[w, s_])
    pos = []
    k = 0
    while ph + ((k * R + 2 ** 31) >> 32) < L:
        pos.append(ph + ((k * R + 2 ** 31) >> 32))
        k += 1
    return onet.score32(e[b, c, pos].sum(), len(pos))


def _check_fold_pool(torch, pn, e, trials, q):
    B, E, L = e.shape
    W, S = trials.shape
    g_ref, arg_ref = onet.fold_pool(e, trials)
    win = pn.Windows(q, np.arange(W + 1, dtype=np.float64) + 1.0, 1.0)
    setattr(win, f"_trials{S}", torch.as_tensor(trials, device="cuda"))
    model_e = torch.as_tensor(e.transpose(0, 2, 1).copy(), dtype=torch.float32, device="cuda")
    print(f"[foldpool] B={B} E={E} L={L} W={W} S={S}", flush=True)
    f, arg = pn.foldpool_fwd(model_e, win, S)
    f, arg = f.cpu().numpy(), arg.cpu().numpy()
    for b in range(B):
        for w in range(W):
            for c in range(E):
                s_, ph = arg_ref[b, w, c]
                assert arg[b, w, c] == (-1 if s_ < 0 else s_ * 65536 + ph), (b, w, c, arg[b, w, c], s_, ph)
                want = np.float32(0.0) if s_ < 0 else _winner_score32(e, trials, arg_ref, b, w, c)
                assert f[b, w, c] == want, (b, w, c, f[b, w, c], want)
                assert abs(f[b, w, c] - g_ref[b, w, c]) <= 2.0 ** -22 * abs(g_ref[b, w, c])
            assert f[b, w, E] == q[w]
    return f, arg, arg_ref, win


def test_fold_pool_kernels(torch, pn):
    """Fold pooling alone on integer-valued events (sums exact in FP32 and
    FP64, so every argmax decision is the oracle's): argmax bit for bit and
    the feature equal to the FP32 score of the oracle's winner, the backward
    to FP32 summation order; trials shorter than one bin are skipped and a
    window without a valid trial gives zero.  Trials of more than 64 phases
    take two phases per lane, with full and tail transits."""
    rng = np.random.default_rng(21)
    B, E, L, W, S = 2, 3, 300, 6, 3
    e = rng.integers(-3, 4, (B, E, L)).astype(np.float64)
    trials = np.array([[5.3, 5.6, 5.9], [17.2, 17.9, 18.3], [40.0, 41.5, 43.0], [0.5, 60.2, 61.7],
                       [149.5, 151.0, 152.5], [0.2, 0.6, 0.9]])
    q = np.linspace(0.05, 0.95, W).astype(np.float32)
    f, arg, arg_ref, win = _check_fold_pool(torch, pn, e, trials, q)
    assert np.all(f[:, 5, :E] == 0) and np.all(arg[:, 5] == -1)
    gg = rng.normal(size=(B, W, E + 1)).astype(np.float32)
    ge = pn.foldpool_bwd(torch.as_tensor(gg, device="cuda"), torch.as_tensor(arg, device="cuda"), win, E, L, S)
    ref = onet.fold_pool_backward(gg[:, :, :E].astype(np.float64), arg_ref, trials, L)
    assert np.allclose(ge.cpu().numpy().transpose(0, 2, 1), ref, rtol=1e-5, atol=1e-6)


def test_fold_pool_full_length(torch, pn):
    """The network's series length, 8 192 bins: trials from one bin to past
    the series (one transit per phase) and a huge trial (the fixed-point
    step near its 2^62 limit), each window's groups of 64 or 128 phases
    with their full and tail transits, bit for bit against the oracle."""
    rng = np.random.default_rng(22)
    B, E, L = 1, 2, 8192
    e = rng.integers(-4, 5, (B, E, L)).astype(np.float64)
    trials = np.array([[1.0, 1.37, 2.9], [7.49, 63.5, 64.2], [127.9, 128.0, 129.3], [700.6, 1023.7, 2049.1],
                       [4095.5, 5000.25, 8191.6], [8192.0, 9000.0, 5.0e8]])
    q = np.linspace(0.1, 0.9, trials.shape[0]).astype(np.float32)
    _check_fold_pool(torch, pn, e, trials, q)


def test_adam_step(torch, pn):
    """Adam on the flat parameter buffer against the update rule in FP64."""
    model = pn.ProposalNet()
    rng = np.random.default_rng(3)
    p0 = model.flat.cpu().numpy().astype(np.float64)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    pcur = p0.copy()
    for step in (1, 2):
        g = rng.normal(0, 1e-2, p0.shape).astype(np.float32).astype(np.float64)
        model.grad.copy_(torch.as_tensor(g, dtype=torch.float32))
        model.adam(lr=1e-3)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        pcur = pcur - 1e-3 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    torch.cuda.synchronize()
    got = model.flat.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - pcur) <= 1e-6 * np.abs(pcur) + 1e-8)
    # packed bf16 weights follow the masters, padding zero
    w0 = model.packed[0].float().cpu().numpy()
    assert np.array_equal(w0[:, :144], onet.bf16(model.view("W0").cpu().numpy())[:, :144]) and np.all(w0[:, 144:] == 0)


def test_training_reduces_loss(torch, pn):
    """Adam steps on a fixed batch lower the loss (periodic spikes in the
    input, label = the window of their spacing); the FP64 oracle network
    falls from 0.69 to 0.08 in 30 steps of this problem at the same rate."""
    B, L = 4, 512
    win = pn.Windows.log_spaced(32, 0.1, 5.0, 0.02)
    x = np.zeros((B, L, 16), dtype=np.float32)
    y = np.zeros((B, win.n), dtype=np.float32)
    rng = np.random.default_rng(5)
    for b in range(B):
        spacing = int(rng.integers(20, 200))
        x[b, int(rng.integers(spacing))::spacing, :] = 1.0
        y[b] = win.labels([spacing * 0.02])[0]
    model = pn.ProposalNet(seed=2)
    xd = torch.as_tensor(x, device="cuda").to(torch.bfloat16)
    yd = torch.as_tensor(y, device="cuda")
    losses = []
    print("[net] training steps", flush=True)
    for _ in range(60):
        model.forward(xd, win)
        losses.append(float(model.backward(yd, pos_weight=8.0).item()))
        model.adam(lr=1e-3)
    assert np.all(np.isfinite(losses)) and min(losses[-10:]) < 0.5 * losses[0], losses


def test_topk_windows(torch, pn):
    rng = np.random.default_rng(9)
    B, W = 3, 700
    s = rng.normal(size=(B, W)).astype(np.float32)
    s[0, 10] = s[0, 20] = s[0, 30] = 5.0  # ties: smaller index first
    for K in (1, 64, W):
        out = pn.topk_windows(torch.as_tensor(s, device="cuda"), K).cpu().numpy()
        for b in range(B):
            ref = np.lexsort((np.arange(W), -s[b]))[:K]
            assert np.array_equal(out[b], ref), (K, b)


def test_windows_to_periods(torch, pn):
    win = pn.Windows.log_spaced(512, 0.5, 45.0, 0.01)
    periods = np.geomspace(0.3, 60.0, 20011)  # partly outside the windows
    sel = np.array([0, 3, 511, 250, 250, -1, 600], dtype=np.int32)  # duplicates and out-of-range ignored
    subset, n = pn.windows_to_periods(torch.as_tensor(periods, device="cuda"), win,
                                      torch.as_tensor(sel, device="cuda"))
    torch.cuda.synchronize()
    w = np.searchsorted(win.edges, periods, side="right") - 1
    keep = np.isin(w, sel[(sel >= 0) & (sel < 512)]) & (w >= 0) & (w < 512)
    ref = np.nonzero(keep)[0]
    assert int(n.item()) == ref.size
    assert np.array_equal(subset.cpu().numpy()[:ref.size], ref)


def test_downsample(torch, pn):
    """The downsample kernel against the net oracle's definition (oracle.net
    .downsample, FP64) on pairs with null elements, a saturated duration, a
    ragged last bin and an empty first bin row: within the bfloat16 rounding
    of the stored feature (2^-8 relative) plus the FP32 arithmetic."""
    from oracle import net as onet
    rng = np.random.default_rng(11)
    for J, I, nb in ((16, 10007, 257), (3, 500, 499), (5, 64, 8)):
        fold = np.stack([rng.normal(0, 1, (J, I)), rng.uniform(0, 2, (J, I))], axis=2).astype(np.float32)
        fold[:, ::7, 1] = 0.0  # null elements
        fold[min(3, J - 1), :, 0] = 1e4  # saturates at 30
        fold[0, : I // nb + 1, 1] = 0.0  # the first bin of duration 0 is all null
        jn = 1 % J
        fold[jn, : 2 * (I // nb) + 2, 0] = -np.abs(fold[jn, : 2 * (I // nb) + 2, 0]) - 0.25  # brightenings only
        print(f"[case] downsample J={J} I={I} bins={nb}", flush=True)
        out = pn.downsample(torch.as_tensor(fold, device="cuda"), nb).float().cpu().numpy()
        ref = onet.downsample(fold, nb)
        assert out.shape == ref.shape
        assert np.all(np.abs(out - ref) <= 2.0 ** -8 * ref + 1e-6), np.max(np.abs(out - ref) - 2.0 ** -8 * ref)
        sat = ref[:, min(3, J - 1)] == 3.75
        assert sat.sum() > nb // 2 and np.all(out[:, min(3, J - 1)][sat] == 3.75) and out[0, 0] == 0.0
        # the signed form: largest S_fm / sqrt(S_mm), clipped to [-30, 30]
        out_s = pn.downsample(torch.as_tensor(fold, device="cuda"), nb, signed=True).float().cpu().numpy()
        ref_s = onet.downsample_signed(fold, nb)
        assert np.all(np.abs(out_s - ref_s) <= 2.0 ** -8 * np.abs(ref_s) + 1e-6)
        assert out_s[0, 0] == 0.0 and (J == 1 or (ref_s[1, jn] < 0 and out_s[1, jn] < 0))


@pytest.mark.parametrize("E,n_pos", [(8, 3000), (5, 2049), (16, 700), (8, 0)])
def test_project_backward_against_the_plain_sums(torch, pn, E, n_pos):
    """dh = ge P, dP += ge^T h, dp += column sums of ge, with a ragged last
    workgroup and the compile-time (E = 8) and run-time channel counts."""
    from paper_2503_20875_amd import _abi
    rng = np.random.default_rng(100 + E + n_pos)
    h = onet.bf16(rng.normal(0, 1, (n_pos, 64)))
    ge = rng.normal(0, 1, (n_pos, E)).astype(np.float32).astype(np.float64)
    P = rng.normal(0, 0.1, (E, 64)).astype(np.float32).astype(np.float64)
    dP0 = rng.normal(0, 1, (E, 64)).astype(np.float32).astype(np.float64)
    dp0 = rng.normal(0, 1, E).astype(np.float32).astype(np.float64)
    print(f"[net] project bwd E={E} n_pos={n_pos}", flush=True)
    h_d = to_dev(torch, h.reshape(max(n_pos, 1), 64) if n_pos else np.zeros((1, 64)), torch.bfloat16)
    ge_d = to_dev(torch, ge if n_pos else np.zeros((1, E)), torch.float32)
    P_d = to_dev(torch, P, torch.float32)
    dh = torch.zeros((max(n_pos, 1), 64), dtype=torch.float32, device="cuda")
    dP = to_dev(torch, dP0, torch.float32)
    dp = to_dev(torch, dp0, torch.float32)
    _abi.check(_abi.load().cetra_net_project_bwd(None, h_d.data_ptr(), ge_d.data_ptr(), n_pos, P_d.data_ptr(), E,
                                                 dh.data_ptr(), dP.data_ptr(), dp.data_ptr()))
    torch.cuda.synchronize()
    ref_P = dP0 + ge.T @ h
    ref_p = dp0 + ge.sum(axis=0)
    for got, ref, absref in ((dP, ref_P, np.abs(dP0) + np.abs(ge).T @ np.abs(h)),
                             (dp, ref_p, np.abs(dp0) + np.abs(ge).sum(axis=0))):
        assert np.all(np.abs(got.cpu().numpy() - ref) <= 1e-5 * absref + 1e-30)
    if n_pos:
        ref_h = ge @ P
        assert np.all(np.abs(dh.cpu().numpy() - ref_h) <= 1e-5 * (np.abs(ge) @ np.abs(P)) + 1e-30)
