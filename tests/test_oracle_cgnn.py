"""Pins of the oracle's CGNN: direct-sum convolution, equivariances, LN, MP, FD gradients (no GPU)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cgnn, nr, receiver, slot_sim


def _direct_conv(x, w, b):
    """Pure-Python loops: out[s,t,o] = b[o] + sum_{i,j,c} w[i,j,c,o] x[s+i-1,t+j-1,c] (zero outside)."""
    S, T, C = x.shape
    O = w.shape[3]
    out = np.zeros((S, T, O))
    for s in range(S):
        for t in range(T):
            for o in range(O):
                acc = b[o]
                for i in range(3):
                    for j in range(3):
                        ss, tt = s + i - 1, t + j - 1
                        if 0 <= ss < S and 0 <= tt < T:
                            for c in range(C):
                                acc += w[i, j, c, o] * x[ss, tt, c]
                out[s, t, o] = acc
    return out


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 4, 3))
    w = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(2)
    assert np.allclose(cgnn.conv3x3(x, w, b), _direct_conv(x, w, b), atol=1e-12)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((9, 14, 4))
    w = rng.standard_normal((3, 3, 4, 3))
    out = cgnn.conv3x3(x, w, np.zeros(3))
    for o in range(3):
        ref = sum(correlate2d(x[:, :, c], w[:, :, c, o], mode="same") for c in range(4))
        assert np.allclose(out[:, :, o], ref, atol=1e-12)


def test_conv_impulse_orientation():
    # a one-hot input at (s0, t0) produces w[i, j] at output (s0 - i + 1, t0 - j + 1)
    w = np.arange(9, dtype=float).reshape(3, 3, 1, 1)
    x = np.zeros((5, 5, 1))
    x[2, 2, 0] = 1
    out = cgnn.conv3x3(x, w, np.zeros(1))[:, :, 0]
    for i in range(3):
        for j in range(3):
            assert out[2 - i + 1, 2 - j + 1] == w[i, j, 0, 0]
    # zero padding: an impulse in the corner only reaches the 2x2 neighbourhood
    x = np.zeros((5, 5, 1))
    x[0, 0, 0] = 1
    out = cgnn.conv3x3(x, np.ones((3, 3, 1, 1)), np.zeros(1))[:, :, 0]
    assert out.sum() == 4


def test_layer_norm_cases():
    g = np.array([2.0, 3.0, 4.0])
    b = np.array([0.5, -1.0, 0.0])
    y, _ = cgnn.layer_norm(np.full((2, 3), 7.0), g, b)
    assert np.allclose(y, b)                                  # constant row -> beta
    z = np.array([[1.0, 2.0, 6.0]])
    y, _ = cgnn.layer_norm(z, np.ones(3), np.zeros(3))
    assert np.isclose(y.mean(), 0) and np.isclose((y ** 2).mean(), 14 / 3 / (14 / 3 + 1e-5))


def test_aggregate_others():
    m = np.arange(12, dtype=float).reshape(1, 3, 4)
    agg = cgnn.aggregate_others(m)
    assert np.allclose(agg, m.sum(axis=1, keepdims=True) - m)
    assert np.all(cgnn.aggregate_others(m[:, :1]) == 0)      # one UE: nothing received


def test_positional_encoding():
    pe = cgnn.positional_encoding(8, 4)
    assert np.isclose(pe[0, :, 0, 0].mean(), 0) and np.isclose(pe[0, :, 0, 0].std(), 1)
    assert pe[0, 2, 0, 0] == pe[0, 11, 0, 0] == pe[0, :, 0, 0].min()
    assert pe[0, 0, 0, 1] == -1 and pe[1, 0, 0, 1] == 1          # CDM group 0 on even subcarriers
    assert pe[0, 0, 2, 1] == 1 and pe[1, 0, 2, 1] == -1          # CDM group 1 on odd subcarriers


def _random_net(cfg, seed=0):
    rng = np.random.default_rng(seed)
    W = {}
    for name, shape in cgnn.layout(cfg):
        if name.endswith(".g"):
            W[name] = 1 + 0.1 * rng.standard_normal(shape)
        elif len(shape) == 1:
            W[name] = 0.1 * rng.standard_normal(shape)
        else:
            fan = np.prod(shape[:-1])
            W[name] = rng.standard_normal(shape) * np.sqrt(2 / fan)
    return W


def _slot(n_prb=2, B=2, U=3, m=4, seed=0):
    cfg = slot_sim.SimConfig(n_taps=3, tap_decay_ns=100, snr_db_lo=5, snr_db_hi=15)
    desc = slot_sim.SlotDesc(n_prb, B, U, [m] * U)
    r = slot_sim.simulate_slot(seed, 0, 0, cfg, desc, m)
    return desc, r, receiver.ls_estimate(r["y"], desc)


def test_layout_counts():
    cfg = cgnn.NetConfig(8, 128, 6, 2, 4)
    names = [n for n, _ in cgnn.layout(cfg)]
    assert names[0] == "conv_in.w" and names[-1] == "readout.b2"
    assert cfg.mp_blocks() == [0, 3]
    assert cgnn.NetConfig(16, 128, 8, 3, 6).mp_blocks() == [0, 2, 5]
    assert dict(cgnn.layout(cfg))["blk0.conv_a.w"] == (3, 3, 258, 128)
    assert dict(cgnn.layout(cfg))["blk1.conv_a.w"] == (3, 3, 128, 128)


def test_ue_permutation_equivariance():
    cfg = cgnn.NetConfig(2, 8, 2, 1, 4)
    W = _random_net(cfg)
    desc, r, h = _slot()
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    perm = [2, 0, 1]
    l1 = cgnn.forward_x(W, cfg, X, [4] * 3)
    l2 = cgnn.forward_x(W, cfg, X[:, :, perm], [4] * 3)
    assert np.allclose(l1[perm], l2, atol=1e-10)


def test_subcarrier_shift_equivariance_interior():
    cfg = cgnn.NetConfig(2, 8, 2, 1, 4)
    W = _random_net(cfg)
    desc, r, h = _slot(n_prb=4)
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    l1 = cgnn.forward_x(W, cfg, X, [4] * 3)
    l2 = cgnn.forward_x(W, cfg, X[2:], [4] * 3)      # drop two subcarriers: PE pattern keeps its phase
    depth = 1 + 2 * cfg.C + 1                         # receptive-field radius in subcarriers
    assert np.allclose(l1[:, :, 2 + depth:-depth], l2[:, :, depth:-depth], atol=1e-10)


def test_single_ue_gets_no_messages_and_masking():
    cfg = cgnn.NetConfig(2, 8, 2, 1, 4)
    W = _random_net(cfg)
    desc, r, h = _slot(U=1)
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    W2 = dict(W)
    W2["mp0.w2"] = W["mp0.w2"] * 5.0
    W2["mp0.b2"] = W["mp0.b2"] + 1.0
    assert np.allclose(cgnn.forward_x(W, cfg, X, [4]), cgnn.forward_x(W2, cfg, X, [4]))
    full = cgnn.forward_x(W, cfg, X, [4])
    part = cgnn.forward_x(W, cfg, X, [2])
    assert np.allclose(part[..., :2], full[..., :2]) and np.all(part[..., 2:] == 0)


def _loss(W, cfg, X, bits, m_list, S):
    llr = cgnn.forward_x(W, cfg, X, m_list)
    lab, msk = cgnn.bit_labels_grid(bits, S, cfg.m_max)
    valid = msk * (np.arange(cfg.m_max) < np.array(m_list)[:, None, None, None])
    return cgnn.bce_terms(llr, lab, valid).sum() / valid.sum()


def test_backward_matches_finite_differences():
    # central differences in fp64 on a small instance (2 PRB, width 6, 2 blocks, 1 MP round, B=2, U=3)
    cfg = cgnn.NetConfig(2, 6, 2, 1, 4)
    W = _random_net(cfg, 3)
    desc, r, h = _slot(seed=4)
    m_list = [4, 2, 4]
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    llr, cache = cgnn.forward_x(W, cfg, X, m_list, keep=True)
    lab, msk = cgnn.bit_labels_grid(r["bits"], desc.n_sc, cfg.m_max)
    valid = msk * (np.arange(cfg.m_max) < np.array(m_list)[:, None, None, None])
    G = cgnn.backward(W, cfg, cache, cgnn.bce_grad(llr, lab, valid, valid.sum()))
    rng = np.random.default_rng(5)
    eps = 1e-6
    for name, shape in cgnn.layout(cfg):
        for _ in range(3):
            idx = tuple(rng.integers(0, n) for n in shape)
            Wp, Wm = dict(W), dict(W)
            Wp[name] = W[name].copy(); Wp[name][idx] += eps
            Wm[name] = W[name].copy(); Wm[name][idx] -= eps
            fd = (_loss(Wp, cfg, X, r["bits"], m_list, desc.n_sc)
                  - _loss(Wm, cfg, X, r["bits"], m_list, desc.n_sc)) / (2 * eps)
            assert abs(fd - G[name][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, G[name][idx])
    # a random direction through all weights at once
    v = {k: rng.standard_normal(w.shape) for k, w in W.items()}
    Wp = {k: W[k] + eps * v[k] for k in W}
    Wm = {k: W[k] - eps * v[k] for k in W}
    fd = (_loss(Wp, cfg, X, r["bits"], m_list, desc.n_sc) - _loss(Wm, cfg, X, r["bits"], m_list, desc.n_sc)) / (2 * eps)
    an = sum(np.sum(G[k] * v[k]) for k in W)
    assert abs(fd - an) <= 1e-6 * abs(fd)


def test_bce_and_adam():
    assert np.isclose(cgnn.bce_terms(np.zeros(1), np.zeros(1), np.ones(1))[0], np.log(2))
    big = np.array([800.0, -800.0])
    assert np.allclose(cgnn.bce_terms(big, np.array([1.0, 0.0]), np.ones(2)), 0)
    assert np.allclose(cgnn.bce_terms(big, np.array([0.0, 1.0]), np.ones(2)), 800)
    # first Adam step moves every weight by lr * sign(g) (up to eps)
    w = np.zeros(4)
    g = np.array([3.0, -0.01, 1e-3, -40.0])
    w1, m, v = cgnn.adam_step(w, g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    assert np.allclose(w1, -1e-3 * np.sign(g), rtol=1e-4)


def test_adam_third_step_against_hand_values():
    """Three Adam steps (Kingma & Ba, Algorithm 1) with gradients 1, 0, 0.  At step 1 the bias
    correction cancels both decay rates, so only a later step sees them.  After step 3:
    m3 = (1 - b1) b1^2 = 0.1 * 0.81 = 0.081, bias-corrected 0.081 / (1 - 0.729) = 0.298893...;
    v3 = (1 - b2) b2^2 = 0.001 * 0.998001 = 9.98001e-4, bias-corrected 9.98001e-4 / (1 - 0.997002999)
    = 0.333000...; the third step moves the weight by -lr * 0.298893 / (0.577062 + eps) = -0.517957 lr.
    Swapped decay rates would give -0.609 lr; a missing bias correction -0.0810 / 0.0316 lr."""
    w = np.array([0.0])
    m = np.zeros(1)
    v = np.zeros(1)
    steps = []
    for t, g in enumerate([1.0, 0.0, 0.0], start=1):
        w_new, m, v = cgnn.adam_step(w, np.array([g]), m, v, t, lr=1e-3)
        steps.append(float(w_new[0] - w[0]))
        w = w_new
    assert abs(m[0] - 0.081) < 1e-15 and abs(v[0] - 9.98001e-4) < 1e-15
    # step 2: m2 = 0.09, mhat = 0.09/0.19; v2 = 9.99e-4, vhat = 9.99e-4/1.999e-3
    assert abs(steps[1] - (-1e-3 * (0.09 / 0.19) / (np.sqrt(9.99e-4 / 1.999e-3) + 1e-8))) < 1e-15
    assert abs(steps[2] / 1e-3 - (-0.5179570)) < 1e-6, steps[2]


def test_window_reproduces_full_grid():
    """The 1 + 2C stacked 3x3 convolutions see C' = 1 + 2C subcarriers either way; with message
    passing and the readout acting per RE, a window of +-16 subcarriers starting on an even
    subcarrier (the PE comb parity) gives the full-grid LLRs at its centre, bit for bit.  The GPU
    test at the benchmark's full size relies on this."""
    from oracle import receiver, slot_sim
    from paper_2409_02912_amd import synth
    net = cgnn.NetConfig(8, 32, 6, 2, 4)
    W = cgnn.unflatten(synth.he_weights(cgnn.layout(net), 3, perturb=True).astype(np.float64), net)
    cfg = slot_sim.SimConfig(n_taps=12, tap_decay_ns=487.42, snr_db_lo=10, snr_db_hi=10)
    d = slot_sim.SlotDesc(6, 8, 4, [4] * 4, slot_number=3)
    r = slot_sim.simulate_slot(0, 0, 0, cfg, d, 4)
    y, S = r["y"], 72
    h = receiver.ls_estimate(y, d)
    full = cgnn.forward(W, net, y, h, d.bits_per_sym)
    for s0 in (0, 35, 71, 20):
        lo, hi = max(0, s0 - 16) & ~1, min(S, s0 + 17)
        win = cgnn.forward(W, net, y[lo:hi], h[lo:hi], d.bits_per_sym)[:, :, s0 - lo, :]
        assert np.array_equal(win, full[:, :, s0, :])


def _truncated(W, cfg, k):
    """The network of the first k CGNN iterations as a network of its own (its config and weights)."""
    ck = cgnn.iteration_ends(cfg)[k - 1]
    sub = cgnn.NetConfig(cfg.B, cfg.d, ck, k if cfg.R else 0, cfg.m_max)
    return {name: W[name] for name, _ in cgnn.layout(sub)}, sub


def test_depth_control_equals_shallower_network():
    # running the first k iterations and reading out (Sec. IV-B) is the plain forward of the network made of
    # those blocks and rounds only; all_iters returns the same LLRs after every iteration
    cfg = cgnn.NetConfig(2, 6, 6, 3, 4)
    assert cgnn.iteration_ends(cfg) == [2, 4, 6]
    assert cgnn.iteration_ends(cgnn.NetConfig(2, 6, 6, 2, 4)) == [3, 6]
    assert cgnn.iteration_ends(cgnn.NetConfig(2, 6, 2, 0, 4)) == [2]
    W = _random_net(cfg, 8)
    desc, r, h = _slot(seed=9)
    m_list = [4, 2, 4]
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    every = cgnn.forward_x(W, cfg, X, m_list, all_iters=True)
    assert len(every) == 3
    assert np.array_equal(every[-1], cgnn.forward_x(W, cfg, X, m_list))
    for k in (1, 2, 3):
        Wk, ck = _truncated(W, cfg, k)
        assert ck.mp_blocks() == cfg.mp_blocks()[:k]
        ref = cgnn.forward_x(Wk, ck, X, m_list)
        assert np.array_equal(cgnn.forward_x(W, cfg, X, m_list, n_iter=k), ref)
        assert np.array_equal(every[k - 1], ref)
    # the readouts differ from iteration to iteration (the state keeps changing)
    assert not np.allclose(every[0], every[1])


def test_multi_loss_gradient():
    # the multi-loss gradient (Sec. II-B: one loss per iteration's readout, readout layers shared) is the sum
    # of the single-readout gradients of the truncated networks, and matches central differences
    cfg = cgnn.NetConfig(2, 6, 4, 2, 4)
    W = _random_net(cfg, 11)
    desc, r, h = _slot(seed=12)
    m_list = [4, 4, 2]
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    llrs, cache = cgnn.forward_x(W, cfg, X, m_list, keep=True, all_iters=True)
    rng = np.random.default_rng(13)
    dl = [rng.standard_normal(l.shape) for l in llrs]
    G = cgnn.backward(W, cfg, cache, dl)
    S = {k: np.zeros_like(v) for k, v in W.items()}
    for k in (1, 2):
        Wk, ck = _truncated(W, cfg, k)
        _, ca = cgnn.forward_x(Wk, ck, X, m_list, keep=True)
        for name, g in cgnn.backward(Wk, ck, ca, dl[k - 1]).items():
            S[name] += g
    for name in W:
        assert np.allclose(G[name], S[name], rtol=1e-12, atol=1e-12), name
    eps = 1e-6

    def f(Wx):
        return sum(np.sum(d * l) for d, l in zip(dl, cgnn.forward_x(Wx, cfg, X, m_list, all_iters=True)))
    v = {k: rng.standard_normal(w.shape) for k, w in W.items()}
    fd = (f({k: W[k] + eps * v[k] for k in W}) - f({k: W[k] - eps * v[k] for k in W})) / (2 * eps)
    an = sum(np.sum(G[k] * v[k]) for k in W)
    assert abs(fd - an) <= 1e-6 * abs(fd)


def test_double_readout_gradient():
    # double readout (Sec. II-A, II-B): loss = sum(dl * llr) + gamma * MSE(ĥ, h) over the readouts of every
    # iteration; the backward with the MSE gradient matches central differences of the forward, on a slot
    # with fewer antennas than the network (the unused ReadoutChEst outputs get no gradient)
    cfg = cgnn.NetConfig(3, 6, 4, 2, 4, chest=True)
    W = _random_net(cfg, 21)
    desc, r, h = _slot(B=2, seed=22)
    m_list = [4, 4, 4]
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    gamma = 0.7
    llrs, cache = cgnn.forward_x(W, cfg, X, m_list, keep=True, all_iters=True, n_ant=2)
    assert len(cache["hests"]) == 2 and cache["hests"][0].shape == r["h"].shape
    rng = np.random.default_rng(23)
    dl = [rng.standard_normal(l.shape) for l in llrs]
    dhe = [cgnn.mse_grad([he], [r["h"]], gamma)[1][0] for he in cache["hests"]]
    G = cgnn.backward(W, cfg, cache, dl, dhe)
    assert np.all(G["readout_ch.w2"][:, 4:] == 0) and np.all(G["readout_ch.b2"][4:] == 0)

    def f(Wx):
        ls, c = cgnn.forward_x(Wx, cfg, X, m_list, keep=True, all_iters=True, n_ant=2)
        return (sum(np.sum(d * l) for d, l in zip(dl, ls))
                + gamma * sum(cgnn.mse_grad([he], [r["h"]], gamma)[0] for he in c["hests"]))
    eps = 1e-8     # small enough that no ReLU of this seed changes side within the step
    v = {k: rng.standard_normal(w.shape) for k, w in W.items()}
    fd = (f({k: W[k] + eps * v[k] for k in W}) - f({k: W[k] - eps * v[k] for k in W})) / (2 * eps)
    an = sum(np.sum(G[k] * v[k]) for k in W)
    assert abs(fd - an) <= 1e-6 * abs(fd)
    # the LLR readout and its gradient are those of the same network without ReadoutChEst
    c0 = cgnn.NetConfig(3, 6, 4, 2, 4)
    W0 = {name: W[name] for name, _ in cgnn.layout(c0)}
    l0, ca0 = cgnn.forward_x(W0, c0, X, m_list, keep=True, all_iters=True, n_ant=2)
    assert all(np.array_equal(a, b) for a, b in zip(l0, llrs))
    G0 = cgnn.backward(W0, c0, ca0, dl)
    Gl = cgnn.backward(W, cfg, cache, dl)
    for name in W0:
        assert np.allclose(G0[name], Gl[name], rtol=1e-12, atol=1e-14), name


def test_chest_readout_closed_form_with_zero_second_layer():
    # with a zero second layer every RE's estimate is the bias pair (b_2b + i b_2b+1) of its antenna, so
    # the MSE and its bias gradient have closed forms: mean |c_b - h|^2 and 2 gamma sum_{antenna b} (c_b - h) / N
    cfg = cgnn.NetConfig(2, 6, 2, 1, 4, chest=True)
    W = _random_net(cfg, 31)
    W["readout_ch.w2"][:] = 0.0
    desc, r, h = _slot(B=2, seed=32)
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    _, cache = cgnn.forward_x(W, cfg, X, [4, 4, 4], keep=True)
    c = W["readout_ch.b2"][0::2] + 1j * W["readout_ch.b2"][1::2]
    assert np.allclose(cache["hests"][0], np.broadcast_to(c, r["h"].shape), rtol=0, atol=1e-15)
    gamma = 0.3
    mse, (g,) = cgnn.mse_grad(cache["hests"], [r["h"]], gamma)
    H = r["h"].reshape(-1, 2)
    assert abs(mse - np.mean(np.abs(H - c) ** 2)) <= 1e-12 * mse
    G = cgnn.backward(W, cfg, cache, np.zeros((3, 14, r["y"].shape[0], 4)), g)
    want = 2 * gamma * np.sum(c - H, axis=0) / H.size
    assert np.allclose(G["readout_ch.b2"][0::2], want.real, rtol=1e-10, atol=1e-14)
    assert np.allclose(G["readout_ch.b2"][1::2], want.imag, rtol=1e-10, atol=1e-14)
    # the first layer of the head gets no gradient through a zero second layer
    assert np.all(G["readout_ch.w1"] == 0) and np.all(G["readout_ch.b1"] == 0)


def test_var_io():
    # Var-IO (Sec. III, Fig. 2): each UE starts from its modulation's own StateInit and is read out by its own
    # ReadoutLLRs with m_u outputs.  (i) with every modulation's layers equal to the shared ones (readout cut to its
    # first m outputs) it is the masking scheme; (ii) central differences of the forward match the backward on a
    # slot mixing two modulations, and the layers of the modulation nobody uses get no gradient
    cfg = cgnn.NetConfig(2, 6, 2, 1, 6, var_io=True)
    plain = cgnn.NetConfig(2, 6, 2, 1, 6)
    Wp = _random_net(plain, 51)
    desc, r, h = _slot(U=3, m=4, seed=52)
    m_list = [4, 2, 4]
    X = cgnn.nrx_inputs(r["y"], h, cfg)
    W = {k: v for k, v in Wp.items() if not k.startswith("readout.") and not k.startswith("conv_in.")}
    for m in cfg.mods():
        W[f"conv_in.m{m}.w"], W[f"conv_in.m{m}.b"] = Wp["conv_in.w"], Wp["conv_in.b"]
        W[f"readout.m{m}.w1"], W[f"readout.m{m}.b1"] = Wp["readout.w1"], Wp["readout.b1"]
        W[f"readout.m{m}.w2"], W[f"readout.m{m}.b2"] = Wp["readout.w2"][:, :m], Wp["readout.b2"][:m]
    assert set(W) == {n for n, _ in cgnn.layout(cfg)}
    # (the per-modulation convolutions over a subset of UEs sum in another order: equal to rounding)
    assert np.allclose(cgnn.forward_x(W, cfg, X, m_list), cgnn.forward_x(Wp, plain, X, m_list), rtol=1e-12,
                       atol=1e-12)
    W = _random_net(cfg, 53)
    llr, cache = cgnn.forward_x(W, cfg, X, m_list, keep=True)
    assert np.all(llr[1, :, :, 2:] == 0) and np.all(llr[0, :, :, 4:] == 0)
    rng = np.random.default_rng(54)
    dl = rng.standard_normal(llr.shape)
    G = cgnn.backward(W, cfg, cache, dl)
    assert all(np.all(G[n] == 0) for n in ("readout.m6.w1", "readout.m6.b1", "readout.m6.w2", "readout.m6.b2",
                                           "conv_in.m6.w", "conv_in.m6.b"))
    assert np.any(G["readout.m2.w2"] != 0) and np.any(G["readout.m4.w2"] != 0)
    assert np.any(G["conv_in.m2.w"] != 0) and np.any(G["conv_in.m4.w"] != 0)
    eps = 1e-8
    v = {k: rng.standard_normal(w.shape) for k, w in W.items()}
    f = lambda Wx: np.sum(dl * cgnn.forward_x(Wx, cfg, X, m_list))  # noqa: E731
    fd = (f({k: W[k] + eps * v[k] for k in W}) - f({k: W[k] - eps * v[k] for k in W})) / (2 * eps)
    an = sum(np.sum(G[k] * v[k]) for k in W)
    assert abs(fd - an) <= 1e-6 * abs(fd)


def test_conv_backward_is_the_adjoint():
    """The 3x3 conv is bilinear in (x, w): for any output cotangent g, <conv(x, w), g> = <x, dx> = <w, dw>, and
    db sums g over the grid.  Exact identities (fp64 rounding only); a transposed kernel, a flipped tap or a
    shifted window in the backward breaks them."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal((6, 5, 2, 3))          # [S, T, U, C]: the UE axis rides along like the conv's
    w = rng.standard_normal((3, 3, 3, 4))
    g = rng.standard_normal((6, 5, 2, 4))
    y = cgnn.conv3x3(x, w, np.zeros(4))
    dx, dw, db = cgnn.conv3x3_backward(x, w, g)
    ref = float(np.sum(y * g))
    assert abs(float(np.sum(x * dx)) - ref) < 1e-10 * abs(ref) + 1e-10
    assert abs(float(np.sum(w * dw)) - ref) < 1e-10 * abs(ref) + 1e-10
    assert np.allclose(db, g.reshape(-1, 4).sum(axis=0), rtol=0, atol=1e-12)
    # per-element: dx[s, t] collects w[i, j] applied to g[s - i + 1, t - j + 1] (direct sum)
    S, T = 6, 5
    want = np.zeros_like(x)
    for s in range(S):
        for t in range(T):
            for i in range(3):
                for j in range(3):
                    so, to = s - i + 1, t - j + 1
                    if 0 <= so < S and 0 <= to < T:
                        want[s, t] += g[so, to] @ w[i, j].T
    assert np.allclose(dx, want, rtol=0, atol=1e-12)


def test_layer_norm_backward_against_central_differences():
    """LayerNorm backward: central differences of <LN(z), r> in z, gamma and beta, and the exact properties of
    the input gradient: zero mean over the normalised axis, and (gamma = 1) a component along the normalised
    input of rstd <r, zhat> (1 - mean zhat^2), which the epsilon inside the square root leaves nonzero."""
    rng = np.random.default_rng(12)
    z = rng.standard_normal((3, 8)) * 2.0 + 0.5
    gam = 1.0 + 0.3 * rng.standard_normal(8)
    bet = 0.2 * rng.standard_normal(8)
    r = rng.standard_normal((3, 8))
    f = lambda zz, gg, bb: float(np.sum(cgnn.layer_norm(zz, gg, bb)[0] * r))
    _, cache = cgnn.layer_norm(z, gam, bet)
    dz, dg, db = cgnn.layer_norm_backward(r, gam, cache)
    eps = 1e-6
    for arr, grad, name in ((z, dz, "z"), (gam, dg, "gamma"), (bet, db, "beta")):
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            p, m = arr.copy(), arr.copy()
            p[idx] += eps
            m[idx] -= eps
            args = {"z": (z, gam, bet), "gamma": (z, gam, bet), "beta": (z, gam, bet)}[name]
            ap = [p if a is arr else a for a in args]
            am = [m if a is arr else a for a in args]
            fd[idx] = (f(*ap) - f(*am)) / (2 * eps)
        assert np.allclose(grad, fd, rtol=1e-6, atol=1e-8), name
    assert np.allclose(dz.sum(axis=-1), 0.0, atol=1e-12)
    _, c1 = cgnn.layer_norm(z, np.ones(8), np.zeros(8))
    dz1, _, _ = cgnn.layer_norm_backward(r, np.ones(8), c1)
    zh, rs = c1
    want = rs[:, 0] * np.sum(r * zh, axis=-1) * (1.0 - np.mean(zh ** 2, axis=-1))
    assert np.allclose(np.sum(dz1 * zh, axis=-1), want, rtol=1e-9, atol=1e-14)
    assert np.all(np.abs(want) < 1e-4)   # orthogonal up to the epsilon term


def test_softplus_and_sigmoid():
    """softplus(x) - softplus(-x) = x, softplus(0) = ln 2, sigmoid(x) + sigmoid(-x) = 1, sigmoid is the
    derivative of softplus, and both stay finite far out (the BCE of a confident LLR)."""
    x = np.linspace(-30.0, 30.0, 601)
    assert np.allclose(cgnn.softplus(x) - cgnn.softplus(-x), x, rtol=0, atol=1e-12)
    assert cgnn.softplus(np.array(0.0)) == pytest.approx(np.log(2.0), abs=1e-15)
    assert np.allclose(cgnn.sigmoid(x) + cgnn.sigmoid(-x), 1.0, rtol=0, atol=1e-15)
    h = 1e-5
    assert np.allclose((cgnn.softplus(x + h) - cgnn.softplus(x - h)) / (2 * h), cgnn.sigmoid(x), rtol=0, atol=1e-9)
    big = np.array([-1000.0, 1000.0])
    assert np.array_equal(cgnn.softplus(big), np.array([0.0, 1000.0]))
    assert np.array_equal(cgnn.sigmoid(big), np.array([0.0, 1.0]))
    assert cgnn.relu(np.array(-2.0)) == 0.0 and cgnn.relu(np.array(3.0)) == 3.0
