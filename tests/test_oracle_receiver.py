"""Pins of the oracle's slot simulator and classical receiver (no GPU)."""
import math

import numpy as np
import pytest
from scipy.special import j0

from oracle import nr, receiver, slot_sim


def _grid_from_h(H, desc, noise_var=0.0, rng=None):
    bits = slot_sim.bits(1, 0, 0, desc, 8)
    x = slot_sim.transmit_grid(desc, bits)
    y = np.einsum('stub,stu->stb', H, x)
    if noise_var:
        y = y + np.sqrt(noise_var / 2) * (rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape))
    return y, x, bits


def test_ls_exact_on_constant_channel_all_ports():
    # Noiseless, frequency/time-flat channel: OCC despreading cancels the co-group port exactly.
    rng = np.random.default_rng(0)
    desc = slot_sim.SlotDesc(4, 4, 4, [4, 4, 4, 4], slot_number=5)
    hc = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    H = np.broadcast_to(hc, (desc.n_sc, 14, 4, 4)).copy()
    y, _, _ = _grid_from_h(H, desc)
    assert np.allclose(receiver.ls_estimate(y, desc), H, atol=1e-12)


def test_ls_affine_channel_reproduced_in_interior():
    # Noiseless channel affine in s and t: a pair average equals the channel at the pair centre, and
    # linear interpolation reproduces an affine function between the outermost pair centres and
    # between the two DMRS symbols.
    rng = np.random.default_rng(1)
    desc = slot_sim.SlotDesc(4, 2, 1, [2], slot_number=1)
    S = desc.n_sc
    a, b, c = (rng.standard_normal(2) + 1j * rng.standard_normal(2) for _ in range(3))
    s = np.arange(S)[:, None, None]
    t = np.arange(14)[None, :, None]
    H = (a + 0.01 * s * b + 0.02 * t * c)[:, :, None, :]
    y, _, _ = _grid_from_h(H, desc)
    est = receiver.ls_estimate(y, desc)
    lo, hi = 1, 4 * (S // 4 - 1) + 1
    assert np.allclose(est[lo:hi + 1, 2:12, 0], H[lo:hi + 1, 2:12, 0], atol=1e-12)


@pytest.mark.parametrize("port", [0, 1, 2, 3])
def test_ls_edge_rules_on_affine_channel(port):
    """Flat extrapolation: on a noiseless channel affine in s and t, seen by one port (the others
    silent, so the OCC sees no co-group leakage), the estimate at (s, t) equals the channel at
    (clamp(s, first pair centre, last pair centre), clamp(t, 2, 11)) everywhere on the grid --
    symbols 0, 1 repeat symbol 2, symbols 12, 13 repeat symbol 11, and subcarriers below the
    first / above the last pair centre of the port's CDM group repeat that centre."""
    rng = np.random.default_rng(11 + port)
    U = port + 1
    desc = slot_sim.SlotDesc(3, 2, U, [2] * U, slot_number=7)
    S = desc.n_sc
    a, b, c = (rng.standard_normal(2) + 1j * rng.standard_normal(2) for _ in range(3))
    s = np.arange(S)[:, None, None]
    t = np.arange(14)[None, :, None]
    H = np.zeros((S, 14, U, 2), dtype=np.complex128)
    H[:, :, port, :] = a + 0.03 * s * b + 0.05 * t * c
    y, _, _ = _grid_from_h(H, desc)
    est = receiver.ls_estimate(y, desc)[:, :, port]
    delta = port // 2
    first, last = 1 + delta, 4 * (S // 4 - 1) + 1 + delta
    sc = np.clip(np.arange(S), first, last)
    tc = np.clip(np.arange(14), 2, 11)
    want = (a + 0.03 * sc[:, None, None] * b + 0.05 * tc[None, :, None] * c)
    assert np.allclose(est, want, atol=1e-12)
    # the rule really extrapolates: the grid's edges differ from the channel there
    assert not np.allclose(est[0, 0], H[0, 0, port]) and not np.allclose(est[S - 1, 13], H[S - 1, 13, port])


def test_lmmse_noiseless_recovers_symbols():
    rng = np.random.default_rng(2)
    desc = slot_sim.SlotDesc(2, 8, 4, [4, 4, 4, 4])
    H = rng.standard_normal((desc.n_sc, 14, 4, 8)) + 1j * rng.standard_normal((desc.n_sc, 14, 4, 8))
    y, x, _ = _grid_from_h(H, desc)
    z, var = receiver.lmmse_equalise(y, H, 0.0)
    dsym = nr.data_symbols()
    assert np.allclose(z[:, dsym], x[:, dsym], atol=1e-10)


def test_lmmse_demap_layout_and_noiseless_decisions():
    """LMMSE + max-log demapping into the LLR layout [u][t][s][j], given the channel: on a noiseless slot with
    the true channel and a tiny N0, every data-RE LLR decides its transmitted bit (l > 0 decides 1), DMRS
    symbols and the outputs j >= m_u are zero, for UEs of different modulations."""
    rng = np.random.default_rng(21)
    desc = slot_sim.SlotDesc(2, 4, 3, [2, 6, 8])
    H = rng.standard_normal((desc.n_sc, 14, 3, 4)) + 1j * rng.standard_normal((desc.n_sc, 14, 3, 4))
    y, _, bits = _grid_from_h(H, desc)
    llr = receiver.lmmse_demap(y, H, 1e-9, desc, 8)
    S = desc.n_sc
    assert llr.shape == (3, 14, S, 8)
    dsym = nr.data_symbols()
    for t in range(14):
        if t not in dsym:
            assert np.all(llr[:, t] == 0.0)
    for u, m in enumerate(desc.bits_per_sym):
        assert np.all(llr[u, :, :, m:] == 0.0)
        for t in dsym:
            for s_ in range(S):
                got = (llr[u, t, s_, :m] > 0).astype(np.uint8)
                assert np.array_equal(got, bits[u, nr.data_re_index(s_, t, S), :m])
        # reliable decisions: every data LLR far from zero at this N0
        assert np.min(np.abs(llr[u][np.ix_(dsym, range(S), range(m))])) > 1e3


def test_lmmse_single_user_is_mrc():
    rng = np.random.default_rng(3)
    h = rng.standard_normal((50, 1, 4)) + 1j * rng.standard_normal((50, 1, 4))
    y = rng.standard_normal((50, 4)) + 1j * rng.standard_normal((50, 4))
    n0 = 0.3
    z, var = receiver.lmmse_equalise(y, h, n0)
    g = np.sum(np.abs(h[:, 0]) ** 2, axis=-1)
    zt = np.sum(np.conj(h[:, 0]) * y, axis=-1) / (g + n0)
    d = g / (g + n0)
    assert np.allclose(z[:, 0], zt / d)
    assert np.allclose(var[:, 0], n0 / g)


def test_maxlog_qpsk_closed_form():
    rng = np.random.default_rng(4)
    z = rng.standard_normal(100) + 1j * rng.standard_normal(100)
    var = rng.uniform(0.1, 2, 100)
    l = receiver.maxlog_llr(z, var, 2)
    assert np.allclose(l[:, 0], -2 * np.sqrt(2) * z.real / var)
    assert np.allclose(l[:, 1], -2 * np.sqrt(2) * z.imag / var)


def test_maxlog_16qam_closed_form():
    a = 1 / np.sqrt(10)
    x = np.linspace(-5 * a, 5 * a, 101)
    z = x + 0.3j
    l = receiver.maxlog_llr(z, np.ones_like(x), 4)
    b0 = np.where(np.abs(x) <= 2 * a, -4 * a * x, np.where(x > 2 * a, -8 * a * (x - a), -8 * a * (x + a)))
    b2 = 4 * a * (np.abs(x) - 2 * a)
    assert np.allclose(l[:, 0], b0)
    assert np.allclose(l[:, 2], b2)


def test_maxlog_brute_force_per_axis():
    # max-log of a Gray-QAM point separates per axis (the label is a product of two PAM labels)
    rng = np.random.default_rng(5)
    for m in (4, 6, 8):
        z = 1.5 * (rng.standard_normal(40) + 1j * rng.standard_normal(40))
        l = receiver.maxlog_llr(z, np.ones(40), m)
        pts, bits = nr.constellation(m)
        re_lv = np.unique(np.round(pts.real, 12))
        for j in range(0, m, 2):
            # bit j depends only on the real part
            lab = {round(p.real, 12): bits[i, j] for i, p in enumerate(pts)}
            d = (z.real[:, None] - re_lv[None, :]) ** 2
            is1 = np.array([lab[round(v, 12)] for v in re_lv])
            ref = np.min(np.where(is1 == 0, d, np.inf), 1) - np.min(np.where(is1 == 1, d, np.inf), 1)
            assert np.allclose(l[:, j], ref)


def test_mrc_qpsk_ber_matches_textbook():
    # Genie CSI, U=1, B-branch MRC over iid Rayleigh: BER = ((1-mu)/2)^B sum_k C(B-1+k,k)((1+mu)/2)^k
    rng = np.random.default_rng(6)
    B, n = 2, 400_000
    n0 = 10 ** (-6 / 10)
    h = (rng.standard_normal((n, 1, B)) + 1j * rng.standard_normal((n, 1, B))) / np.sqrt(2)
    bits = rng.integers(0, 2, (n, 2))
    x = nr.qam_map(bits, 2)
    y = h[:, 0] * x[:, None] + np.sqrt(n0 / 2) * (rng.standard_normal((n, B)) + 1j * rng.standard_normal((n, B)))
    z, var = receiver.lmmse_equalise(y, h, n0)
    l = receiver.maxlog_llr(z[:, 0], var[:, 0], 2)
    ber = np.mean((l > 0) != bits)
    g = 1 / (2 * n0)
    mu = np.sqrt(g / (1 + g))
    p = ((1 - mu) / 2) ** B * sum(math.comb(B - 1 + k, k) * ((1 + mu) / 2) ** k for k in range(B))
    sd = np.sqrt(p * (1 - p) / (2 * n))
    assert abs(ber - p) < 5 * sd


# ---- slot simulator statistics ----

def test_channel_power_and_frequency_correlation():
    cfg = slot_sim.SimConfig(n_taps=12, tap_decay_ns=487.42)
    desc = slot_sim.SlotDesc(4, 4, 2, [2, 2])
    Hs = np.stack([slot_sim.channel(7, 0, k, cfg, desc) for k in range(200)])   # [K, S, T, U, B]
    assert abs(np.mean(np.abs(Hs) ** 2) - 1) < 0.05
    tau, p = slot_sim.pdp(cfg)
    for dk in (1, 4, 12):
        emp = np.mean(Hs[:, dk:] * np.conj(Hs[:, :-dk]))
        ref = np.sum(p * np.exp(-2j * np.pi * dk * 30e3 * tau))
        assert abs(emp - ref) < 0.06


def test_spatial_correlation_and_doppler():
    cfg = slot_sim.SimConfig(n_taps=1, rho=0.5, doppler_max_hz=0.0)
    desc = slot_sim.SlotDesc(1, 4, 1, [2])
    Hs = np.stack([slot_sim.channel(8, 0, k, cfg, desc)[0, 0, 0] for k in range(3000)])   # [K, B]
    R = Hs.T @ np.conj(Hs) / len(Hs)
    ref = 0.5 ** np.abs(np.arange(4)[:, None] - np.arange(4)[None, :])
    assert np.max(np.abs(R - ref)) < 0.08
    # time autocorrelation of the sum-of-sinusoids process is J0(2 pi fD dt) in expectation
    cfg2 = slot_sim.SimConfig(n_taps=1, doppler_max_hz=1000.0)
    desc2 = slot_sim.SlotDesc(1, 1, 1, [2])
    acc, ref2 = 0, 0
    for k in range(3000):
        _, fd = slot_sim.slot_params(9, 0, k, cfg2, 1)
        g = slot_sim.channel(9, 0, k, cfg2, desc2)[0, :, 0, 0]
        acc += g[13] * np.conj(g[0])
        ref2 += j0(2 * np.pi * fd[0] * 13 * slot_sim.T_SYM)
    assert abs(acc / 3000 - ref2 / 3000) < 0.06


def test_noise_variance_and_received_power():
    cfg = slot_sim.SimConfig(n_taps=3, tap_decay_ns=100, snr_db_lo=3, snr_db_hi=3)
    desc = slot_sim.SlotDesc(8, 4, 2, [4, 4])
    n = slot_sim.noise(3, 0, 0, desc, 0.5)
    assert abs(np.var(n) - 0.5) < 0.02
    pw = []
    for k in range(40):
        r = slot_sim.simulate_slot(3, 0, k, cfg, desc, 4)
        pw.append(np.mean(np.abs(r["y"][:, nr.data_symbols()]) ** 2))
    assert abs(np.mean(pw) - (2 + 10 ** -0.3)) < 0.2


def test_bits_and_rg_mapping():
    desc = slot_sim.SlotDesc(4, 4, 2, [2, 6])
    b = slot_sim.bits(11, 2, 3, desc, 8)
    assert b.shape == (2, 48 * 12, 8)
    assert np.all(b[0, :, 2:] == 0) and np.all(b[1, :, 6:] == 0)
    assert abs(b[1, :, :6].mean() - 0.5) < 0.05
    x = slot_sim.transmit_grid(desc, b)
    assert np.isclose(x[5, 3, 1], nr.qam_map(b[1, nr.data_re_index(5, 3, 48), :6], 6))
    assert np.allclose(x[:, 2, 0], nr.dmrs_grid(0, 48, 0, 2))
    assert np.allclose(x[:, 11, 1], nr.dmrs_grid(1, 48, 0, 11))


def test_snr_offset_scales_only_the_noise():
    # a per-slot SNR offset (mixed-MCS training, Sec. III-A) shifts the drawn SNR by exactly that many dB and
    # scales the same noise draw by 10^(-offset/20); channel, bits and symbols are unchanged
    cfg = slot_sim.SimConfig(n_taps=4, tap_decay_ns=100, snr_db_lo=0, snr_db_hi=10)
    d0 = slot_sim.SlotDesc(2, 2, 2, [4, 2])
    d1 = slot_sim.SlotDesc(2, 2, 2, [4, 2], snr_offset_db=7.5)
    a = slot_sim.simulate_slot(3, 1, 0, cfg, d0, 4)
    b = slot_sim.simulate_slot(3, 1, 0, cfg, d1, 4)
    assert abs(b["snr_db"] - a["snr_db"] - 7.5) < 1e-12
    assert np.array_equal(a["h"], b["h"]) and np.array_equal(a["bits"], b["bits"])
    na = a["y"] - np.einsum('stub,stu->stb', a["h"], a["x"])
    nb = b["y"] - np.einsum('stub,stu->stb', b["h"], b["x"])
    assert np.allclose(nb, na * 10 ** (-7.5 / 20), rtol=1e-10, atol=1e-14)
