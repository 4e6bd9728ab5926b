"""GPU parity for the configurations beyond the basic cases: 256-QAM (all eight LLR outputs), 16-antenna
LMMSE, an uneven batch shaped like the mixed 4-273 PRB workload, and the fallback of a slot whose NRX
LLRs are not finite to the LS + LMMSE receiver (Sec. III-B)."""
import numpy as np
import pytest

from nrx_cases import (check_llr, log, oracle_batch, oracle_nrx, pack_complex, rel_err, sim_cfg_oracle, split_llr)
from oracle import cgnn, nr, receiver
from paper_2409_02912_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
L = pytest.importorskip("paper_2409_02912_amd.libnrx")

SIMCFG = dict(n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0, snr=(15.0, 30.0))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def ws_tensor(nbytes):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


# 256-QAM and 16 antennas together (every LLR output of an m_max = 8 network in use)
QAM256 = [dict(n_prb=3, n_ant=16, n_ue=4, bits=[8, 8, 6, 2], slot_number=1),
          dict(n_prb=2, n_ant=16, n_ue=2, bits=[8, 4], slot_number=2, n_id=9),
          dict(n_prb=5, n_ant=4, n_ue=3, bits=[8, 2, 8], slot_number=3, n_scid=1),
          dict(n_prb=4, n_ant=8, n_ue=1, bits=[8], slot_number=4)]


@pytest.mark.parametrize("internal_ls", [False, True])
def test_lmmse_256qam_16_antennas(internal_ls):
    log(f"lmmse_demap: 256-QAM, 16 antennas, internal_ls={internal_ls}")
    ref = oracle_batch(QAM256, sim_cfg_oracle(SIMCFG), 31, 0, 8)
    shapes = [dict(s, n0=r["n0_32"]) for s, r in zip(QAM256, ref)]
    descs, sz = L.make_slots(shapes, 8)
    y = dev(pack_complex([r["y32"] for r in ref]))
    hls = [receiver.ls_estimate(r["y32"], r["desc"]) for r in ref]
    h = None if internal_ls else dev(pack_complex(hls))
    llr = torch.full((sz["llr"],), float("nan"), dtype=torch.float32, device="cuda")
    ws = ws_tensor(L.lmmse_workspace_bytes(descs))
    L.lmmse_demap(descs, 8, y, llr, ws, h=h)
    torch.cuda.synchronize()
    got = split_llr(llr.cpu().numpy(), QAM256, 8)
    for i, r in enumerate(ref):
        exp = receiver.lmmse_demap(r["y32"], hls[i], r["n0_32"], r["desc"], 8)
        for u in range(exp.shape[0]):
            assert rel_err(got[i][u], exp[u]) < 1e-5, (i, u)
            assert np.all(got[i][u][..., r["desc"].bits_per_sym[u]:] == 0)
        assert np.all(got[i][:, list(nr.DMRS_SYMBOLS)] == 0)


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_256qam_all_outputs(prec, tol):
    # m_max = 8: the second readout layer's eight columns all reach a UE's LLRs
    shapes = [dict(s) for s in QAM256]
    net, m_max = cgnn.NetConfig(16, 128, 3, 2, 8), 8
    log(f"nrx_forward: 256-QAM network (m_max 8, 16 antennas), prec={prec}")
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 32, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), 32, perturb=True)
    exp = oracle_nrx(w, net, ref_slots)
    assert any(np.abs(e[..., 7]).max() > 0 for e in exp)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
    try:
        descs, sz = L.make_slots(shapes, m_max)
        y = dev(pack_complex([r["y32"] for r in ref_slots]))
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        for v in (1, 7, 10):
            L.set_all_conv_variants(model, v)
            llr.fill_(float("nan"))
            L.nrx_forward(model, dev(w), descs, y, llr, ws)
            torch.cuda.synchronize()
            got = split_llr(llr.cpu().numpy(), shapes, m_max)
            worst = 0.0
            for i in range(len(shapes)):
                worst = max(worst, check_llr(got[i], exp[i], tol))
            log(f"  conv variant {v}: worst relative error {worst:.2e}")
    finally:
        L.nrx_model_destroy(model)


def _uneven_batch(n, seed):
    """A small batch drawn like the uneven mixed workload: PRBs, UEs, antennas and modulations per slot."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        U = int(rng.integers(1, 5))
        out.append(dict(n_prb=int(rng.integers(4, 13)), n_ant=int(rng.choice([4, 8, 16])), n_ue=U,
                        bits=[int(b) for b in rng.choice([2, 4, 6, 8], size=U)], slot_number=int(rng.integers(0, 20))))
    return out


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_uneven_mixed_batch(prec, tol):
    # the uneven workload's network (d = 128, 6 blocks, 2 rounds, 16-antenna input, m_max = 8) on
    # six slots of 4-12 PRB, 1-4 UEs, 4/8/16 antennas and QPSK-256-QAM, SNR 0-30 dB
    shapes = _uneven_batch(6, 4)
    log(f"nrx_forward: uneven mixed batch {[(s['n_prb'], s['n_ant'], s['n_ue'], s['bits']) for s in shapes]}")
    cfg = dict(SIMCFG, snr=(0.0, 30.0))
    net, m_max = cgnn.NetConfig(16, 128, 6, 2, 8), 8
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(cfg), 41, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), 41, perturb=True)
    exp = oracle_nrx(w, net, ref_slots)
    for flags in (0, 1):   # eager and hipGraph replay
        model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec, flags=flags)
        try:
            descs, sz = L.make_slots(shapes, m_max)
            y = dev(pack_complex([r["y32"] for r in ref_slots]))
            llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
            ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
            for v in ((1, 7, 10) if flags == 0 else (7,)):
                L.set_all_conv_variants(model, v)
                for rep in range(1 + flags):
                    llr.fill_(float("nan"))
                    L.nrx_forward(model, dev(w), descs, y, llr, ws)
                    torch.cuda.synchronize()
                    got = split_llr(llr.cpu().numpy(), shapes, m_max)
                    worst = 0.0
                    for i in range(len(shapes)):
                        worst = max(worst, check_llr(got[i], exp[i], tol))
                    log(f"  flags {flags} conv variant {v} pass {rep}: worst relative error {worst:.2e}")
        finally:
            L.nrx_model_destroy(model)


def test_nan_slot_falls_back_to_lmmse():
    """A received sample that is not finite in one slot: only that slot is flagged (bit 2, the input check: the
    network's ReLUs map a NaN to 0, so its LLRs may stay finite), nrx_fallback_lmmse gives
    it the LS + LMMSE LLRs (what LMMSE cannot produce either -- the REs of that sample -- written as 0), and
    the other slots keep their NRX LLRs bit for bit."""
    shapes = [dict(n_prb=4, n_ant=4, n_ue=2, bits=[4, 4], slot_number=s) for s in range(3)]
    net, m_max = cgnn.NetConfig(4, 128, 2, 1, 4), 4
    ref = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 51, 0, m_max)
    bad_slot, s_bad, t_bad, b_bad = 1, 9, 5, 1          # a data RE (symbol 5), antenna 1
    assert t_bad not in nr.DMRS_SYMBOLS
    ref[bad_slot]["y32"] = ref[bad_slot]["y32"].copy()
    ref[bad_slot]["y32"][s_bad, t_bad, b_bad] = np.nan
    w = synth.he_weights(cgnn.layout(net), 51, perturb=True)
    n0 = np.array([r["n0_32"] for r in ref], dtype=np.float32)
    for prec in (L.NRX_FP32, L.NRX_BF16):
        log(f"fallback: NaN in slot {bad_slot}, prec {prec}")
        model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec, flags=1)
        try:
            descs, sz = L.make_slots(shapes, m_max)
            y = dev(pack_complex([r["y32"] for r in ref]))
            llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
            ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
            lws = ws_tensor(L.lmmse_workspace_bytes(descs))
            flags = torch.full((len(shapes),), 7, dtype=torch.int32, device="cuda")
            for rep in range(2):    # the graph replay clears the flags of the previous pass
                L.nrx_forward(model, dev(w), descs, y, llr, ws)
                L.nrx_slot_flags(model, descs, ws, flags)
                torch.cuda.synchronize()
                f = flags.cpu().tolist()
                # bit 2: a received sample is not finite (bit 0 too if a NaN reaches the LLRs)
                assert f[0] == 0 and f[2] == 0 and (f[bad_slot] & 4), f
            before = llr.cpu().numpy().copy()
            nrx_got = split_llr(before, shapes, m_max)
            assert all(np.all(np.isfinite(nrx_got[i])) for i in (0, 2))
            L.nrx_fallback_lmmse(descs, m_max, y, flags, llr, lws, n0=dev(n0))
            torch.cuda.synchronize()
            after = llr.cpu().numpy()
            got = split_llr(after, shapes, m_max)
            for i in (0, 2):
                assert np.array_equal(got[i], nrx_got[i])
            r = ref[bad_slot]
            with np.errstate(invalid="ignore"):
                exp = receiver.lmmse_demap(r["y32"], receiver.ls_estimate(r["y32"], r["desc"]), r["n0_32"], r["desc"],
                                           m_max)
            assert not np.all(np.isfinite(exp))
            exp = np.where(np.isfinite(exp), exp, 0.0)
            assert np.all(np.isfinite(got[bad_slot]))
            for u in range(2):
                assert rel_err(got[bad_slot][u], exp[u]) <= 1e-5, u
            # the erased entries are exactly those of the sample's RE
            assert np.all(got[bad_slot][:, t_bad, s_bad, :] == 0)
        finally:
            L.nrx_model_destroy(model)
