"""GPU parity of the persistent forward (model flags bit 3): one launch for every layer of every slot.

It runs the same convolution, message-passing and readout bodies as the per-layer launches (ring conv
shape and schedule of variant 14 everywhere), so its LLRs equal those of the per-layer pass bit for bit; both are also
checked against the oracle.  Uneven batches (PRBs, UEs, antennas, modulations), a full-band batch that
spans several slot groups, and hipGraph replays."""
import numpy as np
import pytest

from nrx_cases import check_llr, log, oracle_batch, oracle_nrx, pack_complex, sim_cfg_oracle, split_llr
from oracle import cgnn
from paper_2409_02912_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
L = pytest.importorskip("paper_2409_02912_amd.libnrx")

SIMCFG = dict(n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0, snr=(0.0, 30.0))
RING_VARIANT = 14   # the per-layer kernels with the persistent kernel's conv shape and schedule


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _uneven(n, seed, max_prb):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        U = int(rng.integers(1, 5))
        out.append(dict(n_prb=int(rng.integers(1, max_prb + 1)), n_ant=int(rng.choice([4, 8, 16])), n_ue=U,
                        bits=[int(b) for b in rng.choice([2, 4, 6, 8], size=U)], slot_number=int(rng.integers(0, 20))))
    return out


def _run(shapes, w, net, m_max, flags, y, reps=1):
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, L.NRX_BF16, flags=flags)
    try:
        L.set_all_conv_variants(model, RING_VARIANT)
        descs, sz = L.make_slots(shapes, m_max)
        ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device="cuda")
        llr = torch.empty(sz["llr"], dtype=torch.float32, device="cuda")
        outs, fl = [], torch.full((len(shapes),), -1, dtype=torch.int32, device="cuda")
        for rep in range(reps):
            log(f"  nrx_forward flags={flags} pass {rep} ({len(shapes)} slots)")
            llr.fill_(float("nan"))
            L.nrx_forward(model, w, descs, y, llr, ws)
            L.nrx_slot_flags(model, descs, ws, fl)
            torch.cuda.synchronize()
            outs.append(llr.cpu().numpy().copy())
            assert fl.cpu().numpy().tolist() == [0] * len(shapes), fl.cpu().numpy()
        lat = torch.zeros(len(shapes), dtype=torch.float32, device="cuda")
        L.nrx_slot_latency(model, descs, ws, lat)
        torch.cuda.synchronize()
        return outs, lat.cpu().numpy()
    finally:
        L.nrx_model_destroy(model)


@pytest.mark.parametrize("seed", [3, 8])
def test_persistent_forward_uneven_batch(seed):
    shapes = _uneven(7, seed, 14)
    log(f"persistent forward, uneven batch {[(s['n_prb'], s['n_ant'], s['n_ue'], s['bits']) for s in shapes]}")
    net, m_max = cgnn.NetConfig(16, 128, 6, 2, 8), 8
    ref = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 60 + seed, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), 60 + seed, perturb=True)
    exp = oracle_nrx(w, net, ref)
    y = dev(pack_complex([r["y32"] for r in ref]))
    wd = dev(w)
    layer, _ = _run(shapes, wd, net, m_max, 0, y)
    pers, _ = _run(shapes, wd, net, m_max, 8, y, reps=2)
    graph, _ = _run(shapes, wd, net, m_max, 8 | 1, y, reps=3)
    for k, got in enumerate(pers + graph):
        assert np.array_equal(got, layer[0]), (k, float(np.nanmax(np.abs(got - layer[0]))))
    g = split_llr(pers[0], shapes, m_max)
    worst = max(check_llr(g[i], exp[i], 2e-2) for i in range(len(shapes)))
    log(f"  persistent == per-layer bit for bit; worst relative error against the oracle {worst:.2e}")


def test_persistent_forward_full_band_groups():
    # full-band slots of the headline shape: several 512-row tiles per slot and several slot groups,
    # checked bit for bit against the per-layer pass and on sampled REs against the oracle
    shapes = [dict(n_prb=273, n_ant=8, n_ue=4, bits=[4, 4, 4, 4], slot_number=i) for i in range(3)]
    shapes += [dict(n_prb=10, n_ant=8, n_ue=3, bits=[2, 4, 4], slot_number=7)]
    net, m_max = cgnn.NetConfig(8, 128, 6, 2, 4), 4
    log("persistent forward, 3 x 273 PRB + 10 PRB")
    cfg = L.sim_config(n_taps=12, tap_decay_ns=487.42, snr_db_lo=10, snr_db_hi=10)
    descs, sz = L.make_slots(shapes, m_max)
    y = torch.empty(2 * sz["y"], dtype=torch.float32, device="cuda")
    sws = torch.empty(L.slot_sim_workspace_bytes(cfg, descs), dtype=torch.uint8, device="cuda")
    L.slot_sim(cfg, 7, 0, descs, m_max, y, sws)
    w = synth.he_weights(cgnn.layout(net), 7, perturb=True)
    wd = dev(w)
    layer, _ = _run(shapes, wd, net, m_max, 0, y)
    pers, lat = _run(shapes, wd, net, m_max, 8 | 1, y, reps=2)
    for got in pers:
        assert np.array_equal(got, layer[0])
    log(f"  per-slot completion (us): {np.round(lat, 1).tolist()}")
    # the slot groups finish one after another
    assert lat[0] < lat[-1]
    # oracle on one slot (the 10-PRB one, whole) for the absolute check
    yc = y.cpu().numpy().view(np.complex64)
    o = int(descs[3].y_offset)
    S = 12 * 10
    ys = yc[o:o + S * 14 * 8].reshape(S, 14, 8).astype(np.complex128)
    from oracle import receiver, slot_sim
    d = slot_sim.SlotDesc(10, 8, 3, [2, 4, 4], slot_number=7)
    W = cgnn.unflatten(w.astype(np.float64), net)
    exp = cgnn.forward(W, net, ys, receiver.ls_estimate(ys, d), d.bits_per_sym)
    got = split_llr(pers[0], shapes, m_max)[3]
    err = check_llr(got, exp, 2e-2)
    log(f"  10-PRB slot against the oracle: {err:.2e}")
