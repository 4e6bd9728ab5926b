"""GPU parity: every libnrx entry point against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from nrx_cases import (check_llr, log, oracle_batch, oracle_nrx, pack_bits, pack_complex, rel_err, sim_cfg_oracle,
                       split_h, split_llr)
from oracle import cgnn, nr, receiver
from paper_2409_02912_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
L = pytest.importorskip("paper_2409_02912_amd.libnrx")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda")


def ws_tensor(nbytes):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


RAGGED = [dict(n_prb=4, n_ant=4, n_ue=2, bits=[4, 4], slot_number=3),
          dict(n_prb=7, n_ant=8, n_ue=3, bits=[2, 4, 6], slot_number=7, n_id=5),
          dict(n_prb=5, n_ant=8, n_ue=4, bits=[6, 6, 2, 4], slot_number=11, n_scid=1),
          dict(n_prb=1, n_ant=2, n_ue=1, bits=[6], slot_number=19)]
SIMCFG = dict(n_taps=12, decay_ns=487.42, doppler=100.0, rho=0.5, snr=(0.0, 20.0))


@pytest.mark.parametrize("offsets", [None, [0.0, -3.5, 6.0, 12.25]])
def test_slot_sim_matches_oracle(offsets):
    # offsets: per-slot SNR offsets in dB (mixed-MCS training, Sec. III-A) added to the drawn SNR
    log(f"slot_sim: ragged 4 slots, SNR offsets {offsets}")
    shapes = RAGGED if offsets is None else [dict(sh, snr_offset_db=o) for sh, o in zip(RAGGED, offsets)]
    cfg_o = sim_cfg_oracle(SIMCFG)
    ref = oracle_batch(shapes, cfg_o, 1234, 7, 6)
    descs, sz = L.make_slots(shapes, 6)
    cfg = L.sim_config(n_taps=12, tap_decay_ns=487.42, doppler_max_hz=100.0, rho=0.5, snr_db_lo=0, snr_db_hi=20)
    y = torch.zeros(2 * sz["y"], dtype=torch.float32, device="cuda")
    h = torch.zeros(2 * sz["h"], dtype=torch.float32, device="cuda")
    bits = torch.zeros(sz["bits"], dtype=torch.uint8, device="cuda")
    snr = torch.zeros(len(RAGGED), dtype=torch.float32, device="cuda")
    n0 = torch.zeros(len(RAGGED), dtype=torch.float32, device="cuda")
    ws = ws_tensor(L.slot_sim_workspace_bytes(cfg, descs))
    L.slot_sim(cfg, 1234, 7, descs, 6, y, ws, h_true=h, bits=bits, snr_db=snr, n0=n0)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy(), pack_bits(ref))
    assert np.allclose(snr.cpu().numpy(), [r["snr_db"] for r in ref], atol=1e-4)
    assert np.allclose(n0.cpu().numpy(), [r["n0"] for r in ref], rtol=1e-5)
    yc = y.cpu().numpy().view(np.complex64)
    hc = split_h(h.cpu().numpy().view(np.complex64), RAGGED)
    o = 0
    for i, r in enumerate(ref):
        n = r["y"].size
        assert rel_err(yc[o:o + n].reshape(r["y"].shape), r["y"]) < 2e-5, i
        assert rel_err(hc[i], r["h"]) < 2e-5, i
        o += n


def _upload_batch(shapes, ref):
    y = dev(pack_complex([r["y32"] for r in ref]))
    return y


def test_ls_estimate_matches_oracle():
    log("ls_estimate: ragged 4 slots")
    ref = oracle_batch(RAGGED, sim_cfg_oracle(SIMCFG), 99, 0, 6)
    descs, sz = L.make_slots(RAGGED, 6)
    y = _upload_batch(RAGGED, ref)
    h = torch.zeros(2 * sz["h"], dtype=torch.float32, device="cuda")
    ws = ws_tensor(L.lmmse_workspace_bytes(descs))
    L.nrx_ls_estimate(descs, y, h, ws)
    torch.cuda.synchronize()
    hc = split_h(h.cpu().numpy().view(np.complex64), RAGGED)
    for i, r in enumerate(ref):
        assert rel_err(hc[i], receiver.ls_estimate(r["y32"], r["desc"])) < 1e-6, i


@pytest.mark.parametrize("internal_ls", [False, True])
def test_lmmse_matches_oracle(internal_ls):
    log(f"lmmse_demap: ragged 4 slots, internal_ls={internal_ls}")
    ref = oracle_batch(RAGGED, sim_cfg_oracle(SIMCFG), 5, 1, 6)
    shapes = [dict(s, n0=r["n0_32"]) for s, r in zip(RAGGED, ref)]
    descs, sz = L.make_slots(shapes, 6)
    y = _upload_batch(RAGGED, ref)
    hls = [receiver.ls_estimate(r["y32"], r["desc"]) for r in ref]
    h = None if internal_ls else dev(pack_complex(hls))
    llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
    ws = ws_tensor(L.lmmse_workspace_bytes(descs))
    L.lmmse_demap(descs, 6, y, llr, ws, h=h)
    torch.cuda.synchronize()
    got = split_llr(llr.cpu().numpy(), RAGGED, 6)
    for i, r in enumerate(ref):
        exp = receiver.lmmse_demap(r["y32"], hls[i], r["n0_32"], r["desc"], 6)
        for u in range(exp.shape[0]):
            assert rel_err(got[i][u], exp[u]) < 1e-5, (i, u)
        assert np.all(got[i][:, list(nr.DMRS_SYMBOLS)] == 0)


def _nrx_case(shapes, net, prec, seed, tol, m_max, variants=(0,)):
    log(f"nrx_forward: prec={prec} B={net.B} C={net.C} R={net.R} slots={len(shapes)} variants={variants}")
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), seed, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), seed, perturb=True)
    exp = oracle_nrx(w, net, ref_slots)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
    try:
        descs, sz = L.make_slots(shapes, m_max)
        y = _upload_batch(shapes, ref_slots)
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        hls = torch.zeros(2 * sz["h"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        for v in variants:
            L.set_all_conv_variants(model, v)
            llr.zero_()
            L.nrx_forward(model, dev(w), descs, y, llr, ws, h_ls=hls)
            torch.cuda.synchronize()
            got = split_llr(llr.cpu().numpy(), shapes, m_max)
            worst = 0
            for i in range(len(shapes)):
                worst = max(worst, check_llr(got[i], exp[i], tol))
            log(f"  conv variant {v}: worst relative error {worst:.2e}")
        hc = split_h(hls.cpu().numpy().view(np.complex64), shapes)
        for i, r in enumerate(ref_slots):
            assert rel_err(hc[i], receiver.ls_estimate(r["y32"], r["desc"])) < 1e-6
    finally:
        L.nrx_model_destroy(model)


C1 = [dict(n_prb=4, n_ant=4, n_ue=1, bits=[2], slot_number=i) for i in range(16)]


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
@pytest.mark.parametrize("d", [32, 128])
def test_nrx_forward_single_ue(prec, tol, d):
    # the single-UE workload at its own width (32) and at 128; the StateInit input has 32 channels,
    # one bf16 K chunk (odd count) for the LDS-operand variants
    _nrx_case(C1, cgnn.NetConfig(4, d, 2, 0, 2), prec, 0, tol, 2, variants=(0, 5, 6, 7, 8))


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_reduced_width_multi_ue(prec, tol):
    # d = 64 with message passing: [h, agg] inputs map to two 128-wide segments of 64 live channels
    shapes = [s for s in RAGGED if s["n_ant"] <= 8]
    _nrx_case(shapes, cgnn.NetConfig(8, 64, 3, 2, 6), prec, 4, tol, 6, variants=(1, 5, 7, 8))


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_ragged_multi_ue(prec, tol):
    shapes = [s for s in RAGGED if s["n_ant"] <= 8]
    _nrx_case(shapes, cgnn.NetConfig(8, 128, 3, 2, 6), prec, 3, tol, 6, variants=tuple(range(15)))


def test_bce_and_adam_match_oracle():
    log("nrx_bce / nrx_adam")
    shapes = RAGGED[:3]
    ref = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 11, 0, 6)
    descs, sz = L.make_slots(shapes, 6)
    rng = np.random.default_rng(0)
    llr_np = (3 * rng.standard_normal(sz["llr"])).astype(np.float32)
    llr = dev(llr_np)
    bits = dev(pack_bits(ref))
    dllr = torch.zeros_like(llr)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    nerr = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = ws_tensor(L.nrx_bce_workspace_bytes(descs, 6))
    L.nrx_bce(descs, 6, llr, bits, dllr, loss, nerr, ws)
    torch.cuda.synchronize()
    parts = split_llr(llr_np.astype(np.float64), shapes, 6)
    tot, n, errs, grads = 0.0, 0, 0, []
    for i, r in enumerate(ref):
        lab, msk = cgnn.bit_labels_grid(r["bits"], r["desc"].n_sc, 6)
        valid = msk * (np.arange(6) < np.array(r["desc"].bits_per_sym)[:, None, None, None])
        tot += cgnn.bce_terms(parts[i], lab, valid).sum()
        n += valid.sum()
        errs += int((((parts[i] > 0) != (lab > 0.5)) * valid).sum())
        grads.append((lab, valid))
    assert abs(loss.item() - tot / n) <= 1e-12 * abs(tot / n)
    assert int(nerr.item()) == errs
    g = split_llr(dllr.cpu().numpy().astype(np.float64), shapes, 6)
    for i in range(len(ref)):
        lab, valid = grads[i]
        assert rel_err(g[i], cgnn.bce_grad(parts[i], lab, valid, n)) < 1e-6
    # Adam
    wv = rng.standard_normal(1000).astype(np.float32)
    gv = rng.standard_normal(1000).astype(np.float32)
    mv = (0.1 * rng.standard_normal(1000)).astype(np.float32)
    vv = np.abs(rng.standard_normal(1000)).astype(np.float32)
    tw, tg, tm, tv = dev(wv), dev(gv), dev(mv), dev(vv)
    L.nrx_adam(tw, tg, tm, tv, 3, lr=1e-3)
    torch.cuda.synchronize()
    ew, em, ev = cgnn.adam_step(wv.astype(np.float64), gv, mv, vv, 3)
    assert np.allclose(tw.cpu().numpy(), ew, rtol=0, atol=1e-6)
    assert np.allclose(tm.cpu().numpy(), em, rtol=1e-6, atol=1e-7)
    assert np.allclose(tv.cpu().numpy(), ev, rtol=1e-6, atol=1e-7)


def _away_from_kinks(w, net, ref_slots, sigmas=5.0, iters=4, all_iters=False):
    """Weights whose ReLU units all lie far from their kink on this batch.

    The gradient of a ReLU network jumps where a pre-activation crosses zero.  The fp32 path sums in another
    order than the fp64 oracle, which moves pre-activations by about 1e-6 of their scale, so a unit that close
    to zero can take the other branch; one such unit moves the whole gradient by about 1e-3.  Here the bias in
    front of every ReLU (LayerNorm beta, the first bias of the message and readout MLPs) is set per channel so
    that the channel's pre-activations over the batch sit at +-`sigmas` standard deviations (signs alternate
    over channels, so both branches are taken), iterated because each layer's inputs depend on the earlier
    biases (with all_iters, over the readouts after every CGNN iteration).  Returns the weights and the smallest
    |pre-activation| relative to its layer's RMS."""
    w = w.astype(np.float64).copy()
    offs, off = {}, 0
    for name, shape in cgnn.layout(net):
        offs[name] = off
        off += int(np.prod(shape))
    sign = np.where(np.arange(net.d) % 2 == 0, 1.0, -1.0)
    units = [(f"blk{i}", f"blk{i}.ln.b", 1) for i in range(net.C)] + \
            [(f"mp{r}", f"mp{r}.b1", 1) for r in range(net.R)] + [("readout", "readout.b1", 1)]
    if getattr(net, "chest", False):
        units.append(("readout_ch", "readout_ch.b1", 1))
    if getattr(net, "var_io", False):
        units = [x for x in units if x[0] != "readout"] + [(f"readout_m{m}", f"readout.m{m}.b1", m)
                                                           for m in net.mods()]
    margin = 0.0
    for it in range(iters + 1):
        W = cgnn.unflatten(w, net)
        pre = {k: [] for k, _, _ in units}
        for r in ref_slots:
            h = receiver.ls_estimate(r["y32"], r["desc"])
            _, cache = cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, keep=True, all_iters=all_iters)
            for k, _, j in units:
                if k == "readout":
                    pre[k] += [rc[1].reshape(-1, net.d) for _, rc in cache["readouts"]]
                elif k == "readout_ch":
                    pre[k] += [cc[1].reshape(-1, net.d) for cc in cache["chest"]]
                elif k.startswith("readout_m"):   # Var-IO: the rows of this modulation's UEs
                    us = [u for u, b in enumerate(r["desc"].bits_per_sym) if b == j]
                    pre[k] += [rc[1][:, :, us].reshape(-1, net.d) for _, rc in cache["readouts"]]
                else:
                    pre[k].append(cache[k][j].reshape(-1, net.d))
        margin = np.inf
        for k, bname, _ in units:
            if not sum(len(x) for x in pre[k]):
                continue                                 # a Var-IO modulation no UE of the batch uses
            x = np.concatenate(pre[k])
            b = w[offs[bname]:offs[bname] + net.d]
            x0 = x - b                                   # the pre-activation without its bias
            margin = min(margin, float(np.min(np.abs(x)) / np.sqrt(np.mean(x0 * x0))))
            if it < iters:
                w[offs[bname]:offs[bname] + net.d] = -x0.mean(axis=0) + sign * sigmas * x0.std(axis=0)
    return w.astype(np.float32), margin


def _grad_case(prec, tol, cos_min, seed=21, variant=1, multi=False):
    shapes = [dict(n_prb=4, n_ant=4, n_ue=2, bits=[4, 2], slot_number=1),
              dict(n_prb=3, n_ant=4, n_ue=3, bits=[4, 4, 2], slot_number=2)]
    m_max = 4
    net = cgnn.NetConfig(4, 128, 4, 2, m_max) if multi else cgnn.NetConfig(4, 128, 3, 1, m_max)
    n_ro = len(cgnn.iteration_ends(net)) if multi else 1
    log(f"nrx_backward: prec={prec} slots={len(shapes)} C={net.C} R={net.R} conv variant {variant} readouts {n_ro}")
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), seed, 0, m_max)
    w, margin = _away_from_kinks(synth.he_weights(cgnn.layout(net), seed, perturb=True), net, ref_slots,
                                 all_iters=multi)
    log(f"  smallest |ReLU input| / layer RMS {margin:.2e}")
    assert margin > 1e-4   # a hundred times the ~1e-6 displacement by rounding
    W = cgnn.unflatten(w.astype(np.float64), net)
    rng = np.random.default_rng(seed)
    descs, sz = L.make_slots(shapes, m_max)
    stride = sz["llr"]
    dllr_np = rng.standard_normal(n_ro * stride).astype(np.float32)
    dparts = [split_llr(dllr_np[k * stride:(k + 1) * stride].astype(np.float64), shapes, m_max) for k in range(n_ro)]
    G = {k: np.zeros_like(v) for k, v in W.items()}
    for i, r in enumerate(ref_slots):
        h = receiver.ls_estimate(r["y32"], r["desc"])
        _, cache = cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, keep=True, all_iters=multi)
        g = cgnn.backward(W, net, cache, [dparts[k][i] for k in range(n_ro)] if multi else dparts[0][i])
        for k in G:
            G[k] += g[k]
    ref = cgnn.flatten(G, net)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
    try:
        y = _upload_batch(shapes, ref_slots)
        llr = torch.zeros(n_ro * stride, dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs, save_acts=True))
        dw = torch.full((len(w),), float("nan"), dtype=torch.float32, device="cuda")
        wt = dev(w)
        L.set_all_conv_variants(model, variant)
        if multi:
            L.nrx_forward_iters(model, wt, descs, y, llr, stride, ws, save_acts=True)
            L.nrx_backward_iters(model, wt, descs, dev(dllr_np), stride, dw, ws)
        else:
            L.nrx_forward(model, wt, descs, y, llr, ws, save_acts=True)
            L.nrx_backward(model, wt, descs, dev(dllr_np), dw, ws)
        torch.cuda.synchronize()
        got = dw.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got)), "gradient entries left unwritten"
        e = rel_err(got, ref)
        log(f"  gradient relative error (all weights) {e:.2e}")
        off = 0
        worst = (0.0, 1.0, "")
        for name, shape in cgnn.layout(net):
            n = int(np.prod(shape))
            et = rel_err(got[off:off + n], ref[off:off + n])
            cos = float(got[off:off + n] @ ref[off:off + n] /
                        (np.linalg.norm(got[off:off + n]) * np.linalg.norm(ref[off:off + n]) + 1e-300))
            assert et <= tol and cos >= cos_min, f"{name}: relative error {et:.3e}, cosine {cos:.5f}"
            if et > worst[0]:
                worst = (et, cos, name)
            off += n
        log(f"  worst tensor {worst[2]}: relative error {worst[0]:.3e}, cosine {worst[1]:.6f}")
        assert e <= tol
    finally:
        L.nrx_model_destroy(model)


@pytest.mark.parametrize("variant", [1, 4, 5, 6, 7, 8])
def test_nrx_backward_fp32_matches_oracle(variant):
    _grad_case(0, 1e-4, 0.9999999, variant=variant)


VARIO_SHAPES = [dict(n_prb=4, n_ant=4, n_ue=2, bits=[4, 2], slot_number=1),
                dict(n_prb=3, n_ant=4, n_ue=3, bits=[6, 4, 2], slot_number=2)]
# slots of one modulation each beside a mixed one: each modulation's StateInit and readout launches walk only
# the tiles of the slots with a UE of that modulation
VARIO_SLOT_SHAPES = [dict(n_prb=4, n_ant=4, n_ue=2, bits=[2, 2], slot_number=3),
                     dict(n_prb=3, n_ant=4, n_ue=3, bits=[4, 4, 4], slot_number=4),
                     dict(n_prb=5, n_ant=4, n_ue=1, bits=[8], slot_number=5),
                     dict(n_prb=2, n_ant=4, n_ue=2, bits=[6, 2], slot_number=6)]


@pytest.mark.parametrize("shapes", ["mixed", "per_slot"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_var_io_matches_oracle(prec, tol, shapes):
    """Var-IO (Sec. III, Fig. 2): one StateInit and one ReadoutLLRs per modulation (2, 4, 6, 8 bits), each UE's
    state initialised and read out by its own.  "mixed": every slot mixes QPSK, 16-QAM and 64-QAM UEs, the 256-QAM
    layers are unused; "per_slot": most slots use one modulation, so each modulation's launches cover a subset of
    the slots (also with the pass replayed as a hipGraph)."""
    shp = VARIO_SHAPES if shapes == "mixed" else VARIO_SLOT_SHAPES
    net = cgnn.NetConfig(4, 128, 3, 1, 8, var_io=True)
    log(f"Var-IO forward: prec={prec}, {shapes} modulations")
    ref_slots = oracle_batch(shp, sim_cfg_oracle(SIMCFG), 61, 0, 8)
    w = synth.he_weights(cgnn.layout(net), 61, perturb=True)
    exp = oracle_nrx(w, net, ref_slots)
    descs, sz = L.make_slots(shp, 8)
    y = _upload_batch(shp, ref_slots)
    for flags in ((4,) if shapes == "mixed" else (4, 4 | 1)):
        model = L.nrx_model_create(net.B, net.d, net.C, net.R, 8, prec, flags=flags)
        try:
            assert [(n, tuple(s)) for n, _, s in L.weight_layout(model)] == [(n, tuple(s)) for n, s in cgnn.layout(net)]
            llr = torch.full((sz["llr"],), float("nan"), dtype=torch.float32, device="cuda")
            ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
            for rep in range(2 if flags & 1 else 1):
                llr.fill_(float("nan"))
                L.nrx_forward(model, dev(w), descs, y, llr, ws)
                torch.cuda.synchronize()
                got = llr.cpu().numpy().astype(np.float64)
                assert np.all(np.isfinite(got)), "LLR entries left unwritten"
                e = rel_err(np.concatenate([x.reshape(-1) for x in split_llr(got, shp, 8)]),
                            np.concatenate([x.reshape(-1) for x in exp]))
                log(f"  flags {flags} pass {rep}: LLR relative error {e:.2e}")
                assert e <= tol
        finally:
            L.nrx_model_destroy(model)


def test_nrx_backward_var_io_fp32_matches_oracle():
    """Var-IO gradient: each modulation's StateInit and readout learn from their own UEs only; the unused ones get
    zero."""
    net = cgnn.NetConfig(4, 128, 3, 1, 8, var_io=True)
    m_max = 8
    log("Var-IO backward: fp32")
    ref_slots = oracle_batch(VARIO_SHAPES, sim_cfg_oracle(SIMCFG), 67, 0, m_max)
    w, margin = _away_from_kinks(synth.he_weights(cgnn.layout(net), 67, perturb=True), net, ref_slots)
    log(f"  smallest |ReLU input| / layer RMS {margin:.2e}")
    assert margin > 1e-4
    W = cgnn.unflatten(w.astype(np.float64), net)
    rng = np.random.default_rng(67)
    descs, sz = L.make_slots(VARIO_SHAPES, m_max)
    dllr_np = rng.standard_normal(sz["llr"]).astype(np.float32)
    dparts = split_llr(dllr_np.astype(np.float64), VARIO_SHAPES, m_max)
    G = {k: np.zeros_like(v) for k, v in W.items()}
    for i, r in enumerate(ref_slots):
        h = receiver.ls_estimate(r["y32"], r["desc"])
        _, cache = cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, keep=True)
        for k, g in cgnn.backward(W, net, cache, dparts[i]).items():
            G[k] += g
    ref = cgnn.flatten(G, net)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, 0, flags=4)
    try:
        y = _upload_batch(VARIO_SHAPES, ref_slots)
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs, save_acts=True))
        dw = torch.full((len(w),), float("nan"), dtype=torch.float32, device="cuda")
        wt = dev(w)
        L.set_all_conv_variants(model, 7)
        L.nrx_forward(model, wt, descs, y, llr, ws, save_acts=True)
        L.nrx_backward(model, wt, descs, dev(dllr_np), dw, ws)
        torch.cuda.synchronize()
        got = dw.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got)), "gradient entries left unwritten"
        off = 0
        for name, shape in cgnn.layout(net):
            n = int(np.prod(shape))
            if name.startswith("readout.m8.") or name.startswith("conv_in.m8."):
                assert np.all(got[off:off + n] == 0), name
            else:
                et = rel_err(got[off:off + n], ref[off:off + n])
                assert et <= 1e-4, f"{name}: relative error {et:.3e}"
            off += n
        e = rel_err(got, ref)
        log(f"  gradient relative error (all weights) {e:.2e}")
        assert e <= 1e-4
    finally:
        L.nrx_model_destroy(model)


def test_nrx_backward_var_io_chest_multi_loss_fp32_matches_oracle():
    """The training extensions together: Var-IO layers, the double readout and the multi-loss (readouts after both
    CGNN iterations), one gradient against the oracle's."""
    net = cgnn.NetConfig(4, 128, 4, 2, 8, chest=True, var_io=True)
    m_max = 8
    log("Var-IO + double readout + multi-loss backward: fp32")
    ref_slots = oracle_batch(VARIO_SHAPES, sim_cfg_oracle(SIMCFG), 71, 0, m_max)
    w, margin = _away_from_kinks(synth.he_weights(cgnn.layout(net), 71, perturb=True), net, ref_slots,
                                 all_iters=True)
    log(f"  smallest |ReLU input| / layer RMS {margin:.2e}")
    assert margin > 1e-4
    W = cgnn.unflatten(w.astype(np.float64), net)
    rng = np.random.default_rng(71)
    descs, sz = L.make_slots(VARIO_SHAPES, m_max)
    ls_, hs_ = sz["llr"], 2 * sz["h"]
    dllr_np = rng.standard_normal(2 * ls_).astype(np.float32)
    dh_np = rng.standard_normal(2 * hs_).astype(np.float32)
    dl = [split_llr(dllr_np[k * ls_:(k + 1) * ls_].astype(np.float64), VARIO_SHAPES, m_max) for k in range(2)]
    dhc = [split_h(dh_np[k * hs_:(k + 1) * hs_].astype(np.float64).view(np.complex128), VARIO_SHAPES)
           for k in range(2)]
    G = {k: np.zeros_like(v) for k, v in W.items()}
    for i, r in enumerate(ref_slots):
        h = receiver.ls_estimate(r["y32"], r["desc"])
        _, cache = cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, keep=True, all_iters=True)
        for k, g in cgnn.backward(W, net, cache, [dl[j][i] for j in range(2)], [dhc[j][i] for j in range(2)]).items():
            G[k] += g
    ref = cgnn.flatten(G, net)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, 0, flags=6)
    try:
        y = _upload_batch(VARIO_SHAPES, ref_slots)
        llr = torch.zeros(2 * ls_, dtype=torch.float32, device="cuda")
        hest = torch.zeros(2 * hs_, dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs, save_acts=True))
        dw = torch.full((len(w),), float("nan"), dtype=torch.float32, device="cuda")
        wt = dev(w)
        L.set_all_conv_variants(model, 7)
        L.nrx_forward_chest(model, wt, descs, y, llr, hest, ws, llr_stride=ls_, h_stride=hs_, save_acts=True)
        L.nrx_backward_chest(model, wt, descs, dev(dllr_np), dev(dh_np), dw, ws, llr_stride=ls_, h_stride=hs_)
        torch.cuda.synchronize()
        got = dw.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got)), "gradient entries left unwritten"
        off = 0
        for name, shape in cgnn.layout(net):
            n = int(np.prod(shape))
            if ".m8." in name:
                assert np.all(got[off:off + n] == 0), name
            else:
                et = rel_err(got[off:off + n], ref[off:off + n])
                assert et <= 1e-4, f"{name}: relative error {et:.3e}"
            off += n
        e = rel_err(got, ref)
        log(f"  gradient relative error (all weights) {e:.2e}")
        assert e <= 1e-4
    finally:
        L.nrx_model_destroy(model)


def test_nrx_backward_multi_loss_fp32_matches_oracle():
    # the multi-loss gradient (Sec. II-B): readouts after both CGNN iterations, one dllr each
    _grad_case(0, 1e-4, 0.9999999, variant=7, multi=True)


CHEST_SHAPES = [dict(n_prb=4, n_ant=8, n_ue=2, bits=[4, 2], slot_number=1),
                dict(n_prb=3, n_ant=4, n_ue=3, bits=[4, 4, 2], slot_number=2)]


def _pack_h(parts):
    """Per-slot complex [S, T, U, B] arrays -> the flat interleaved h layout (fp32)."""
    c = np.concatenate([p.reshape(-1) for p in parts])
    return np.stack([c.real, c.imag], axis=-1).reshape(-1).astype(np.float32)


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_chest_forward_matches_oracle(prec, tol):
    """Double readout (Sec. II-A): ReadoutChEst after both CGNN iterations, 16 outputs for the 8-antenna network,
    a 4-antenna slot using the first 8; LLRs of the same pass unchanged."""
    net = cgnn.NetConfig(8, 128, 4, 2, 4, chest=True)
    m_max = 4
    log(f"chest forward: prec={prec} C={net.C} R={net.R}")
    ref_slots = oracle_batch(CHEST_SHAPES, sim_cfg_oracle(SIMCFG), 43, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), 43, perturb=True)
    W = cgnn.unflatten(w.astype(np.float64), net)
    ref_l, ref_h = [], []
    for r in ref_slots:
        h = receiver.ls_estimate(r["y32"], r["desc"])
        ls, cache = cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, keep=True, all_iters=True)
        ref_l.append(ls)
        ref_h.append(cache["hests"])
    descs, sz = L.make_slots(CHEST_SHAPES, m_max)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec, flags=2)
    try:
        assert L.nrx_weight_count(model) == len(w)
        y = _upload_batch(CHEST_SHAPES, ref_slots)
        ls_, hs_ = sz["llr"], 2 * sz["h"]
        llr = torch.zeros(2 * ls_, dtype=torch.float32, device="cuda")
        hest = torch.full((2 * hs_,), float("nan"), dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        L.nrx_forward_chest(model, dev(w), descs, y, llr, hest, ws, llr_stride=ls_, h_stride=hs_)
        torch.cuda.synchronize()
        gl, gh = llr.cpu().numpy().astype(np.float64), hest.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(gh)), "channel-estimate entries left unwritten"
        for k in range(2):
            el = rel_err(np.concatenate([x.reshape(-1) for x in split_llr(gl[k * ls_:(k + 1) * ls_], CHEST_SHAPES,
                                                                        m_max)]),
                         np.concatenate([ref_l[i][k].reshape(-1) for i in range(len(ref_slots))]))
            hk = gh[k * hs_:(k + 1) * hs_]
            eh = rel_err(hk, _pack_h([ref_h[i][k] for i in range(len(ref_slots))]).astype(np.float64))
            log(f"  readout {k}: LLR relative error {el:.2e}, channel estimate {eh:.2e}")
            assert el <= tol and eh <= tol
    finally:
        L.nrx_model_destroy(model)


def test_nrx_backward_chest_fp32_matches_oracle():
    """Double-readout gradient (Sec. II-B): BCE-side dllr and channel-side dh_est after both CGNN iterations."""
    net = cgnn.NetConfig(8, 128, 4, 2, 4, chest=True)
    m_max = 4
    log(f"chest backward: fp32 C={net.C} R={net.R}")
    ref_slots = oracle_batch(CHEST_SHAPES, sim_cfg_oracle(SIMCFG), 47, 0, m_max)
    w, margin = _away_from_kinks(synth.he_weights(cgnn.layout(net), 47, perturb=True), net, ref_slots,
                                 all_iters=True)
    log(f"  smallest |ReLU input| / layer RMS {margin:.2e}")
    assert margin > 1e-4
    W = cgnn.unflatten(w.astype(np.float64), net)
    rng = np.random.default_rng(47)
    descs, sz = L.make_slots(CHEST_SHAPES, m_max)
    ls_, hs_ = sz["llr"], 2 * sz["h"]
    dllr_np = rng.standard_normal(2 * ls_).astype(np.float32)
    dh_np = rng.standard_normal(2 * hs_).astype(np.float32)
    dl = [split_llr(dllr_np[k * ls_:(k + 1) * ls_].astype(np.float64), CHEST_SHAPES, m_max) for k in range(2)]
    dhc = [split_h(dh_np[k * hs_:(k + 1) * hs_].astype(np.float64).view(np.complex128), CHEST_SHAPES)
           for k in range(2)]
    G = {k: np.zeros_like(v) for k, v in W.items()}
    for i, r in enumerate(ref_slots):
        h = receiver.ls_estimate(r["y32"], r["desc"])
        _, cache = cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, keep=True, all_iters=True)
        g = cgnn.backward(W, net, cache, [dl[k][i] for k in range(2)], [dhc[k][i] for k in range(2)])
        for k in G:
            G[k] += g[k]
    ref = cgnn.flatten(G, net)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, 0, flags=2)
    try:
        y = _upload_batch(CHEST_SHAPES, ref_slots)
        llr = torch.zeros(2 * ls_, dtype=torch.float32, device="cuda")
        hest = torch.zeros(2 * hs_, dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs, save_acts=True))
        dw = torch.full((len(w),), float("nan"), dtype=torch.float32, device="cuda")
        wt = dev(w)
        L.set_all_conv_variants(model, 7)
        L.nrx_forward_chest(model, wt, descs, y, llr, hest, ws, llr_stride=ls_, h_stride=hs_, save_acts=True)
        L.nrx_backward_chest(model, wt, descs, dev(dllr_np), dev(dh_np), dw, ws, llr_stride=ls_, h_stride=hs_)
        torch.cuda.synchronize()
        got = dw.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got)), "gradient entries left unwritten"
        off = 0
        for name, shape in cgnn.layout(net):
            n = int(np.prod(shape))
            et = rel_err(got[off:off + n], ref[off:off + n])
            assert et <= 1e-4, f"{name}: relative error {et:.3e}"
            off += n
        e = rel_err(got, ref)
        log(f"  gradient relative error (all weights) {e:.2e}")
        assert e <= 1e-4
        # the plain multi-loss backward after this forward leaves the ReadoutChEst gradient zero
        L.nrx_backward_iters(model, wt, descs, dev(dllr_np), ls_, dw, ws)
        torch.cuda.synchronize()
        g2 = dw.cpu().numpy()
        n_ch = sum(int(np.prod(sh)) for nm, sh in cgnn.layout(net) if nm.startswith("readout_ch"))
        assert np.all(g2[len(w) - n_ch:] == 0) and np.all(np.isfinite(g2))
    finally:
        L.nrx_model_destroy(model)


def test_nrx_mse_matches_oracle():
    """Channel-estimate loss of the double readout (Sec. II-B): MSE over the batch and its gamma-scaled gradient."""
    log("nrx_mse: 2 slots")
    descs, sz = L.make_slots(CHEST_SHAPES, 4)
    rng = np.random.default_rng(5)
    he = rng.standard_normal(2 * sz["h"]).astype(np.float32)
    ht = rng.standard_normal(2 * sz["h"]).astype(np.float32)
    hec = split_h(he.astype(np.float64).view(np.complex128), CHEST_SHAPES)
    htc = split_h(ht.astype(np.float64).view(np.complex128), CHEST_SHAPES)
    mse, g = cgnn.mse_grad(hec, htc, 0.25)
    dh = torch.full((2 * sz["h"],), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = ws_tensor(L.nrx_mse_workspace_bytes(descs))
    L.nrx_mse(descs, dev(he), dev(ht), 0.25, dh, loss, ws)
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - mse) <= 1e-12 * mse
    assert rel_err(dh.cpu().numpy().astype(np.float64), _pack_h(g).astype(np.float64)) <= 1e-6


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_depth_control(prec, tol):
    """Inference-time depth control (Sec. IV-B): the first k CGNN iterations and a readout, against the oracle
    at depth k; and the readouts after every iteration in one pass."""
    shapes = [s for s in RAGGED if s["n_ant"] <= 8]
    net = cgnn.NetConfig(8, 128, 4, 2, 6)
    m_max = 6
    log(f"depth control: prec={prec} C={net.C} R={net.R} iterations {cgnn.iteration_ends(net)}")
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 5, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), 5, perturb=True)
    W = cgnn.unflatten(w.astype(np.float64), net)
    exp = []
    for r in ref_slots:
        h = receiver.ls_estimate(r["y32"], r["desc"])
        exp.append(cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym, all_iters=True))
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
    try:
        assert L.nrx_num_iterations(model) == 2
        descs, sz = L.make_slots(shapes, m_max)
        y = _upload_batch(shapes, ref_slots)
        stride = sz["llr"]
        llr = torch.zeros(2 * stride, dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        wt = dev(w)
        L.set_all_conv_variants(model, 7)
        for k in (1, 2):
            L.nrx_set_iterations(model, k)
            llr.zero_()
            L.nrx_forward(model, wt, descs, y, llr, ws)
            torch.cuda.synchronize()
            got = split_llr(llr[:stride].cpu().numpy(), shapes, m_max)
            worst = max(check_llr(got[i], exp[i][k - 1], tol) for i in range(len(shapes)))
            log(f"  depth {k}: worst relative error {worst:.2e}")
        L.nrx_set_iterations(model, 0)
        llr.zero_()
        L.nrx_forward_iters(model, wt, descs, y, llr, stride, ws)
        torch.cuda.synchronize()
        for k in (0, 1):
            got = split_llr(llr[k * stride:(k + 1) * stride].cpu().numpy(), shapes, m_max)
            worst = max(check_llr(got[i], exp[i][k], tol) for i in range(len(shapes)))
            log(f"  readout after iteration {k + 1} (one pass): worst relative error {worst:.2e}")
        with pytest.raises(L.NrxError):
            L.nrx_set_iterations(model, 3)
    finally:
        L.nrx_model_destroy(model)


def test_nrx_backward_bf16_close_to_oracle():
    # BF16 stores activations and gradients with 8 significant bits (relative rounding up to 2^-9), FP32
    # accumulation; the error grows with the depth the gradient travels back.  Measured: 5.2e-3 over all
    # weights, worst tensor (first block's conv_a weights) 1.0e-2 at cosine 0.99995; the bar is three times
    # the worst tensor
    _grad_case(1, 0.03, 0.9995)


def test_training_reduces_loss():
    """A short run of the training loop (GPU slots, BCE, backward, Adam) learns: the BCE falls from ln 2."""
    from paper_2409_02912_amd.train import Trainer
    log("training: workload t, 400 steps")
    tr = Trainer(synth.WORKLOADS["t"], L.NRX_BF16, seed=5, lr=1e-3)
    try:
        first = None
        for k in range(400):
            tr.train_step()
            if k == 0:
                torch.cuda.synchronize()
                first = tr.loss.item()
        torch.cuda.synchronize()
        last, ber = tr.loss.item(), tr.nerr.item() / tr.n_bits
        log(f"  loss {first:.3f} -> {last:.3f}, ber {ber:.3f}")
        assert first > 0.6 and last < 0.55 and ber < 0.3
    finally:
        tr.close()


def test_multi_loss_training_gives_usable_shallow_readout():
    """Multi-loss training (Sec. II-B) makes the network usable at every depth (Sec. IV-B): after the same number
    of steps, the readout after the first of two CGNN iterations has learned (BCE well below ln 2), the deeper
    readout is no worse, and the shallow readout is better than that of a network trained on the last readout
    alone (same seed, data and steps; measured 0.374 against 0.439 held-out BCE)."""
    from paper_2409_02912_amd.train import Trainer, evaluate
    w = synth.WORKLOADS["t2"]
    res = {}
    for multi in (True, False):
        log(f"training: workload t2 (2 CGNN iterations), 400 steps, multi-loss {multi}")
        tr = Trainer(w, L.NRX_BF16, seed=5, lr=1e-3, multi_loss=multi)
        try:
            for _ in range(400):
                tr.train_step()
            torch.cuda.synchronize()
            res[multi] = [evaluate(tr.params, w, seed=99, batches=2, snr_db=10.0, n_iter=k)["bce_nrx"] for k in (1, 2)]
            log(f"  held-out BCE at depth 1, 2: {res[multi][0]:.3f}, {res[multi][1]:.3f}")
        finally:
            tr.close()
    assert res[True][0] < 0.55 and res[True][1] < res[True][0] + 0.02
    assert res[False][0] > res[True][0] + 0.02


def test_double_readout_training_refines_channel_estimate():
    """Double-readout training (Sec. II-A, II-B): with the gamma-scaled MSE against the true channel, ReadoutChEst
    learns a channel estimate more accurate than the LS estimate with interpolation the network starts from
    (held-out MSE at 10 dB after 2500 steps from scratch, gamma = 1: measured 0.024 against 0.035).  The refined
    estimate is also worth bits to a classical receiver: LMMSE equalisation + max-log demapping given ReadoutChEst's
    estimate makes fewer errors than given the LS estimate (same slots, genie N0; measured BER 0.033 against
    0.041)."""
    from paper_2409_02912_amd.train import Trainer, evaluate_chest
    w = synth.WORKLOADS["t"]
    log("training: workload t, double readout (gamma 1), 2500 steps")
    tr = Trainer(w, L.NRX_BF16, seed=5, lr=1e-3, gamma=1.0)
    try:
        for _ in range(2500):
            tr.train_step()
        torch.cuda.synchronize()
        r = evaluate_chest(tr.params, w, seed=99, batches=2, snr_db=10.0)
    finally:
        tr.close()
    log(f"  held-out channel MSE: ReadoutChEst {r['mse_nrx']:.4f}, LS {r['mse_ls']:.4f}")
    log(f"  LMMSE BER given ReadoutChEst {r['ber_lmmse_refined']:.4f}, given LS {r['ber_lmmse_ls']:.4f}")
    assert r["mse_nrx"] < 0.85 * r["mse_ls"]
    assert r["ber_lmmse_refined"] < r["ber_lmmse_ls"]


@pytest.mark.parametrize("var_io", [False, True])
def test_mixed_mcs_training_learns_every_modulation(var_io):
    """Mixed-MCS training (Sec. III, III-A; U_A drawn per batch, Sec. II-B) of the two Var-MCS receivers: LLR masking
    (one readout with six outputs) and Var-IO (one StateInit and readout per modulation).  Trained on batches of
    random U_A, iid per-UE QPSK / 16-QAM / 64-QAM and modulation-dependent SNR offsets, each detects every
    modulation: held-out BCE per coded bit at 10 dB below 0.12 / 0.30 / 0.45 for both (measured with masking after
    1500 steps 0.056 / 0.242 / 0.396).  The Var-IO input and output layers each see a third of the data, so that
    network trains three times as many steps to the same bound."""
    from paper_2409_02912_amd.train import Trainer, evaluate
    w = synth.WORKLOADS["tm"]
    steps = 6000 if var_io else 2000
    log(f"training: workload tm, mixed MCS (pool of 16 batch shapes), Var-IO {var_io}, {steps} steps")
    tr = Trainer(w, L.NRX_BF16, seed=5, lr=1e-3, mixed_pool=16, var_io=var_io)
    try:
        assert len({tuple(s["n_ue"] for s in e[0]) for e in tr.pool}) > 1   # U_A varies over the batches
        for _ in range(steps):
            tr.train_step()
        torch.cuda.synchronize()
        bce = {b: evaluate(tr.params, w, seed=99, batches=2, snr_db=10.0, bits=b, var_io=var_io)["bce_nrx"]
               for b in w["mcs"]}
    finally:
        tr.close()
    log(f"  held-out BCE per modulation (bits: BCE) {bce}")
    assert bce[2] < 0.12 and bce[4] < 0.30 and bce[6] < 0.45


def test_site_fine_tuning_improves_site_receiver():
    """Site-specific fine-tuning (Sec. V): the committed workload-t weights, trained on the generic channel, fine-tuned
    for 300 steps on a fixed site channel (6 taps of 150 ns decay, array correlation 0.7, UE speeds up to 8 m/s),
    get a lower held-out BCE on that site than before."""
    from paper_2409_02912_amd.train import Trainer, evaluate
    import os
    w0 = np.load(os.path.join(os.path.dirname(L.LIB_PATH), "weights", "nrx_t.npy"), allow_pickle=False)
    site = synth.WORKLOADS["t_site"]
    before = evaluate(w0, site, seed=99, batches=2, snr_db=10.0)["bce_nrx"]
    tr = Trainer(site, L.NRX_BF16, seed=7, lr=1e-3)
    try:
        tr.params.copy_(torch.from_numpy(w0))
        for _ in range(300):
            tr.train_step()
        torch.cuda.synchronize()
        after = evaluate(tr.params, site, seed=99, batches=2, snr_db=10.0)["bce_nrx"]
    finally:
        tr.close()
    log(f"  site held-out BCE: before fine-tuning {before:.3f}, after 300 steps {after:.3f}")
    assert after < before - 0.01


def test_trained_nrx_beats_lmmse():
    """The trained network (committed weights, 12k steps of workload t) against LS + LMMSE on held-out slots."""
    import os
    from paper_2409_02912_amd.train import evaluate
    path = os.path.join(os.path.dirname(L.LIB_PATH), "weights", "nrx_t.npy")
    w = np.load(path, allow_pickle=False)
    log("trained NRX vs LS+LMMSE: workload t, 5 dB, held-out seed")
    r = evaluate(w, synth.WORKLOADS["t"], seed=777, batches=8, snr_db=5.0)
    b1, b2, n = r["ber_nrx"], r["ber_lmmse"], r["n_bits"]
    sd = np.sqrt(b2 * (1 - b2) / n)
    log(f"  BER nrx {b1:.4f}  lmmse {b2:.4f}  bits {n}")
    assert b1 < b2 - 5 * sd


def test_trained_c5_network_against_lmmse():
    """The committed C5 network (6 blocks, 2 message-passing rounds, 4 UEs x 8 antennas, Sec. II-B training) against
    LS + LMMSE with genie N0 at 10 dB on held-out C5 slots.  It does not beat the classical receiver yet (its BER
    is 1.08 times LS + LMMSE on these slots after 908k training steps, still falling with training): the bar
    holds it within 20 % of it, so that a regression of the weights or of the forward pass shows."""
    import os
    from paper_2409_02912_amd.train import evaluate
    w = np.load(os.path.join(os.path.dirname(L.LIB_PATH), "weights", "nrx_c5.npy"), allow_pickle=False)
    log("trained C5 NRX vs LS+LMMSE: 10 dB, held-out seed")
    r = evaluate(w, synth.WORKLOADS["c5"], seed=99, batches=2, snr_db=10.0)
    b1, b2, n = r["ber_nrx"], r["ber_lmmse"], r["n_bits"]
    log(f"  BER nrx {b1:.4f}  lmmse {b2:.4f}  ratio {b1 / b2:.3f}  bits {n}")
    assert b1 < 1.2 * b2


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_graph_replay_matches_eager(prec, tol):
    """Model flag bit 0: the forward pass captured once and replayed on new inputs in the same
    buffers gives the eager result on every replay, with unrelated eager work in between, also
    when the depth changes between replays."""
    shapes = [s for s in RAGGED if s["n_ant"] <= 8]
    net, m_max = cgnn.NetConfig(8, 128, 3, 2, 6), 6
    w = synth.he_weights(cgnn.layout(net), 5, perturb=True)
    eager = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
    graph = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec, flags=1)
    try:
        descs, sz = L.make_slots(shapes, m_max)
        wd = dev(w)
        y = torch.zeros(2 * sz["y"], dtype=torch.float32, device="cuda")
        llr_e = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        llr_g = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws_e = ws_tensor(L.nrx_workspace_bytes(eager, descs))
        ws_g = ws_tensor(L.nrx_workspace_bytes(graph, descs))
        for rep in range(4):
            # replay 2 runs the first CGNN iteration only (a graph of its own); replay 3 reuses the full one
            depth = 1 if rep == 2 else 0
            L.nrx_set_iterations(graph, depth)
            L.nrx_set_iterations(eager, depth)
            log(f"graph replay {rep}: prec={prec} depth {depth or 'all'}")
            ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 11, rep, m_max)
            y.copy_(torch.from_numpy(pack_complex([r["y32"] for r in ref_slots])))
            llr_g.fill_(float("nan"))
            L.nrx_forward(graph, wd, descs, y, llr_g, ws_g)
            junk = torch.randn(1 << 20, device="cuda")
            junk = (junk * 2).sum()
            torch.cuda.synchronize()
            L.nrx_forward(eager, wd, descs, y, llr_e, ws_e)
            torch.cuda.synchronize()
            assert torch.equal(llr_g, llr_e), f"replay {rep} differs from the eager pass"
            if rep in (0, 3):
                exp = oracle_nrx(w, net, ref_slots)
                got = split_llr(llr_g.cpu().numpy(), shapes, m_max)
                for i in range(len(shapes)):
                    check_llr(got[i], exp[i], tol)
    finally:
        L.nrx_model_destroy(eager)
        L.nrx_model_destroy(graph)


def test_slot_latency_stamps():
    """Per-slot completion times from the readout kernel lie inside the forward pass."""
    shapes = synth.ragged_shapes(24, 0, max_prb=64)
    m_max = max(max(s["bits"]) for s in shapes)
    n_ant = max(s["n_ant"] for s in shapes)
    model = L.nrx_model_create(n_ant, 128, 2, 1, m_max, 1)
    try:
        descs, sz = L.make_slots(shapes, m_max)
        w = synth.he_weights([(n, sh) for n, _, sh in L.weight_layout(model)], 1)
        y = torch.randn(2 * sz["y"], dtype=torch.float32, device="cuda")
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        lat = torch.full((len(shapes),), -1.0, dtype=torch.float32, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        L.nrx_forward(model, dev(w), descs, y, llr, ws)
        torch.cuda.synchronize()
        e0.record()
        L.nrx_forward(model, dev(w), descs, y, llr, ws)
        e1.record()
        L.nrx_slot_latency(model, descs, ws, lat)
        torch.cuda.synchronize()
        total_us = e0.elapsed_time(e1) * 1e3
        v = lat.cpu().numpy()
        log(f"slot latency us: min {v.min():.1f} max {v.max():.1f}, forward {total_us:.1f}")
        assert np.all(np.isfinite(v)) and np.all(v > 0)
        assert v.max() <= total_us * 1.05 + 20.0
    finally:
        L.nrx_model_destroy(model)


def test_autograd_function_gradient():
    """NrxFunction: torch autograd through the hand-written backward equals nrx_backward, and a
    central finite difference of the fp32 GPU forward along a random direction matches the
    gradient's directional derivative."""
    from paper_2409_02912_amd.autograd import Nrx
    shapes = [dict(n_prb=4, n_ant=4, n_ue=2, bits=[4, 4], slot_number=s) for s in range(4)]
    net, m_max = cgnn.NetConfig(4, 128, 2, 1, 4), 4
    w = synth.he_weights(cgnn.layout(net), 7, perturb=True)
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 7, 0, m_max)
    y = dev(pack_complex([r["y32"] for r in ref_slots]))
    nrx = Nrx(net.B, net.d, net.C, net.R, m_max, 0, shapes)
    try:
        rng = np.random.default_rng(7)
        r = dev(rng.standard_normal(nrx.sizes["llr"]).astype(np.float32))
        wt = dev(w).requires_grad_(True)
        llr = nrx(wt, y)
        (llr * r).sum().backward()
        g = wt.grad.detach().clone()
        # direct call on the same saved activations
        g2 = torch.empty_like(g)
        L.nrx_backward(nrx.model, wt.detach(), nrx.slots, r, g2, nrx.ws)
        torch.cuda.synchronize()
        assert torch.equal(g, g2)
        v = rng.standard_normal(w.size)
        v /= np.linalg.norm(v)
        rn = r.double().cpu().numpy()

        def loss(wv):
            with torch.no_grad():
                return float(np.dot(nrx(dev(wv.astype(np.float32)), y).double().cpu().numpy(), rn))
        gn = g.double().cpu().numpy()
        # (a) the LLRs are affine in the readout's second-layer weights: a central difference
        # along a direction in that tensor is exact up to rounding, so the step can be large
        off = {n: (o, sh) for n, o, sh in L.weight_layout(nrx.model)}
        o2, sh2 = off["readout.w2"]
        v2 = np.zeros(w.size)
        v2[o2:o2 + int(np.prod(sh2))] = rng.standard_normal(int(np.prod(sh2)))
        v2 /= np.linalg.norm(v2)
        an2 = float(np.dot(gn, v2))
        fd2 = (loss(w + 0.5 * v2) - loss(w - 0.5 * v2)) / 1.0
        log(f"readout.w2 direction: analytic {an2:.6e} finite difference {fd2:.6e}")
        assert abs(fd2 - an2) <= 1e-3 * abs(an2)
        # (b) a random direction through every layer: ReLU kinks bias a large step and the fp32
        # rounding of the forward pass (about 1e-6 of each LLR) swamps a small one; the best of
        # three steps must agree to 5 %
        an = float(np.dot(gn, v))
        errs = []
        for rel in (1e-3, 3e-4, 1e-4):
            eps = rel * float(np.linalg.norm(w))
            fd = (loss(w + eps * v) - loss(w - eps * v)) / (2 * eps)
            errs.append(abs(fd - an) / abs(an))
            log(f"directional derivative: analytic {an:.6e} finite difference {fd:.6e} (eps {eps:.2e})")
        assert min(errs) <= 5e-2
    finally:
        nrx.close()


FP8_TOL = 0.25        # norm-wise LLR error bound of the E4M3 block convs (derivation in the design notes)
FP8_AGREE = 0.99      # hard-decision agreement where |LLR_oracle| > 2


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_nrx_forward_fp8(variant):
    """FP8 model: calibrated per-layer activation scales, E4M3 block convs, LLRs against the
    FP64 oracle (norm-wise error and hard decisions), for each FP8 conv tile shape."""
    shapes = [dict(n_prb=6, n_ant=8, n_ue=4, bits=[4, 4, 4, 4], slot_number=s) for s in range(3)] + \
             [dict(n_prb=5, n_ant=4, n_ue=2, bits=[4, 2], slot_number=7)]
    net, m_max = cgnn.NetConfig(8, 128, 4, 2, 4), 4
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(SIMCFG), 21, 0, m_max)
    w = synth.he_weights(cgnn.layout(net), 21, perturb=True)
    exp = oracle_nrx(w, net, ref_slots)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, L.NRX_FP8)
    try:
        descs, sz = L.make_slots(shapes, m_max)
        y = _upload_batch(shapes, ref_slots)
        wd = dev(w)
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        with pytest.raises(L.NrxError):
            L.nrx_forward(model, wd, descs, y, llr, ws)        # no scales yet
        L.nrx_calibrate(model, wd, descs, y, llr, ws)
        scales = L.nrx_act_scales(model)
        log(f"fp8 scales: {np.array2string(scales, precision=4)}")
        assert scales.size == 2 * net.C + net.R and np.all(scales > 0)
        for c in (L.NRX_K_CONV_A, L.NRX_K_CONV_A_MP, L.NRX_K_CONV_B):
            L.nrx_conv_variant(model, c, variant)
        # E4M3 for both block convs, then (variant 0) for only one of them, the other in BF16
        errs = {}
        for mask in ((3, 1, 2) if variant == 0 else (3,)):
            L.nrx_fp8_layers(model, mask)
            llr.zero_()
            L.nrx_forward(model, wd, descs, y, llr, ws)
            torch.cuda.synchronize()
            got = split_llr(llr.cpu().numpy(), shapes, m_max)
            worst, agree_n, agree_d = 0.0, 0, 0
            for i in range(len(shapes)):
                for u in range(shapes[i]["n_ue"]):
                    worst = max(worst, rel_err(got[i][u], exp[i][u]))
                    big = np.abs(exp[i][u]) > 2.0
                    agree_n += int(np.sum((got[i][u][big] > 0) == (exp[i][u][big] > 0)))
                    agree_d += int(np.sum(big))
            log(f"fp8 variant {variant}, E4M3 layers {mask}: worst relative error {worst:.3e}, decision agreement "
                f"{agree_n / max(agree_d, 1):.5f} over {agree_d}")
            assert worst <= FP8_TOL
            assert agree_n >= FP8_AGREE * agree_d
            errs[mask] = worst
        if len(errs) == 3:
            # half the quantised convolutions: a smaller error than with both, for at least one of the halves
            assert min(errs[1], errs[2]) < errs[3]
    finally:
        L.nrx_model_destroy(model)


def test_nrx_forward_fp8_var_io():
    """FP8 Var-IO model (Sec. III, Fig. 2, with the E4M3 block convs): each modulation's StateInit (BF16) writes
    the E4M3 copy of its own UEs' rows only, the block convs read that copy, each modulation's readout reads its
    UEs; slots of one modulation beside mixed ones, eager and replayed as a hipGraph.  LLRs against the FP64
    oracle to the FP8 bars."""
    shp = VARIO_SLOT_SHAPES
    net = cgnn.NetConfig(4, 128, 3, 1, 8, var_io=True)
    ref_slots = oracle_batch(shp, sim_cfg_oracle(SIMCFG), 62, 0, 8)
    w = synth.he_weights(cgnn.layout(net), 62, perturb=True)
    exp = oracle_nrx(w, net, ref_slots)
    descs, sz = L.make_slots(shp, 8)
    y = _upload_batch(shp, ref_slots)
    wd = dev(w)
    for flags in (4, 4 | 1):
        log(f"FP8 Var-IO forward: flags {flags}")
        model = L.nrx_model_create(net.B, net.d, net.C, net.R, 8, L.NRX_FP8, flags=flags)
        try:
            llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
            ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
            L.nrx_calibrate(model, wd, descs, y, llr, ws)
            for rep in range(2 if flags & 1 else 1):
                llr.fill_(float("nan"))
                L.nrx_forward(model, wd, descs, y, llr, ws)
                torch.cuda.synchronize()
                got = llr.cpu().numpy().astype(np.float64)
                assert np.all(np.isfinite(got)), "LLR entries left unwritten"
                got = split_llr(got, shp, 8)
                worst, agree_n, agree_d = 0.0, 0, 0
                for i in range(len(shp)):
                    for u in range(shp[i]["n_ue"]):
                        worst = max(worst, rel_err(got[i][u], exp[i][u]))
                        big = np.abs(exp[i][u]) > 2.0
                        agree_n += int(np.sum((got[i][u][big] > 0) == (exp[i][u][big] > 0)))
                        agree_d += int(np.sum(big))
                log(f"  pass {rep}: worst relative error {worst:.3e}, decision agreement "
                    f"{agree_n / max(agree_d, 1):.5f} over {agree_d}")
                assert worst <= FP8_TOL
                assert agree_n >= FP8_AGREE * agree_d
        finally:
            L.nrx_model_destroy(model)


def test_full_size_sampled_parity():
    """The benchmark workload at full size and in the benchmark's launch configuration (32 slots x
    273 PRB x 14 symbols, 4 UEs, 8 antennas, 16-QAM; d = 128, 6 blocks, 2 rounds; autotuned conv
    variants; trained weights): LLRs at sampled subcarriers (both band edges and inside the band)
    against the oracle run on a window of +-16 subcarriers around each.  The 13 stacked 3x3
    convolutions see 13 subcarriers either way, message passing and the readout act per RE, and the
    window starts on an even subcarrier (the PE comb parity), so the window reproduces the full grid
    at its centre."""
    import os
    w = synth.WORKLOADS["m"]
    shapes = synth.uniform_shapes(w)
    m_max, S = w["m"], 12 * w["n_prb"]
    net = cgnn.NetConfig(w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], m_max)
    path = os.path.join(os.path.dirname(L.__file__), "weights", "nrx_c5.npy")
    wts = np.load(path) if os.path.exists(path) else synth.he_weights(cgnn.layout(net), 0)
    W = cgnn.unflatten(wts.astype(np.float64), net)
    log("full-size parity: oracle slots")
    ref = oracle_batch(shapes, sim_cfg_oracle(w), 0, 0, m_max)
    samples = [(0, 0), (0, 1638), (17, S - 1), (31, 911)]
    expected = {}
    for slot, s0 in samples:
        lo, hi = max(0, s0 - 16) & ~1, min(S, s0 + 17)
        r = ref[slot]
        h = receiver.ls_estimate(r["y32"], r["desc"])
        expected[(slot, s0)] = cgnn.forward(W, net, r["y32"][lo:hi], h[lo:hi], r["desc"].bits_per_sym)[:, :, s0 - lo, :]
    descs, sz = L.make_slots(shapes, m_max)
    y = _upload_batch(shapes, ref)
    wd = dev(wts)
    for prec, tol in ((L.NRX_FP32, 1e-4), (L.NRX_BF16, 2e-2)):
        model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
        try:
            llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
            ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
            L.nrx_autotune(model, wd, descs, y, llr, ws)
            llr.fill_(float("nan"))
            L.nrx_forward(model, wd, descs, y, llr, ws)
            torch.cuda.synchronize()
            got = split_llr(llr.cpu().numpy(), shapes, m_max)
            worst = 0.0
            for (slot, s0), e in expected.items():
                g = got[slot][:, :, s0, :]
                err = rel_err(g, e)
                worst = max(worst, err)
                big = np.abs(e) > 0.5
                assert np.all((g[big] > 0) == (e[big] > 0)), f"slot {slot} subcarrier {s0}: hard decisions differ"
                assert err <= tol, f"slot {slot} subcarrier {s0}: relative error {err:.3e} > {tol}"
            log(f"  prec {prec}: worst relative error {worst:.2e} over {len(expected)} sampled subcarriers")
        finally:
            L.nrx_model_destroy(model)
    # FP8 at the same size: activation scales calibrated on another batch of the workload (the GPU
    # simulator's batch 1, an input only), the FP8 bar of the small cases on the sampled subcarriers
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, L.NRX_FP8)
    try:
        cfg = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"], rho=w["rho"],
                           snr_db_lo=w["snr"][0], snr_db_hi=w["snr"][1])
        y_cal = torch.empty_like(y)
        sws = ws_tensor(L.slot_sim_workspace_bytes(cfg, descs))
        L.slot_sim(cfg, 0, 1, descs, m_max, y_cal, sws)
        del sws
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        L.nrx_calibrate(model, wd, descs, y_cal, llr, ws)
        L.nrx_autotune(model, wd, descs, y, llr, ws)
        llr.fill_(float("nan"))
        L.nrx_forward(model, wd, descs, y, llr, ws)
        torch.cuda.synchronize()
        got = split_llr(llr.cpu().numpy(), shapes, m_max)
        worst, agree_n, agree_d = 0.0, 0, 0
        for (slot, s0), e in expected.items():
            g = got[slot][:, :, s0, :]
            worst = max(worst, rel_err(g, e))
            big = np.abs(e) > 2.0
            agree_n += int(np.sum((g[big] > 0) == (e[big] > 0)))
            agree_d += int(np.sum(big))
        log(f"  fp8: worst relative error {worst:.3e}, decision agreement {agree_n / max(agree_d, 1):.5f} over {agree_d}")
        assert worst <= FP8_TOL and agree_n >= FP8_AGREE * agree_d
    finally:
        L.nrx_model_destroy(model)


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_nrx_forward_mu_mimo_16_antennas(prec, tol):
    # the MU-MIMO workload's network and channel (16 antennas, 4 UEs, 64-QAM, 24-tap spatially
    # correlated Rayleigh; d = 128, 8 blocks, 3 message-passing rounds) on a few 6-PRB slots
    w = synth.WORKLOADS["c3"]
    shapes = [dict(n_prb=6, n_ant=16, n_ue=4, bits=[6] * 4, slot_number=s) for s in range(3)]
    net, m_max = cgnn.NetConfig(16, 128, 8, 3, 6), 6
    log(f"nrx_forward 16 antennas: prec={prec}")
    ref_slots = oracle_batch(shapes, sim_cfg_oracle(w), 9, 0, m_max)
    wts = synth.he_weights(cgnn.layout(net), 9, perturb=True)
    exp = oracle_nrx(wts, net, ref_slots)
    model = L.nrx_model_create(net.B, net.d, net.C, net.R, m_max, prec)
    try:
        descs, sz = L.make_slots(shapes, m_max)
        y = _upload_batch(shapes, ref_slots)
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = ws_tensor(L.nrx_workspace_bytes(model, descs))
        for v in (1, 5, 7):
            L.set_all_conv_variants(model, v)
            L.nrx_forward(model, dev(wts), descs, y, llr, ws)
            torch.cuda.synchronize()
            got = split_llr(llr.cpu().numpy(), shapes, m_max)
            for i in range(len(shapes)):
                check_llr(got[i], exp[i], tol)
    finally:
        L.nrx_model_destroy(model)
