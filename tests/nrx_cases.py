"""Shared helpers for GPU parity tests: oracle-generated batches and packing to the C-ABI layouts.

Every input fed to both sides comes from the oracle's own simulator or from the seeded
generators in paper_2409_02912_amd.synth; nothing the HIP path computes is fed back to the oracle.
"""
import sys

import numpy as np

from oracle import cgnn, receiver, slot_sim
from paper_2409_02912_amd import synth


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sim_cfg_oracle(w):
    return slot_sim.SimConfig(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"],
                              rho=w["rho"], snr_db_lo=w["snr"][0], snr_db_hi=w["snr"][1])


def oracle_batch(shapes, cfg, seed, batch, m_max):
    """Oracle slots for a list of shape dicts; y rounded to complex64 as the GPU sees it."""
    out = []
    for i, sh in enumerate(shapes):
        d = slot_sim.SlotDesc(sh["n_prb"], sh["n_ant"], sh["n_ue"], sh["bits"], slot_number=sh.get("slot_number", 0),
                              n_id=sh.get("n_id", 0), n_scid=sh.get("n_scid", 0),
                              snr_offset_db=sh.get("snr_offset_db", 0.0))
        r = slot_sim.simulate_slot(seed, batch, i, cfg, d, m_max)
        r["desc"] = d
        r["y32"] = r["y"].astype(np.complex64).astype(np.complex128)
        r["n0_32"] = float(np.float32(r["n0"]))
        out.append(r)
    return out


def pack_complex(arrs):
    flat = np.concatenate([a.reshape(-1) for a in arrs]).astype(np.complex64)
    return flat.view(np.float32)


def pack_bits(slots):
    return np.concatenate([s["bits"].reshape(-1) for s in slots]).astype(np.uint8)


def split_llr(flat, shapes, m_max):
    out, o = [], 0
    for sh in shapes:
        S, U = 12 * sh["n_prb"], sh["n_ue"]
        n = U * 14 * S * m_max
        out.append(flat[o:o + n].reshape(U, 14, S, m_max))
        o += n
    return out


def split_h(flat_c, shapes):
    out, o = [], 0
    for sh in shapes:
        S, U, B = 12 * sh["n_prb"], sh["n_ue"], sh["n_ant"]
        n = S * 14 * U * B
        out.append(flat_c[o:o + n].reshape(S, 14, U, B))
        o += n
    return out


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def oracle_nrx(wflat, net, slots):
    W = cgnn.unflatten(wflat.astype(np.float64), net)
    res = []
    for r in slots:
        h = receiver.ls_estimate(r["y32"], r["desc"])
        res.append(cgnn.forward(W, net, r["y32"], h, r["desc"].bits_per_sym))
    return res


def check_llr(gpu, ref, tol, thresh=0.5):
    """Norm-wise relative error per UE; hard decisions agree where |ref| > thresh."""
    worst = 0.0
    for u in range(ref.shape[0]):
        e = rel_err(gpu[u], ref[u])
        worst = max(worst, e)
        assert e <= tol, f"UE {u}: relative error {e:.3e} > {tol}"
        big = np.abs(ref[u]) > thresh
        assert np.all((gpu[u][big] > 0) == (ref[u][big] > 0)), f"UE {u}: hard decisions differ"
    return worst
