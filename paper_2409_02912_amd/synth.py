"""Seeded synthetic inputs shared by tests, benchmark and training driver.

Holds no receiver arithmetic: only random draws (network weights, batch shapes)
and the workload configurations.  Slots themselves come from slot_sim.
"""
import numpy as np

# Workloads (Rayleigh tapped-delay stand-ins for the paper's channels; see the design notes).
WORKLOADS = {
    # small single-UE case the oracle finishes in seconds
    "c1": dict(n_slots=16, n_prb=4, n_ant=4, n_ue=1, m=2, n_taps=3, decay_ns=100.0, doppler=0.0, rho=0.0,
               snr=(10.0, 10.0), d=32, n_blocks=2, n_rounds=0),
    "c2": dict(n_slots=32, n_prb=273, n_ant=4, n_ue=2, m=4, n_taps=12, decay_ns=487.42, doppler=100.0, rho=0.0,
               snr=(0.0, 20.0), d=128, n_blocks=6, n_rounds=2),
    "c3": dict(n_slots=64, n_prb=106, n_ant=16, n_ue=4, m=6, n_taps=24, decay_ns=305.02, doppler=0.0, rho=0.5,
               snr=(5.0, 30.0), d=128, n_blocks=8, n_rounds=3),
    "c5": dict(n_slots=64, n_prb=106, n_ant=8, n_ue=4, m=4, n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0,
               snr=(-2.0, 20.0), d=128, n_blocks=6, n_rounds=2),
    # a fixed "site" (stand-in for the site-specific data of Sec. V): the C5 shape with one channel profile of its
    # own, 6 taps of 150 ns decay, BS-array correlation 0.7, UE speeds uniform in 0..8 m/s (Doppler up to 93 Hz
    # at a 3.5 GHz carrier)
    "site": dict(n_slots=64, n_prb=106, n_ant=8, n_ue=4, m=4, n_taps=6, decay_ns=150.0, doppler=93.0, rho=0.7,
                 snr=(-2.0, 20.0), d=128, n_blocks=6, n_rounds=2),
    # the small training workload on the site channel (fine-tuning test)
    "t_site": dict(n_slots=32, n_prb=8, n_ant=4, n_ue=2, m=4, n_taps=6, decay_ns=150.0, doppler=93.0, rho=0.7,
                   snr=(0.0, 15.0), d=128, n_blocks=2, n_rounds=1),
    # uneven batch: per slot PRBs 4..273, 1..4 UEs, 4/8/16 antennas, QPSK..256-QAM (ragged_shapes)
    "c4": dict(n_slots=256, ragged=True, n_prb=273, n_ant=16, n_ue=4, m=8, n_taps=12, decay_ns=487.42,
               doppler=0.0, rho=0.0, snr=(0.0, 30.0), d=128, n_blocks=6, n_rounds=2),
    # small training workload (learning test: trains in about a minute)
    "t": dict(n_slots=32, n_prb=8, n_ant=4, n_ue=2, m=4, n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0,
              snr=(0.0, 15.0), d=128, n_blocks=2, n_rounds=1),
    # the small workload for mixed-MCS training: QPSK, 16-QAM and 64-QAM UEs (LLRs masked to m_u), up to 2 UEs
    "tm": dict(n_slots=32, n_prb=8, n_ant=4, n_ue=2, m=6, mcs=[2, 4, 6], n_taps=12, decay_ns=487.42, doppler=0.0,
               rho=0.0, snr=(0.0, 15.0), d=128, n_blocks=2, n_rounds=1),
    # the small training workload with two CGNN iterations (multi-loss and depth control)
    "t2": dict(n_slots=32, n_prb=8, n_ant=4, n_ue=2, m=4, n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0,
               snr=(0.0, 15.0), d=128, n_blocks=4, n_rounds=2),
    # the C5 network and channel on small slots (8 PRB, 32 per batch): many more optimiser steps per GPU
    # second than the 106-PRB batches (the network does not depend on the PRB count), to separate what the
    # architecture can reach from what the C5 budget reaches
    "c5s": dict(n_slots=32, n_prb=8, n_ant=8, n_ue=4, m=4, n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0,
                snr=(-2.0, 20.0), d=128, n_blocks=6, n_rounds=2),
    # headline workload: 273 PRB, 4 UEs, 8 antennas, 16-QAM, batch 32
    "m": dict(n_slots=32, n_prb=273, n_ant=8, n_ue=4, m=4, n_taps=12, decay_ns=487.42, doppler=0.0, rho=0.0,
              snr=(10.0, 10.0), d=128, n_blocks=6, n_rounds=2),
}


def he_weights(layout, seed, perturb=False):
    """Flat fp32 weight vector: He-normal N(0, 2/fan_in) for conv/dense kernels (fan_in = all axes but the
    last), zero biases, LN gamma 1 / beta 0.  perturb=True draws biases and LN parameters too (tests)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in layout:
        n = int(np.prod(shape))
        if len(shape) >= 2:
            fan = int(np.prod(shape[:-1]))
            v = rng.standard_normal(n) * np.sqrt(2.0 / fan)
        elif name.endswith(".g"):
            v = 1.0 + (0.1 * rng.standard_normal(n) if perturb else np.zeros(n))
        else:
            v = 0.1 * rng.standard_normal(n) if perturb else np.zeros(n)
        parts.append(v)
    return np.concatenate(parts).astype(np.float32)


def ragged_shapes(n_slots, seed, max_prb=273, ants=(4, 8, 16), mods=(2, 4, 6, 8)):
    """Uneven batch: PRBs uniform in 4..max_prb, UEs 1..4, antennas and modulation per slot."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_slots):
        u = int(rng.integers(1, 5))
        out.append(dict(n_prb=int(rng.integers(4, max_prb + 1)), n_ant=int(rng.choice(ants)), n_ue=u,
                        bits=[int(rng.choice(mods))] * u, slot_number=i % 20))
    return out


def uniform_shapes(w, n_slots=None, n_prb=None, bits=None):
    """The workload's batch of identical slots; bits overrides the modulation (bits per symbol) of every UE."""
    n = n_slots or w["n_slots"]
    if w.get("ragged"):
        return ragged_shapes(n, 0, max_prb=n_prb or w["n_prb"])
    return [dict(n_prb=n_prb or w["n_prb"], n_ant=w["n_ant"], n_ue=w["n_ue"], bits=[bits or w["m"]] * w["n_ue"],
                 slot_number=i % 20) for i in range(n)]


# Mixed-MCS training (Sec. III-A with the U_A draw of Sec. II-B).  Readings where the paper gives no numbers:
#   * U_A, the number of active UEs of a batch, is drawn from the discrete triangular law P(U_A = k) = 2k / (U(U+1))
#     on 1..U (more UEs more likely);
#   * every active UE of every slot draws its modulation iid and uniform from the workload's set;
#   * the SNR offset of a slot is the mean over its UEs of a per-modulation offset (roughly the SNR gap between
#     Gray-QAM orders at equal uncoded BER, 16-QAM = 0 dB) plus a fixed step per UE beyond the first.
MOD_SNR_OFFSET_DB = {2: -6.0, 4: 0.0, 6: 6.0, 8: 12.0}
UE_SNR_STEP_DB = 1.0


def mixed_mcs_shapes(w, rng, n_slots=None, n_prb=None):
    """One training batch of the mixed-MCS scheme: U_A active UEs for the whole batch (triangular), an iid
    modulation per UE and slot from w["mcs"], and the per-slot SNR offset."""
    n = n_slots or w["n_slots"]
    U = w["n_ue"]
    k = np.arange(1, U + 1)
    ua = int(rng.choice(k, p=2.0 * k / (U * (U + 1))))
    out = []
    for i in range(n):
        bits = [int(b) for b in rng.choice(w["mcs"], size=ua)]
        off = float(np.mean([MOD_SNR_OFFSET_DB[b] for b in bits])) + UE_SNR_STEP_DB * (ua - 1)
        out.append(dict(n_prb=n_prb or w["n_prb"], n_ant=w["n_ant"], n_ue=ua, bits=bits, slot_number=i % 20,
                        snr_offset_db=off))
    return out
