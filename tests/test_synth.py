"""Host-side input generators: the mixed-MCS training batches (Sec. II-B, III-A)."""
import numpy as np

from paper_2409_02912_amd import synth


def test_mixed_mcs_batches():
    w = synth.WORKLOADS["tm"]
    rng = np.random.default_rng(0)
    U = w["n_ue"]
    counts = np.zeros(U + 1)
    mods = {b: 0 for b in w["mcs"]}
    for _ in range(3000):
        shapes = synth.mixed_mcs_shapes(w, rng, n_slots=4)
        ua = shapes[0]["n_ue"]
        counts[ua] += 1
        for sh in shapes:
            # one U_A for the whole batch, an iid modulation per active UE, the offset of that association
            assert sh["n_ue"] == ua and len(sh["bits"]) == ua
            want = np.mean([synth.MOD_SNR_OFFSET_DB[b] for b in sh["bits"]]) + synth.UE_SNR_STEP_DB * (ua - 1)
            assert abs(sh["snr_offset_db"] - want) < 1e-12
            for b in sh["bits"]:
                mods[b] += 1
    k = np.arange(1, U + 1)
    p = counts[1:] / counts.sum()
    assert np.allclose(p, 2 * k / (U * (U + 1)), atol=0.03)     # triangular U_A
    f = np.array(list(mods.values()), dtype=float)
    assert np.allclose(f / f.sum(), 1 / len(mods), atol=0.02)   # uniform modulation
    # higher orders and more UEs are trained at higher SNR
    assert synth.MOD_SNR_OFFSET_DB[2] < synth.MOD_SNR_OFFSET_DB[4] < synth.MOD_SNR_OFFSET_DB[6]
