"""Host-side input generators: weight initialisation, the uniform and uneven batches, the mixed-MCS training
batches (Sec. II-B, III-A)."""
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


def test_he_weights_statistics():
    """He-normal kernels (variance 2 / fan_in over all axes but the last), zero biases, LayerNorm gamma 1 and
    beta 0; perturb=True moves biases and LayerNorm parameters off those values; the draw is seeded."""
    layout = [("conv.w", (3, 3, 64, 128)), ("conv.b", (128,)), ("ln.g", (128,)), ("ln.beta", (128,)),
              ("dense.w1", (128, 256))]
    w = synth.he_weights(layout, 3).astype(np.float64)
    assert w.size == sum(int(np.prod(s)) for _, s in layout)
    k = w[:3 * 3 * 64 * 128]
    assert abs(k.var() * (3 * 3 * 64) / 2.0 - 1.0) < 0.03 and abs(k.mean()) < 0.01
    o = k.size
    assert np.all(w[o:o + 128] == 0.0) and np.all(w[o + 128:o + 256] == 1.0) and np.all(w[o + 256:o + 384] == 0.0)
    d = w[o + 384:]
    assert abs(d.var() * 128 / 2.0 - 1.0) < 0.03
    assert np.array_equal(synth.he_weights(layout, 3), synth.he_weights(layout, 3))
    assert not np.array_equal(synth.he_weights(layout, 3), synth.he_weights(layout, 4))
    p = synth.he_weights(layout, 3, perturb=True).astype(np.float64)
    assert np.all(p[o:o + 128] != 0.0) and np.all(p[o + 128:o + 256] != 1.0)
    assert abs(p[o + 128:o + 256].mean() - 1.0) < 0.05


def test_ragged_shapes_ranges():
    """The uneven batch: PRBs in 4..max_prb, 1..4 UEs sharing one modulation per slot, antennas and modulation
    from the given sets, every value of each range drawn, the same list for the same seed."""
    shapes = synth.ragged_shapes(2000, 7, max_prb=273)
    prb = np.array([s["n_prb"] for s in shapes])
    assert prb.min() >= 4 and prb.max() <= 273 and len(set(prb.tolist())) > 200
    assert {s["n_ue"] for s in shapes} == {1, 2, 3, 4}
    assert {s["n_ant"] for s in shapes} == {4, 8, 16}
    assert {s["bits"][0] for s in shapes} == {2, 4, 6, 8}
    for i, s in enumerate(shapes):
        assert len(s["bits"]) == s["n_ue"] and len(set(s["bits"])) == 1 and s["slot_number"] == i % 20
    assert synth.ragged_shapes(50, 7) == synth.ragged_shapes(50, 7)
    assert synth.ragged_shapes(50, 7) != synth.ragged_shapes(50, 8)


def test_uniform_shapes_follow_the_workload():
    w = synth.WORKLOADS["m"]
    shapes = synth.uniform_shapes(w)
    assert len(shapes) == w["n_slots"]
    assert all(s["n_prb"] == w["n_prb"] and s["n_ant"] == w["n_ant"] and s["n_ue"] == w["n_ue"]
               and s["bits"] == [w["m"]] * w["n_ue"] for s in shapes)
    assert [s["slot_number"] for s in shapes[:22]] == list(range(20)) + [0, 1]
    assert synth.uniform_shapes(w, n_slots=3, n_prb=8, bits=6) == [
        dict(n_prb=8, n_ant=w["n_ant"], n_ue=w["n_ue"], bits=[6] * w["n_ue"], slot_number=i) for i in range(3)]
    # a ragged workload gives the seed-0 uneven batch
    c4 = synth.WORKLOADS["c4"]
    assert synth.uniform_shapes(c4) == synth.ragged_shapes(c4["n_slots"], 0, max_prb=c4["n_prb"])
