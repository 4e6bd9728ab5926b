"""Throughput of the NRX forward pass on one MI355X.

A step is one nrx_forward call (LS + interpolation, StateInit, CGNN iterations,
readout, masking) over a batch of synthetic PUSCH slots already resident in
HBM.  The headline workload is 273 PRB x 14 symbols, 4 UEs, 8 BS antennas,
16-QAM, batch 32, CGNN width 128 / 6 blocks / 2 message-passing rounds; the
timed precision is BF16 with the FP32 pass timed beside it at the same weights
and slots, and the bit error rates of both and of LS + LMMSE reported.

Prints one JSON line.  Only 1 GPU is supported.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NRX slots/s & REs/s at 273 PRB, 4 UE: BF16/FP8 vs FP32 at matched BER"
PEAKS = {"bf16": 2.5e15, "fp32": 157.3e12, "fp8": 5.0e15}


def flops_per_row(B, d, C, R, m_max):
    """Algorithmic FLOPs per (UE, RE) row of the CGNN forward (multiply-add = 2)."""
    mpb = [(r * C) // R for r in range(R)]
    f = 2 * 9 * (4 * B + 2) * d                                   # StateInit
    for i in range(C):
        f += 2 * 9 * ((2 * d + 2) if i in mpb else d) * d         # conv_a
        f += 2 * 9 * d * d                                        # conv_b
    f += R * 2 * (2 * d * d)                                      # message MLPs
    f += 2 * d * d + 2 * d * m_max                                # readout
    return f


def cpu_baseline(w, weights, net_args, budget_s):
    """Times the FP64 oracle (LS + CGNN forward) on whole slots of the same workload."""
    import numpy as np
    from oracle import cgnn, receiver, slot_sim
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu_model)
    except OSError:  # pragma: no cover
        pass
    net = cgnn.NetConfig(*net_args)
    W = cgnn.unflatten(weights.astype(np.float64), net)
    cfg = slot_sim.SimConfig(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"],
                             rho=w["rho"], snr_db_lo=w["snr"][0], snr_db_hi=w["snr"][1])
    n, t_total = 0, 0.0
    while n < 1 or (t_total < budget_s and n < 4):
        d = slot_sim.SlotDesc(w["n_prb"], w["n_ant"], w["n_ue"], [w["m"]] * w["n_ue"], slot_number=n)
        r = slot_sim.simulate_slot(0, 0, n, cfg, d, w["m"])
        t0 = time.perf_counter()
        h = receiver.ls_estimate(r["y"], d)
        cgnn.forward(W, net, r["y"], h, d.bits_per_sym)
        t_total += time.perf_counter() - t0
        n += 1
    out = {"value": n / t_total, "unit": "slots/s", "cores": int(cores), "kind": "oracle",
           "cpu_model": cpu_model, "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
           "sample": f"{n} slot(s) of {w['n_prb']} PRB x 14 x {w['n_ue']} UE x {w['n_ant']} ant, "
                     f"fp64 numpy LS + CGNN forward, {t_total:.1f} s"}
    # the LS + LMMSE + max-log oracle on one slot of the same workload
    d = slot_sim.SlotDesc(w["n_prb"], w["n_ant"], w["n_ue"], [w["m"]] * w["n_ue"], slot_number=0)
    r = slot_sim.simulate_slot(0, 0, 0, cfg, d, w["m"])
    t0 = time.perf_counter()
    receiver.lmmse_demap(r["y"], receiver.ls_estimate(r["y"], d), r["n0"], d, w["m"])
    tl = time.perf_counter() - t0
    out["lmmse_oracle_slots_per_s"] = 1.0 / tl
    # the small single-UE configuration in full: 16 slots of 4 PRB, 4 antennas, QPSK, d = 32, 2 blocks
    from paper_2409_02912_amd import synth
    c1 = synth.WORKLOADS["c1"]
    net1 = cgnn.NetConfig(c1["n_ant"], c1["d"], c1["n_blocks"], c1["n_rounds"], c1["m"])
    W1 = cgnn.unflatten(synth.he_weights(cgnn.layout(net1), 0).astype(np.float64), net1)
    cfg1 = slot_sim.SimConfig(n_taps=c1["n_taps"], tap_decay_ns=c1["decay_ns"], snr_db_lo=c1["snr"][0],
                              snr_db_hi=c1["snr"][1])
    t1 = 0.0
    for k in range(c1["n_slots"]):
        d1 = slot_sim.SlotDesc(c1["n_prb"], c1["n_ant"], c1["n_ue"], [c1["m"]] * c1["n_ue"], slot_number=k)
        r1 = slot_sim.simulate_slot(0, 0, k, cfg1, d1, c1["m"])
        t0 = time.perf_counter()
        cgnn.forward(W1, net1, r1["y"], receiver.ls_estimate(r1["y"], d1), d1.bits_per_sym)
        t1 += time.perf_counter() - t0
    out["c1_oracle_slots_per_s"] = c1["n_slots"] / t1
    out["sample"] += f"; LS + LMMSE oracle 1 slot {tl:.1f} s; C1 16 slots {t1:.2f} s"
    return out


def ragged_batch(steps, no_autotune, tune_cache=None, persistent=False):
    """Uneven batch of 256 slots (PRBs 4..273, 1..4 UEs, 4/8/16 antennas, QPSK..256-QAM) in BF16,
    replayed from a captured hipGraph; per-slot latency = start of the pass to the end of the
    slot's last readout tile, from the device wall clock.  persistent: the CGNN runs as one
    persistent launch over slot groups (model flags bit 3) instead of one launch per layer."""
    import numpy as np
    import torch
    from paper_2409_02912_amd import libnrx as L
    from paper_2409_02912_amd import synth
    w = synth.WORKLOADS["c4"]
    shapes = synth.uniform_shapes(w)
    m_max = w["m"]
    descs, sz = L.make_slots(shapes, m_max)
    model = L.nrx_model_create(w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], m_max, L.NRX_BF16,
                               flags=1 | (8 if persistent else 0))
    try:
        layout = [(n, s) for n, _, s in L.weight_layout(model)]
        dw = torch.from_numpy(synth.he_weights(layout, 0)).cuda()
        cfg = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"],
                           rho=w["rho"], snr_db_lo=w["snr"][0], snr_db_hi=w["snr"][1])
        y = torch.empty(2 * sz["y"], dtype=torch.float32, device="cuda")
        sws = torch.empty(L.slot_sim_workspace_bytes(cfg, descs), dtype=torch.uint8, device="cuda")
        L.slot_sim(cfg, 0, 0, descs, m_max, y, sws)
        del sws
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device="cuda")
        if not no_autotune and not persistent:
            L.nrx_autotune(model, dw, descs, y, llr, ws, cache_path=tune_cache)
        variants = ({L.KERNEL_CLASSES[c]: L.nrx_conv_variant(model, c)[0] for c in L.CONV_CLASSES}
                    if not persistent else "persistent kernel (ring conv shape and schedule of variant 14)")
        flags = torch.full((len(shapes),), -1, dtype=torch.int32, device="cuda")
        lat = torch.zeros(len(shapes), dtype=torch.float32, device="cuda")
        for _ in range(2):
            L.nrx_forward(model, dw, descs, y, llr, ws)      # first call captures the graph
        torch.cuda.synchronize()
        lats = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        total = 0.0
        for _ in range(steps):
            e0.record()
            L.nrx_forward(model, dw, descs, y, llr, ws)
            e1.record()
            L.nrx_slot_latency(model, descs, ws, lat)
            torch.cuda.synchronize()
            total += e0.elapsed_time(e1)
            lats.append(lat.cpu().numpy().copy())
        ms = total / steps
        L.nrx_slot_flags(model, descs, ws, flags)
        n_flagged = int((flags != 0).sum().item())
        v = np.concatenate(lats)
        res = sum(12 * s["n_prb"] * 14 for s in shapes)
        llr_bf16 = llr.clone()
    finally:
        L.nrx_model_destroy(model)
    # the same batch once through the FP32 pass: LLR error of the timed BF16 pass against it
    m32 = L.nrx_model_create(w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], m_max, L.NRX_FP32)
    try:
        del ws
        ws = torch.empty(L.nrx_workspace_bytes(m32, descs), dtype=torch.uint8, device="cuda")
        llr32 = torch.zeros_like(llr)
        L.nrx_forward(m32, dw, descs, y, llr32, ws)
        torch.cuda.synchronize()
        rel = (torch.linalg.vector_norm(llr_bf16 - llr32) / torch.linalg.vector_norm(llr32)).item()
    finally:
        L.nrx_model_destroy(m32)
    return {"workload": f"{len(shapes)} uneven slots: PRB 4-273, 1-4 UE, 4/8/16 ant, QPSK..256-QAM, bf16, "
                        f"hipGraph replay" + (", one persistent launch" if persistent else ", one launch per layer"),
            "slots_flagged": n_flagged,
            "slots_per_s": len(shapes) / (ms * 1e-3), "res_per_s": res / (ms * 1e-3), "ms_per_step": ms,
            "steps": steps, "latency_us_p50": float(np.percentile(v, 50)),
            "latency_us_p99": float(np.percentile(v, 99)),
            "llr_rel_err_bf16_vs_fp32": rel, "conv_variants": variants}


# kernel templates behind the conv variant indices of the library (kConvVariants), for reporting
CONV_VARIANT_KERNELS = [
    "conv3x3_kernel<MB 4, OCC 1, weights one tap ahead>", "conv3x3_kernel<MB 4, OCC 2>",
    "conv3x3_kernel<MB 2, OCC 2, weights one tap ahead>", "conv3x3_kernel<MB 2, OCC 2>",
    "conv3x3_lds_kernel<MB 6, NW 4>", "conv3x3_lds_kernel<MB 4, NW 8>",
    "conv3x3_ring_kernel<MB 4, NW 4, G 1, OCC 2, NBUF 2>", "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 2>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 1, OCC 1, NBUF 6>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 2, compiler-scheduled>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 2, raised wave priority>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 2, staggered start>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 2, raised wave priority, staggered start>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 3, 504-row subcarrier-aligned tiles>",
    "conv3x3_ring_kernel<MB 4, NW 8, G 3, OCC 1, NBUF 2, falling wave priority>",
]


def stored_traffic(conv_b_variant):
    """HBM bytes per conv_b launch from the committed FETCH_SIZE / WRITE_SIZE passes, or None when the
    kernel sources or the tile variant differ from the ones the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "conv_b_bf16_m273_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for src in d["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != d["sources_sha256"]:
        return None
    return d["hbm_bytes_per_launch"].get(str(conv_b_variant))


def paper_rt_latency(reps=50):
    """Batch-1 latency of the real-time-sized network of Sec. IV-B (d_S = 56, two CGNN iterations;
    here 2 conv blocks with 2 message-passing rounds) on the setup the paper times there: one slot of
    132 PRB, 2 UEs, 4 BS antennas, 16-QAM.  The paper's A100 TensorRT figure is context only."""
    import torch
    from paper_2409_02912_amd import libnrx as L
    from paper_2409_02912_amd import synth
    shapes = [dict(n_prb=132, n_ant=4, n_ue=2, bits=[4, 4], slot_number=0)]
    descs, sz = L.make_slots(shapes, 4)
    cfg = L.sim_config(n_taps=12, tap_decay_ns=487.42, snr_db_lo=10.0, snr_db_hi=10.0)
    y = torch.empty(2 * sz["y"], dtype=torch.float32, device="cuda")
    sws = torch.empty(L.slot_sim_workspace_bytes(cfg, descs), dtype=torch.uint8, device="cuda")
    L.slot_sim(cfg, 0, 0, descs, 4, y, sws)
    out = {"setup": "1 slot, 132 PRB x 14 sym, 2 UE, 4 ant, 16-QAM; CGNN d=56, 2 blocks, 2 MP rounds",
           "paper_a100_tensorrt_ms": 0.97,
           "paper_note": "Sec. IV-B: about 270 us + 350 us per CGNN iteration on an A100 (float16, TensorRT)"}
    for prec, name in ((L.NRX_BF16, "bf16"), (L.NRX_FP32, "fp32")):
        for flags, mode in ((0, "eager"), (1, "graph")):
            model = L.nrx_model_create(4, 56, 2, 2, 4, prec, flags=flags)
            try:
                layout = [(n, sh) for n, _, sh in L.weight_layout(model)]
                dw = torch.from_numpy(synth.he_weights(layout, 0)).cuda()
                llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
                ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device="cuda")
                L.nrx_autotune(model, dw, descs, y, llr, ws)
                for _ in range(5):
                    L.nrx_forward(model, dw, descs, y, llr, ws)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    L.nrx_forward(model, dw, descs, y, llr, ws)
                e1.record()
                torch.cuda.synchronize()
                out[f"{name}_{mode}_ms"] = e0.elapsed_time(e1) / reps
            finally:
                L.nrx_model_destroy(model)
    return out


def depth_latency(reps=30):
    """Batch-1 latency against the number of CGNN iterations run (Sec. IV-B, Fig. 4): the Large NRX shape
    (N_it = 8 iterations of message passing + one conv block, d_S = 56) on the paper's timing setup (one slot of
    132 PRB, 2 UEs, 4 antennas, 16-QAM), BF16, hipGraph replay, depth set with nrx_set_iterations.  The state
    depth 56 runs zero-padded at 128 channels.  Latency is independent of the weights (seeded here)."""
    import numpy as np
    import torch
    from paper_2409_02912_amd import libnrx as L
    from paper_2409_02912_amd import synth
    shapes = [dict(n_prb=132, n_ant=4, n_ue=2, bits=[4, 4], slot_number=0)]
    descs, sz = L.make_slots(shapes, 4)
    cfg = L.sim_config(n_taps=12, tap_decay_ns=487.42, snr_db_lo=10.0, snr_db_hi=10.0)
    y = torch.empty(2 * sz["y"], dtype=torch.float32, device="cuda")
    sws = torch.empty(L.slot_sim_workspace_bytes(cfg, descs), dtype=torch.uint8, device="cuda")
    L.slot_sim(cfg, 0, 0, descs, 4, y, sws)
    model = L.nrx_model_create(4, 56, 8, 8, 4, L.NRX_BF16, flags=1)
    ms = []
    try:
        layout = [(n, sh) for n, _, sh in L.weight_layout(model)]
        dw = torch.from_numpy(synth.he_weights(layout, 0)).cuda()
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device="cuda")
        L.nrx_autotune(model, dw, descs, y, llr, ws)
        for k in range(1, L.nrx_num_iterations(model) + 1):
            L.nrx_set_iterations(model, k)
            for _ in range(5):
                L.nrx_forward(model, dw, descs, y, llr, ws)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                L.nrx_forward(model, dw, descs, y, llr, ws)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1) / reps)
    finally:
        L.nrx_model_destroy(model)
    k = np.arange(1, len(ms) + 1)
    slope, icpt = np.polyfit(k, ms, 1)
    resid = float(np.max(np.abs(np.array(ms) - (icpt + slope * k))))
    return {"setup": "1 slot, 132 PRB x 14 sym, 2 UE, 4 ant, 16-QAM; Large NRX shape: 8 CGNN iterations "
                     "(MP round + conv block), d=56 (run at 128), bf16, hipGraph",
            "ms_by_iterations": ms, "affine_fit_ms": {"per_iteration": float(slope), "overhead": float(icpt),
                                                       "max_residual": resid},
            "paper_note": "Sec. IV-B / Fig. 4: latency grows linearly with the iterations; about 350 us per "
                          "iteration and 270 us overhead on an A100 (TensorRT)"}


def secondary_rows(steps, tune_cache):
    """Throughput of the secondary shapes with seeded weights (no trained network exists for them, so LLR error
    against the FP32 pass stands in for BER): B = 4 antennas / 2 UEs at 273 PRB (32 slots), and B = 16 antennas /
    4 UEs / 64-QAM at 106 PRB with 8 blocks and 3 message-passing rounds (64 slots)."""
    import numpy as np
    import torch
    from paper_2409_02912_amd import libnrx as L
    from paper_2409_02912_amd import synth
    out = {}
    for name in ("c2", "c3"):
        w = synth.WORKLOADS[name]
        shapes = synth.uniform_shapes(w)
        descs, sz = L.make_slots(shapes, w["m"])
        cfg = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"],
                           rho=w["rho"], snr_db_lo=w["snr"][0], snr_db_hi=w["snr"][1])
        y = torch.empty(2 * sz["y"], dtype=torch.float32, device="cuda")
        sws = torch.empty(L.slot_sim_workspace_bytes(cfg, descs), dtype=torch.uint8, device="cuda")
        L.slot_sim(cfg, 0, 0, descs, w["m"], y, sws)
        del sws
        net_args = (w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], w["m"])
        row, llrs = {}, {}
        for prec, pname in ((L.NRX_BF16, "bf16"), (L.NRX_FP32, "fp32")):
            model = L.nrx_model_create(*net_args, prec)
            try:
                dw = torch.from_numpy(synth.he_weights([(n, sh) for n, _, sh in L.weight_layout(model)], 0)).cuda()
                ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device="cuda")
                llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
                if pname == "bf16":
                    L.nrx_autotune(model, dw, descs, y, llr, ws, cache_path=tune_cache)
                n = steps if pname == "bf16" else 1
                L.nrx_forward(model, dw, descs, y, llr, ws)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(n):
                    L.nrx_forward(model, dw, descs, y, llr, ws)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / n
                row[pname] = {"ms_per_step": ms, "slots_per_s": len(shapes) / (ms * 1e-3)}
                llrs[pname] = llr.cpu().numpy().astype(np.float64)
                del ws
            finally:
                L.nrx_model_destroy(model)
        row["res_per_s_bf16"] = row["bf16"]["slots_per_s"] * 12 * w["n_prb"] * 14
        row["llr_rel_err_bf16_vs_fp32"] = float(np.linalg.norm(llrs["bf16"] - llrs["fp32"]) /
                                               np.linalg.norm(llrs["fp32"]))
        row["workload"] = (f"{len(shapes)} slots x {w['n_prb']} PRB x 14 sym, {w['n_ue']} UE, {w['n_ant']} ant, "
                           f"{2 ** w['m']}-QAM; CGNN d={w['d']}, {w['n_blocks']} blocks, {w['n_rounds']} MP rounds; "
                           "seeded weights")
        out[name] = row
        progress(f"secondary {name}: {row['bf16']['ms_per_step']:.3f} ms/step bf16")
    return out


def training_row(steps):
    """One training step (Sec. II-B) on the C5 training batch (64 slots x 106 PRB x 14 symbols, 4 UEs, 8 antennas,
    16-QAM; CGNN d = 128, 6 blocks, 2 MP rounds), BF16: slot generation, forward keeping activations, BCE, the
    hand-written backward and the Adam step, all on the GPU."""
    import torch
    from paper_2409_02912_amd import libnrx as L
    from paper_2409_02912_amd import synth
    from paper_2409_02912_amd.train import Trainer
    w = synth.WORKLOADS["c5"]
    tr = Trainer(w, L.NRX_BF16, seed=0)
    try:
        for _ in range(2):
            tr.train_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            tr.train_step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    finally:
        tr.close()
    return {"workload": "64 slots x 106 PRB x 14 sym, 4 UE, 8 ant, 16-QAM; CGNN d=128, 6 blocks, 2 MP rounds; "
                        "bf16; slot_sim + forward + BCE + backward + Adam",
            "ms_per_step": ms, "slots_per_s": w["n_slots"] / (ms * 1e-3), "steps": steps}


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="m")
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--autotune-headline", action="store_true",
                    help="let the autotuner choose the BF16 / FP8 conv variants too (default: the library's defaults)")
    ap.add_argument("--bf16-only", action="store_true", help="skip the FP32 pass and batch-1 runs (profiling)")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 pass")
    ap.add_argument("--no-fp8-policies", action="store_true",
                    help="skip the FP8 passes with only conv_a or only conv_b in E4M3")
    ap.add_argument("--no-persistent", action="store_true", help="skip the persistent-launch BF16 pass")
    ap.add_argument("--variant-sweep", action="store_true", help="time every conv variant per layer class")
    ap.add_argument("--ragged-steps", type=int, default=5,
                    help="timed replays of the uneven 256-slot batch under a hipGraph (0: skip)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache (JSON lines): reuse its tile-shape choices, append new ones")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain elementwise copy kernel over this many MiB (HBM-counter calibration)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the B = 4 and B = 16 throughput rows")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2409_02912_amd", "weights", "nrx_c5.npy"))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the NRX batch is data-parallel over slots with no exchange, "
              "and the benchmark has no multi-GPU mode.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_02912_amd import libnrx as L
    from paper_2409_02912_amd import synth

    if args.calib_copy_mib:
        n = args.calib_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)   # one elementwise kernel: reads and writes n floats
        torch.cuda.synchronize()
        del src, dst

    w = synth.WORKLOADS[args.workload]
    shapes = synth.uniform_shapes(w)
    m_max = w["m"]
    descs, sz = L.make_slots(shapes, m_max)
    n_slots = len(shapes)
    net_args = (w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], m_max)
    m0 = L.nrx_model_create(*net_args)           # host-only: the weight layout the library uses
    layout = [(n, sh) for n, _, sh in L.weight_layout(m0)]
    L.nrx_model_destroy(m0)
    trained = os.path.exists(args.weights)
    weights = np.load(args.weights) if trained else synth.he_weights(layout, 0)
    dw = torch.from_numpy(weights).cuda()

    # synthetic slots resident in HBM
    cfg = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"], rho=w["rho"],
                       snr_db_lo=w["snr"][0], snr_db_hi=w["snr"][1])
    y = torch.empty(2 * sz["y"], dtype=torch.float32, device="cuda")
    bits = torch.empty(sz["bits"], dtype=torch.uint8, device="cuda")
    n0 = torch.empty(n_slots, dtype=torch.float32, device="cuda")
    sws = torch.empty(L.slot_sim_workspace_bytes(cfg, descs), dtype=torch.uint8, device="cuda")
    L.slot_sim(cfg, 0, 0, descs, m_max, y, sws, bits=bits, n0=n0)
    # FP8 activation scales are calibrated on a different batch of the same workload
    y_cal = None
    if not args.no_fp8:
        y_cal = torch.empty_like(y)
        L.slot_sim(cfg, 0, 1, descs, m_max, y_cal, sws)
    del sws

    results = {}
    llrs = {}
    flag_words = {}    # per-slot health words of each pass (non-finite input or LLRs)
    passes = [(L.NRX_BF16, "bf16")]
    if not args.no_persistent:
        passes.append((L.NRX_BF16, "bf16_persistent"))
    # FP8 passes: both block convs in E4M3 (the library default), then each alone (the other in BF16)
    fp8_masks = {"fp8": 3, "fp8_conv_a": 1, "fp8_conv_b": 2}
    if not args.no_fp8:
        passes.append((L.NRX_FP8, "fp8"))
        if not args.no_fp8_policies:
            passes += [(L.NRX_FP8, "fp8_conv_a"), (L.NRX_FP8, "fp8_conv_b")]
    if not args.bf16_only:
        passes.append((L.NRX_FP32, "fp32"))
    for prec, name in passes:
        # flags bit 0: the timed pass is the captured launch sequence replayed as a hipGraph
        model = L.nrx_model_create(*net_args, prec, flags=1 | (8 if name == "bf16_persistent" else 0))
        ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device="cuda")
        llr = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
        if name in fp8_masks:
            L.nrx_calibrate(model, dw, descs, y_cal, llr, ws)
            L.nrx_fp8_layers(model, fp8_masks[name])
            if name == "fp8":
                results.setdefault("fp8_scales", L.nrx_act_scales(model).tolist())
        steps = args.fp32_steps if name == "fp32" else args.steps
        warm = 1 if name == "fp32" else args.warmup
        if args.variant_sweep:
            sweep = {}
            for v in range(L.nrx_conv_variant(model, L.NRX_K_CONV_B)[1]):
                L.set_all_conv_variants(model, v)
                L.nrx_forward(model, dw, descs, y, llr, ws)
                torch.cuda.synchronize()
                L.nrx_profile_enable(model, True)
                for c in range(len(L.KERNEL_CLASSES)):
                    L.nrx_profile_read(model, c, reset=True)
                for _ in range(3):
                    L.nrx_forward(model, dw, descs, y, llr, ws)
                sweep[v] = {L.KERNEL_CLASSES[c]: round(L.nrx_profile_read(model, c)[0] / 3 /
                                                       max(1, L.nrx_profile_read(model, c)[1] / 3), 4)
                            for c in L.CONV_CLASSES}
                L.nrx_profile_enable(model, False)
            results.setdefault("sweep", {})[name] = sweep
        # the BF16 and FP8 passes keep the library's default variants (fixed, so that the kernel the roofline
        # names is the one profiled); the FP32 pass is autotuned
        tune = name == "fp32" or (args.autotune_headline and name != "bf16_persistent")
        if tune and not args.no_autotune:
            L.nrx_autotune(model, dw, descs, y, llr, ws, cache_path=args.tune_cache)
        results.setdefault("variants", {})[name] = {L.KERNEL_CLASSES[c]: L.nrx_conv_variant(model, c)[0]
                                                    for c in L.CONV_CLASSES}
        for _ in range(warm):
            L.nrx_forward(model, dw, descs, y, llr, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            L.nrx_forward(model, dw, descs, y, llr, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # per-kernel durations: the same passes launched one by one, each kernel between two HIP events on the
        # stream it runs on (profiling replaces the graph replay by the eager launch sequence)
        L.nrx_profile_enable(model, True)
        for c in range(len(L.KERNEL_CLASSES)):
            L.nrx_profile_read(model, c, reset=True)
        psteps = min(steps, 5)
        for _ in range(psteps):
            L.nrx_forward(model, dw, descs, y, llr, ws)
        torch.cuda.synchronize()
        kern = {}
        for c, cname in enumerate(L.KERNEL_CLASSES):
            t, n = L.nrx_profile_read(model, c)
            kern[cname] = {"ms_per_launch": t / max(n, 1), "launches_per_step": n / psteps}
        L.nrx_profile_enable(model, False)
        results[name] = {"ms_per_step": ms, "kernels": kern}
        progress(f"{name}: {ms:.3f} ms/step")
        llrs[name] = llr
        flag_words[name] = torch.zeros(n_slots, dtype=torch.int32, device="cuda")
        L.nrx_slot_flags(model, descs, ws, flag_words[name])
        if args.bf16_only or name in ("fp8_conv_a", "fp8_conv_b"):
            results[name]["batch1_ms"] = None
            L.nrx_model_destroy(model)
            continue
        # batch-1 latency (the real-time regime: no inter-slot batching)
        d1, s1 = L.make_slots(shapes[:1], m_max)
        ws1 = torch.empty(L.nrx_workspace_bytes(model, d1), dtype=torch.uint8, device="cuda")
        l1 = torch.zeros(s1["llr"], dtype=torch.float32, device="cuda")
        for _ in range(3):
            L.nrx_forward(model, dw, d1, y, l1, ws1)
        torch.cuda.synchronize()
        reps = 3 if name == "fp32" else 20
        e0.record()
        for _ in range(reps):
            L.nrx_forward(model, dw, d1, y, l1, ws1)
        e1.record()
        torch.cuda.synchronize()
        results[name]["batch1_ms"] = e0.elapsed_time(e1) / reps
        del ws, ws1
        L.nrx_model_destroy(model)

    # bit errors: NRX (both precisions) and the LS + LMMSE judge on the same slots
    bws = torch.empty(L.nrx_bce_workspace_bytes(descs, m_max), dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    nerr = torch.zeros(1, dtype=torch.int64, device="cuda")
    n_bits = sum(12 * 12 * s["n_prb"] * sum(s["bits"]) for s in shapes)
    ber = {}
    # fallback policy (Sec. III-B baseline beside the NRX): slots flagged by the pass get the LS + LMMSE LLRs
    lws = torch.empty(L.lmmse_workspace_bytes(descs), dtype=torch.uint8, device="cuda")
    flagged = {}
    for name, l in llrs.items():
        flagged[name] = int((flag_words[name] != 0).sum().item())
        L.nrx_fallback_lmmse(descs, m_max, y, flag_words[name], l, lws, n0=n0)
    for name, l in llrs.items():
        L.nrx_bce(descs, m_max, l, bits, None, loss, nerr, bws)
        torch.cuda.synchronize()
        ber[name] = nerr.item() / n_bits
    llm = torch.zeros(sz["llr"], dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.lmmse_demap(descs, m_max, y, llm, lws, n0=n0)
    torch.cuda.synchronize()
    lmmse_ms = (time.perf_counter() - t0) * 1e3
    L.nrx_bce(descs, m_max, llm, bits, None, loss, nerr, bws)
    torch.cuda.synchronize()
    ber["lmmse"] = nerr.item() / n_bits
    if "fp32" in llrs:
        b32 = ber["fp32"]
        tol = max(0.05 * b32, 3 * math.sqrt(max(b32 * (1 - b32), 1e-30) / n_bits))
        ber["matched"] = abs(ber["bf16"] - b32) <= tol
        for k8 in ("fp8", "fp8_conv_a", "fp8_conv_b"):
            if k8 in ber:
                ber[k8 + "_matched"] = abs(ber[k8] - b32) <= tol
        ber["tolerance"] = tol
        rel_llr = (torch.linalg.vector_norm(llrs["bf16"] - llrs["fp32"]) /
                   torch.linalg.vector_norm(llrs["fp32"])).item()
        rel_llr8 = ((torch.linalg.vector_norm(llrs["fp8"] - llrs["fp32"]) /
                     torch.linalg.vector_norm(llrs["fp32"])).item() if "fp8" in llrs else None)
    else:
        rel_llr = rel_llr8 = None
    ber["n_bits"] = n_bits
    ber["slots_on_lmmse_fallback"] = flagged

    S = 12 * w["n_prb"]
    ms = results["bf16"]["ms_per_step"]
    slots_s = n_slots / (ms * 1e-3)
    fpr = flops_per_row(*net_args)
    rows = S * 14 * w["n_ue"] * n_slots
    # roofline of the dominant kernel: the residual-block 3x3 conv (128 -> 128 channels)
    cb = results["bf16"]["kernels"]["conv_b"]["ms_per_launch"]
    conv_flops = rows * 2 * 9 * w["d"] * w["d"]
    achieved = conv_flops / (cb * 1e-3)
    out = {
        "metric": METRIC,
        "value": slots_s,
        "unit": "slots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"{w['n_prb']} PRB x 14 sym, {w['n_ue']} UE, {w['n_ant']} ant, "
                               f"{2 ** w['m']}-QAM, batch {n_slots} slots",
                   "n_prb": w["n_prb"], "n_ue": w["n_ue"], "n_ant": w["n_ant"], "qam": 2 ** w["m"],
                   "batch_slots": n_slots, "cgnn": {"d": w["d"], "blocks": w["n_blocks"], "mp_rounds": w["n_rounds"]},
                   "weights": "trained (config-5 recipe)" if trained else "seeded He-init (untrained)"},
        "res_per_s": slots_s * S * 14,
        "tflops": fpr * rows / (ms * 1e-3) / 1e12,
        "ber": ber,
        "llr_rel_err_bf16_vs_fp32": rel_llr,
        "llr_rel_err_fp8_vs_fp32": rel_llr8,
        "lmmse_ms": lmmse_ms,
        "conv_variants": results.get("variants"),
        "conv_variant_sweep_ms": results.get("sweep"),
        "kernels_bf16": results["bf16"]["kernels"],
        "batch1_latency_ms": {k: results[k]["batch1_ms"] for k in llrs},
        "roofline": {"bound": "mfma", "kernel": "conv_b (residual add, bf16): " + CONV_VARIANT_KERNELS[results["variants"]["bf16"]["conv_b"]],
                     "achieved": achieved / 1e12,
                     "peak": PEAKS["bf16"] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAKS["bf16"],
                     "traffic": (stored_traffic(results["variants"]["bf16"]["conv_b"])
                                 if args.workload == "m" else None),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE, WRITE_SIZE; profiles/)",
                     "algorithmic_bytes": rows * 768},
    }
    if "fp8" in results:
        ms8 = results["fp8"]["ms_per_step"]
        cb8 = results["fp8"]["kernels"]["conv_b"]["ms_per_launch"]
        out["fp8"] = {"slots_per_s": n_slots / (ms8 * 1e-3), "ms_per_step": ms8, "res_per_s": n_slots * S * 14 / (ms8 * 1e-3),
                      "speedup_vs_bf16": ms / ms8, "kernels": results["fp8"]["kernels"],
                      "act_scales": results.get("fp8_scales"),
                      # E4M3 conv_b: 294,912 FLOP and 768 B per row (E4M3 a in, BF16 residual in,
                      # BF16 h and its E4M3 copy out) -> 384 FLOP/B, below the fp8 ridge of 625: HBM-bound
                      "conv_b_roofline": {"bound": "hbm", "achieved": rows * 768 / (cb8 * 1e-3) / 1e9,
                                          "peak": 8000.0, "unit": "GB/s",
                                          "frac": rows * 768 / (cb8 * 1e-3) / 8e12,
                                          "mfma_frac": conv_flops / (cb8 * 1e-3) / PEAKS["fp8"]}}
    pol = {k: {"fp8_layers": {1: "conv_a", 2: "conv_b", 3: "conv_a + conv_b"}[fp8_masks[k]],
               "slots_per_s": n_slots / (results[k]["ms_per_step"] * 1e-3), "ms_per_step": results[k]["ms_per_step"],
               "speedup_vs_bf16": ms / results[k]["ms_per_step"], "ber": ber.get(k),
               "ber_matched": ber.get(k + "_matched")}
           for k in fp8_masks if k in results}
    if pol:
        out["fp8_policies"] = pol
        ok = [k for k in pol if pol[k]["ber_matched"]]
        if "fp8" in out:   # the fastest E4M3 policy whose BER matches the FP32 pass (null: none does)
            best = max(ok, key=lambda k: pol[k]["slots_per_s"]) if ok else None
            out["fp8"]["matched_ber_policy"] = None if best is None else {
                "fp8_layers": pol[best]["fp8_layers"], "slots_per_s": pol[best]["slots_per_s"],
                "speedup_vs_bf16": pol[best]["speedup_vs_bf16"]}
    if "bf16_persistent" in results:
        msp = results["bf16_persistent"]["ms_per_step"]
        out["bf16_persistent"] = {"slots_per_s": n_slots / (msp * 1e-3), "ms_per_step": msp,
                                  "batch1_ms": results["bf16_persistent"]["batch1_ms"],
                                  "llr_identical_to_layer_path": bool(torch.equal(llrs["bf16_persistent"],
                                                                                  llrs["bf16"]))}
    if "fp32" in results:
        out["fp32"] = {"slots_per_s": n_slots / (results["fp32"]["ms_per_step"] * 1e-3),
                       "ms_per_step": results["fp32"]["ms_per_step"], "kernels": results["fp32"]["kernels"]}
        out["speedup_bf16_vs_fp32"] = results["fp32"]["ms_per_step"] / ms
    progress("ber done")
    if args.ragged_steps > 0:
        out["ragged"] = ragged_batch(args.ragged_steps, args.no_autotune, args.tune_cache)
        progress("uneven batch (per-layer launches) done")
        out["ragged_persistent"] = ragged_batch(args.ragged_steps, args.no_autotune, args.tune_cache, persistent=True)
    progress("uneven batch done")
    if not args.bf16_only:
        out["paper_rt_batch1"] = paper_rt_latency()
        out["depth_latency"] = depth_latency()
        if not args.no_secondary:
            out["secondary"] = secondary_rows(max(3, args.steps // 4), args.tune_cache)
            out["training"] = training_row(max(3, args.steps // 4))
            progress(f"training: {out['training']['ms_per_step']:.2f} ms/step")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, weights, net_args, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
