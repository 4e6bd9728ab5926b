"""Training of the neural receiver on slots generated on the GPU (Sec. II-B).

Every step draws a fresh batch of slots with slot_sim (batch index = step, so a
run is a pure function of the seed and resumes bit-exactly from a checkpoint),
runs nrx_forward keeping activations, the BCE loss on the coded bits of the data
REs (nrx_bce, fp64 reduction), nrx_backward and one Adam step on the fp32 master
weights.  With multi_loss the readout follows every CGNN iteration and the loss is
the sum of their BCEs (Sec. II-B), so the trained network can later run at any
depth (nrx_set_iterations, Sec. IV-B).  With gamma > 0 (the double readout, Sec. II-B) the network also
has ReadoutChEst, and gamma times the MSE between its channel estimate and the true channel of the slot
(slot_sim's h_true, nrx_mse) is added to the loss of every readout.  All work is enqueued on one stream; the host only reads the loss every
`log_every` steps.

    python -m paper_2409_02912_amd.train --workload c5 --steps 2000 --out weights.npy
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2409_02912_amd import libnrx as L  # noqa: E402
from paper_2409_02912_amd import synth  # noqa: E402


def weight_layout(model):
    return [(n, s) for n, _, s in L.weight_layout(model)]


class Trainer:
    def __init__(self, w, precision=L.NRX_BF16, seed=0, lr=1e-3, batch=None, n_prb=None, snr=None,
                 multi_loss=False, data_batches=0, gamma=0.0, mixed_pool=0, var_io=False):
        import torch
        self.torch = torch
        self.w = w
        self.seed = seed
        self.lr = lr
        self.data_batches = data_batches   # > 0: a finite training set of this many batches, cycled
        self.m_max = w["m"]
        if mixed_pool > 0:
            # mixed-MCS training (Sec. III-A): a pool of batches with random U_A, per-UE modulations and SNR
            # offsets, drawn once (each batch shape is planned once) and cycled; the slots are fresh every step
            rng = np.random.default_rng(seed + 7919)
            pool = [synth.mixed_mcs_shapes(w, rng, n_slots=batch, n_prb=n_prb) for _ in range(mixed_pool)]
        else:
            pool = [synth.uniform_shapes(w, n_slots=batch or w["n_slots"], n_prb=n_prb)]
        self.pool = [(shapes,) + L.make_slots(shapes, self.m_max) for shapes in pool]
        sz = {k: max(e[2][k] for e in self.pool) for k in ("y", "h", "llr", "bits")}
        self.shapes, self.descs = self.pool[0][0], self.pool[0][1]
        snr = snr or w["snr"]
        self.sim = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"],
                                rho=w["rho"], snr_db_lo=snr[0], snr_db_hi=snr[1])
        self.gamma = float(gamma)
        self.var_io = var_io   # one ReadoutLLRs per modulation (Sec. III)
        self.model = L.nrx_model_create(w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], self.m_max, precision,
                                        flags=(2 if self.gamma > 0 else 0) | (4 if var_io else 0))

        def pool_max(f):
            return max(f(e[1]) for e in self.pool)
        dev = "cuda"
        self.params = torch.from_numpy(synth.he_weights(weight_layout(self.model), seed)).to(dev)
        # weights before the ReadoutChEst tensors (which close the vector)
        self._n_no_chest = sum(int(np.prod(s)) for n, s in weight_layout(self.model) if not n.startswith("readout_ch"))
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.y = torch.empty(2 * sz["y"], dtype=torch.float32, device=dev)
        self.bits = torch.empty(sz["bits"], dtype=torch.uint8, device=dev)
        # one LLR (and gradient) array per readout: every CGNN iteration with multi_loss, else the last
        self.n_ro = L.nrx_num_iterations(self.model) if multi_loss else 1
        self.multi = multi_loss
        self.stride = sz["llr"]
        self.llr = torch.empty(self.n_ro * sz["llr"], dtype=torch.float32, device=dev)
        self.dllr = torch.empty(self.n_ro * sz["llr"], dtype=torch.float32, device=dev)
        self.losses = torch.zeros(self.n_ro, dtype=torch.float64, device=dev)
        self.loss = self.losses[self.n_ro - 1:]          # BCE of the last readout
        self.nerr = torch.zeros(1, dtype=torch.int64, device=dev)
        if self.gamma > 0:
            # double readout: the true channel, one channel estimate (and gradient) per readout, their MSEs
            self.hstride = 2 * sz["h"]
            self.h_true = torch.empty(self.hstride, dtype=torch.float32, device=dev)
            self.hest = torch.empty(self.n_ro * self.hstride, dtype=torch.float32, device=dev)
            self.dhest = torch.empty_like(self.hest)
            self.mses = torch.zeros(self.n_ro, dtype=torch.float64, device=dev)
            self.mws = torch.empty(pool_max(L.nrx_mse_workspace_bytes), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(pool_max(lambda d: L.nrx_workspace_bytes(self.model, d, save_acts=True)),
                              dtype=torch.uint8, device=dev)
        self.sws = torch.empty(pool_max(lambda d: L.slot_sim_workspace_bytes(self.sim, d)), dtype=torch.uint8,
                               device=dev)
        self.bws = torch.empty(pool_max(lambda d: L.nrx_bce_workspace_bytes(d, self.m_max)), dtype=torch.uint8,
                               device=dev)
        self.step = 0
        self.pool_bits = [sum(12 * 12 * s["n_prb"] * sum(s["bits"]) for s in e[0]) for e in self.pool]
        self.n_bits = self.pool_bits[0]
        # pick the convolution tile shapes for this batch (forward timing only)
        L.slot_sim(self.sim, self.seed, 0, self.descs, self.m_max, self.y, self.sws, bits=self.bits)
        L.nrx_autotune(self.model, self.params, self.descs, self.y, self.llr[:self.stride], self.ws)

    def load(self, path):
        z = np.load(path, allow_pickle=False)
        self.params.copy_(self.torch.from_numpy(z["w"]))
        self.m.copy_(self.torch.from_numpy(z["m"]))
        self.v.copy_(self.torch.from_numpy(z["v"]))
        self.step = int(z["step"])

    def save(self, path):
        np.savez(path, w=self.params.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.int64(self.step))

    def init_from(self, w0):
        """Start from fp32 weights w0; a vector without ReadoutChEst fills the prefix (the head stays He-initialised)."""
        w0 = self.torch.as_tensor(np.asarray(w0, dtype=np.float32))
        if w0.numel() > self.params.numel():
            raise ValueError(f"{w0.numel()} weights for a model of {self.params.numel()}")
        if self.var_io and w0.numel() < self._n_no_chest:
            raise ValueError("a Var-IO model starts from Var-IO weights (the layouts differ)")
        self.params[:w0.numel()].copy_(w0)

    def train_step(self):
        bi = self.step % self.data_batches if self.data_batches else self.step
        if len(self.pool) > 1:
            p = bi % len(self.pool)
            self.shapes, self.descs, self.n_bits = self.pool[p][0], self.pool[p][1], self.pool_bits[p]
        L.slot_sim(self.sim, self.seed, bi, self.descs, self.m_max, self.y, self.sws, bits=self.bits,
                   h_true=self.h_true if self.gamma > 0 else None)
        if self.gamma > 0:
            lstride = self.stride if self.multi else 0
            hstride = self.hstride if self.multi else 0
            L.nrx_forward_chest(self.model, self.params, self.descs, self.y, self.llr, self.hest, self.ws,
                                llr_stride=lstride, h_stride=hstride, save_acts=True)
            for k in range(self.n_ro):
                sl = slice(k * self.stride, (k + 1) * self.stride)
                hs = slice(k * self.hstride, (k + 1) * self.hstride)
                L.nrx_bce(self.descs, self.m_max, self.llr[sl], self.bits, self.dllr[sl], self.losses[k:k + 1],
                          self.nerr, self.bws)
                L.nrx_mse(self.descs, self.hest[hs], self.h_true, self.gamma, self.dhest[hs], self.mses[k:k + 1],
                          self.mws)
            L.nrx_backward_chest(self.model, self.params, self.descs, self.dllr, self.dhest, self.grad, self.ws,
                                 llr_stride=lstride, h_stride=hstride)
        elif self.multi:
            L.nrx_forward_iters(self.model, self.params, self.descs, self.y, self.llr, self.stride, self.ws,
                                save_acts=True)
            for k in range(self.n_ro):
                sl = slice(k * self.stride, (k + 1) * self.stride)
                L.nrx_bce(self.descs, self.m_max, self.llr[sl], self.bits, self.dllr[sl], self.losses[k:k + 1],
                          self.nerr, self.bws)
            L.nrx_backward_iters(self.model, self.params, self.descs, self.dllr, self.stride, self.grad, self.ws)
        else:
            L.nrx_forward(self.model, self.params, self.descs, self.y, self.llr, self.ws, save_acts=True)
            L.nrx_bce(self.descs, self.m_max, self.llr, self.bits, self.dllr, self.loss, self.nerr, self.bws)
            L.nrx_backward(self.model, self.params, self.descs, self.dllr, self.grad, self.ws)
        self.step += 1
        L.nrx_adam(self.params, self.grad, self.m, self.v, self.step, lr=self.lr_at(self.step))

    def lr_at(self, step):
        """Learning rate of an Adam step: self.lr, or with a schedule set by set_schedule a linear warm-up over
        `warmup` steps from its start, then a cosine decay to lr_final at step `end` (steps before the start
        take the schedule's first rate)."""
        sch = getattr(self, "schedule", None)
        if not sch:
            return self.lr
        k = max(step - sch["start"], 0)
        if k < sch["warmup"]:
            return self.lr * (k + 1) / sch["warmup"]
        span = max(sch["end"] - sch["start"] - sch["warmup"], 1)
        f = min(max((k - sch["warmup"]) / span, 0.0), 1.0)
        return sch["lr_final"] + 0.5 * (self.lr - sch["lr_final"]) * (1.0 + math.cos(math.pi * f))

    def set_schedule(self, start, end, warmup=0, lr_final=None):
        self.schedule = {"start": int(start), "end": int(end), "warmup": int(warmup),
                         "lr_final": self.lr if lr_final is None else float(lr_final)}

    def close(self):
        L.nrx_model_destroy(self.model)


def evaluate(w_params, w, seed, batches, snr_db, precision=L.NRX_BF16, batch=None, n_prb=None, n_iter=0, bits=None,
             var_io=False):
    """BER of the NRX and of LS + LMMSE on held-out slots (a seed not used in training) at a fixed SNR;
    n_iter > 0 runs the NRX at that many CGNN iterations; bits sets every UE's modulation (default the workload's,
    which is also the network's LLR count m_max: lower orders read the first bits outputs, Sec. III)."""
    import torch
    m_max = w["m"]
    shapes = synth.uniform_shapes(w, n_slots=batch or w["n_slots"], n_prb=n_prb, bits=bits)
    descs, sz = L.make_slots(shapes, m_max)
    sim = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"], rho=w["rho"],
                       snr_db_lo=snr_db, snr_db_hi=snr_db)
    model = L.nrx_model_create(w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], m_max, precision,
                               flags=4 if var_io else 0)
    try:
        L.nrx_set_iterations(model, n_iter)
        dev = "cuda"
        params = w_params if isinstance(w_params, torch.Tensor) else torch.from_numpy(w_params).to(dev)
        y = torch.empty(2 * sz["y"], dtype=torch.float32, device=dev)
        bits = torch.empty(sz["bits"], dtype=torch.uint8, device=dev)
        n0 = torch.empty(len(shapes), dtype=torch.float32, device=dev)
        llr = torch.empty(sz["llr"], dtype=torch.float32, device=dev)
        ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device=dev)
        sws = torch.empty(L.slot_sim_workspace_bytes(sim, descs), dtype=torch.uint8, device=dev)
        bws = torch.empty(L.nrx_bce_workspace_bytes(descs, m_max), dtype=torch.uint8, device=dev)
        lws = torch.empty(L.lmmse_workspace_bytes(descs), dtype=torch.uint8, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        nerr = torch.zeros(1, dtype=torch.int64, device=dev)
        n_bits = sum(12 * 12 * s["n_prb"] * sum(s["bits"]) for s in shapes)
        e_nrx = e_lmmse = 0
        bce = 0.0
        for b in range(batches):
            L.slot_sim(sim, seed, b, descs, m_max, y, sws, bits=bits, n0=n0)
            L.nrx_forward(model, params, descs, y, llr, ws)
            L.nrx_bce(descs, m_max, llr, bits, None, loss, nerr, bws)
            torch.cuda.synchronize()
            e_nrx += nerr.item()
            bce += loss.item()
            L.lmmse_demap(descs, m_max, y, llr, lws, n0=n0)
            L.nrx_bce(descs, m_max, llr, bits, None, loss, nerr, bws)
            torch.cuda.synchronize()
            e_lmmse += nerr.item()
        n = batches * n_bits
        return {"ber_nrx": e_nrx / n, "ber_lmmse": e_lmmse / n, "bce_nrx": bce / batches, "n_bits": n}
    finally:
        L.nrx_model_destroy(model)


def evaluate_chest(w_params, w, seed, batches, snr_db, precision=L.NRX_BF16, batch=None, n_prb=None, var_io=False):
    """Held-out channel-estimation MSE (mean |ĥ - h|^2 over the batch's complex entries) of the ReadoutChEst output
    after the last CGNN iteration, next to that of the LS estimate with linear interpolation the network starts from
    (Sec. II-A), on fresh slots at one SNR; and the BER of LMMSE equalisation + max-log demapping (genie N0) given
    either estimate, i.e. what the refined estimate is worth to a classical receiver."""
    import torch
    dev = "cuda"
    m_max = w["m"]
    shapes = synth.uniform_shapes(w, n_slots=batch or w["n_slots"], n_prb=n_prb)
    descs, sz = L.make_slots(shapes, m_max)
    sim = L.sim_config(n_taps=w["n_taps"], tap_decay_ns=w["decay_ns"], doppler_max_hz=w["doppler"], rho=w["rho"],
                       snr_db_lo=snr_db, snr_db_hi=snr_db)
    model = L.nrx_model_create(w["n_ant"], w["d"], w["n_blocks"], w["n_rounds"], m_max, precision,
                               flags=6 if var_io else 2)
    try:
        params = torch.as_tensor(w_params, dtype=torch.float32, device=dev)
        if params.numel() != L.nrx_weight_count(model):
            raise ValueError("the weights have no ReadoutChEst")
        y = torch.empty(2 * sz["y"], dtype=torch.float32, device=dev)
        h_true = torch.empty(2 * sz["h"], dtype=torch.float32, device=dev)
        h_ls = torch.empty_like(h_true)
        hest = torch.empty_like(h_true)
        llr = torch.empty(sz["llr"], dtype=torch.float32, device=dev)
        ws = torch.empty(L.nrx_workspace_bytes(model, descs), dtype=torch.uint8, device=dev)
        sws = torch.empty(L.slot_sim_workspace_bytes(sim, descs), dtype=torch.uint8, device=dev)
        mws = torch.empty(L.nrx_mse_workspace_bytes(descs), dtype=torch.uint8, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        bits = torch.empty(sz["bits"], dtype=torch.uint8, device=dev)
        n0 = torch.empty(len(shapes), dtype=torch.float32, device=dev)
        llm = torch.empty(sz["llr"], dtype=torch.float32, device=dev)
        lws = torch.empty(L.lmmse_workspace_bytes(descs), dtype=torch.uint8, device=dev)
        bws = torch.empty(L.nrx_bce_workspace_bytes(descs, m_max), dtype=torch.uint8, device=dev)
        nerr = torch.zeros(1, dtype=torch.int64, device=dev)
        m_nrx = m_ls = 0.0
        e_ls = e_ref = n_bits = 0
        for b in range(batches):
            L.slot_sim(sim, seed, b, descs, m_max, y, sws, h_true=h_true, bits=bits, n0=n0)
            L.nrx_forward_chest(model, params, descs, y, llr, hest, ws, h_ls=h_ls)
            L.nrx_mse(descs, hest, h_true, 1.0, None, loss, mws)
            torch.cuda.synchronize()
            m_nrx += loss.item()
            L.nrx_mse(descs, h_ls, h_true, 1.0, None, loss, mws)
            torch.cuda.synchronize()
            m_ls += loss.item()
            for h, acc in ((h_ls, "ls"), (hest, "ref")):
                L.lmmse_demap(descs, m_max, y, llm, lws, h=h, n0=n0)
                L.nrx_bce(descs, m_max, llm, bits, None, loss, nerr, bws)
                torch.cuda.synchronize()
                if acc == "ls":
                    e_ls += nerr.item()
                else:
                    e_ref += nerr.item()
            n_bits += sum(12 * 12 * s["n_prb"] * sum(s["bits"]) for s in shapes)
        return {"mse_nrx": m_nrx / batches, "mse_ls": m_ls / batches,
                "ber_lmmse_ls": e_ls / n_bits, "ber_lmmse_refined": e_ref / n_bits}
    finally:
        L.nrx_model_destroy(model)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--n-prb", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--ckpt", default=None, help="checkpoint (.npz) to resume from and to write")
    ap.add_argument("--out", default=None, help="write the trained fp32 weights (.npy)")
    ap.add_argument("--log-every", type=int, default=50)
    ap.add_argument("--ckpt-every", type=int, default=500)
    ap.add_argument("--time-limit", type=float, default=1e9, help="stop (and checkpoint) after this many seconds")
    ap.add_argument("--eval-batches", type=int, default=0)
    ap.add_argument("--eval-snr", type=float, default=10.0)
    ap.add_argument("--multi-loss", action="store_true", help="readout and BCE after every CGNN iteration")
    ap.add_argument("--mixed-pool", type=int, default=0,
                    help="mixed-MCS training: cycle this many pre-drawn batch shapes (workloads with an mcs set)")
    ap.add_argument("--var-io", action="store_true", help="one ReadoutLLRs per modulation (Var-IO output layers)")
    ap.add_argument("--gamma", type=float, default=0.0,
                    help="double readout: add gamma x the channel-estimate MSE of ReadoutChEst to the loss")
    ap.add_argument("--init", default=None, help="start from these fp32 weights (.npy), e.g. to fine-tune")
    ap.add_argument("--data-batches", type=int, default=0, help="train on a finite set of this many batches")
    ap.add_argument("--eval-every", type=int, default=0, help="evaluate every this many steps (and at the start)")
    ap.add_argument("--lr-final", type=float, default=None,
                    help="cosine decay of the learning rate from --lr to this value at --steps")
    ap.add_argument("--schedule-start", type=int, default=None,
                    help="step at which the warm-up and decay begin (default: the step the run starts at)")
    ap.add_argument("--warmup", type=int, default=0, help="linear learning-rate warm-up steps")
    ap.add_argument("--eval-workloads", default=None,
                    help="comma-separated workloads to evaluate on (default: the training workload)")
    args = ap.parse_args()
    import torch
    w = synth.WORKLOADS[args.workload]
    prec = L.NRX_BF16 if args.precision == "bf16" else L.NRX_FP32
    tr = Trainer(w, prec, args.seed, args.lr, args.batch, args.n_prb, multi_loss=args.multi_loss,
                 data_batches=args.data_batches, gamma=args.gamma, mixed_pool=args.mixed_pool, var_io=args.var_io)
    if args.ckpt and os.path.exists(args.ckpt):
        tr.load(args.ckpt)
        print(json.dumps({"resumed_at": tr.step}), flush=True)
    elif args.init:
        tr.init_from(np.load(args.init, allow_pickle=False))
        print(json.dumps({"init": args.init}), flush=True)
    evals = (args.eval_workloads or args.workload).split(",")
    if args.lr_final is not None or args.warmup:
        s0 = tr.step if args.schedule_start is None else args.schedule_start
        tr.set_schedule(s0, args.steps, args.warmup, args.lr_final)

    def eval_all():
        if args.gamma > 0:
            r = evaluate_chest(tr.params, w, seed=args.seed + 1000003, batches=args.eval_batches, snr_db=args.eval_snr,
                               precision=prec, batch=args.batch, n_prb=args.n_prb, var_io=args.var_io)
            print(json.dumps({"eval_chest": r, "snr_db": args.eval_snr, "step": tr.step}), flush=True)
        for name in evals:
            we = synth.WORKLOADS[name]
            for k in range(1, tr.n_ro + 1) if args.multi_loss else [0]:
                for bits in we.get("mcs", [None]):   # mixed-MCS workloads: every modulation on its own
                    r = evaluate(tr.params, we, seed=args.seed + 1000003, batches=args.eval_batches,
                                 snr_db=args.eval_snr, precision=prec, batch=args.batch, n_prb=args.n_prb, n_iter=k,
                                 bits=bits, var_io=args.var_io)
                    print(json.dumps({"eval": r, "workload": name, "snr_db": args.eval_snr, "step": tr.step,
                                      "n_iter": k, "bits": bits}), flush=True)
    t0 = time.time()
    start = tr.step
    if args.eval_every and args.eval_batches:
        eval_all()
    while tr.step < args.steps:
        tr.train_step()
        if args.eval_every and args.eval_batches and tr.step % args.eval_every == 0:
            eval_all()
        if tr.step % args.log_every == 0 or tr.step == args.steps:
            torch.cuda.synchronize()
            el = time.time() - t0
            rec = {"step": tr.step, "loss": tr.loss.item(), "losses": tr.losses.tolist(),
                   "ber": tr.nerr.item() / tr.n_bits, "s_per_step": el / max(tr.step - start, 1),
                   "lr": tr.lr_at(tr.step)}
            if tr.gamma > 0:
                rec["mse"] = tr.mses.tolist()
            print(json.dumps(rec), flush=True)
        if args.ckpt and tr.step % args.ckpt_every == 0:
            tr.save(args.ckpt)
        if time.time() - t0 > args.time_limit:
            break
    torch.cuda.synchronize()
    if args.ckpt:
        tr.save(args.ckpt)
    if args.out:
        np.save(args.out, tr.params.cpu().numpy())
    if args.eval_batches and not (args.eval_every and tr.step % args.eval_every == 0):
        eval_all()
    tr.close()


if __name__ == "__main__":
    main()
