"""Neural receiver (CGNN) forward, backward, loss and Adam step (oracle side), fp64.

TEST INFRASTRUCTURE ONLY (oracle).

Structure (Sec. II-A, Fig. 1): StateInit, a small CNN over the whole resource
grid mapping [received signal, per-UE LS estimate, positional encoding of the
distance to the pilots] to a real state of depth d per UE and RE; N_it CGNN
iterations, each a message-passing step (an MLP turns every UE's state into a
message; each UE receives the sum of the messages of all *other* UEs) followed by
a CNN that updates the state from [previous state, aggregated messages, PE];
and ReadoutLLRs, an MLP from the final state to m LLRs per UE and RE.  With the
double readout (Sec. II-A, II-B) a second MLP, ReadoutChEst, maps the same state to
a refined channel estimate per UE, RE and antenna, trained by a gamma-scaled MSE
against the true channel added to the BCE.  Under Var-IO (Sec. III) every
modulation has its own StateInit and its own ReadoutLLRs with just its m outputs, the
CGNN iterations shared.  Unused
higher-order LLR outputs are masked for lower-order QAM (Sec. III).  Training
minimises the BCE between LLRs and bit labels, averaged over the batch
(Sec. II-B).

Readings where the paper gives no detail (layer forms, widths, the block
structure) are fixed here and listed in the design notes:
  * 3x3 "same" cross-correlation over (subcarrier, symbol), zero outside the grid;
    complex inputs enter as separate real and imaginary channels;
  * StateInit = one 3x3 conv, (4B+2) -> d, inputs [Re y, Im y, Re Ĥ_u, Im Ĥ_u, pe_t, pe_f];
  * C residual blocks h <- h + conv_b(ReLU(LN(conv_a(in)))), LN over the d
    channels of one RE (biased variance, eps 1e-5, affine);
  * R message-passing rounds, round r placed before block floor(r*C/R); the first
    conv of that block sees [h, agg, pe_t, pe_f] (2d+2 channels), others see h;
  * MP MLP m = W2 ReLU(W1 h + b1) + b2 (d -> d -> d); readout d -> d -> m_max;
  * ReadoutChEst d -> d -> 2B, the same two-layer form, outputs interleaved
    (Re h_b, Im h_b) per antenna b; MSE = mean over the slot's complex entries of |ĥ - h|^2;
  * PE: pe_t = standardised distance (in symbols) to the nearest DMRS symbol,
    pe_f = +1/-1 for REs off/on this UE's DMRS comb.
"""
import numpy as np

from . import nr

EPS_LN = 1e-5


class NetConfig:
    def __init__(self, n_ant, d, n_blocks, n_rounds, m_max, chest=False, var_io=False):
        self.B = n_ant
        self.d = d
        self.C = n_blocks
        self.R = n_rounds
        self.m_max = m_max
        self.chest = chest      # second readout (ReadoutChEst)
        self.var_io = var_io    # one ReadoutLLRs per modulation (Var-IO output layers)

    def mods(self):
        """Modulations (bits per symbol) with a ReadoutLLRs of their own under Var-IO."""
        return list(range(2, self.m_max + 1, 2))

    def mp_blocks(self):
        return [(r * self.C) // self.R for r in range(self.R)]


def layout(cfg):
    """Ordered list of (name, shape) of the flat weight vector."""
    d, B = cfg.d, cfg.B
    mpb = cfg.mp_blocks()
    if cfg.var_io:
        L = []
        for m in cfg.mods():
            L += [(f"conv_in.m{m}.w", (3, 3, 4 * B + 2, d)), (f"conv_in.m{m}.b", (d,))]
    else:
        L = [("conv_in.w", (3, 3, 4 * B + 2, d)), ("conv_in.b", (d,))]
    for i in range(cfg.C):
        cin = 2 * d + 2 if i in mpb else d
        L += [(f"blk{i}.conv_a.w", (3, 3, cin, d)), (f"blk{i}.conv_a.b", (d,)),
              (f"blk{i}.ln.g", (d,)), (f"blk{i}.ln.b", (d,)),
              (f"blk{i}.conv_b.w", (3, 3, d, d)), (f"blk{i}.conv_b.b", (d,))]
    for r in range(cfg.R):
        L += [(f"mp{r}.w1", (d, d)), (f"mp{r}.b1", (d,)), (f"mp{r}.w2", (d, d)), (f"mp{r}.b2", (d,))]
    if cfg.var_io:
        for m in cfg.mods():
            L += [(f"readout.m{m}.w1", (d, d)), (f"readout.m{m}.b1", (d,)),
                  (f"readout.m{m}.w2", (d, m)), (f"readout.m{m}.b2", (m,))]
    else:
        L += [("readout.w1", (d, d)), ("readout.b1", (d,)),
              ("readout.w2", (d, cfg.m_max)), ("readout.b2", (cfg.m_max,))]
    if cfg.chest:
        L += [("readout_ch.w1", (d, d)), ("readout_ch.b1", (d,)),
              ("readout_ch.w2", (d, 2 * B)), ("readout_ch.b2", (2 * B,))]
    return L


def n_params(cfg):
    return int(sum(np.prod(s) for _, s in layout(cfg)))


def unflatten(w, cfg):
    out, off = {}, 0
    for name, shape in layout(cfg):
        n = int(np.prod(shape))
        out[name] = np.asarray(w[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    return out


def flatten(tensors, cfg):
    return np.concatenate([np.asarray(tensors[name], dtype=np.float64).reshape(-1)
                           for name, _ in layout(cfg)])


# ----------------------------------------------------------- building blocks ---

def positional_encoding(n_sc, n_ue):
    """pe[s, t, u, 2]: (pe_t, pe_f)."""
    t = np.arange(nr.N_SYMB)
    dist_t = np.min(np.abs(t[:, None] - np.array(nr.DMRS_SYMBOLS)[None, :]), axis=1).astype(np.float64)
    pe_t = (dist_t - dist_t.mean()) / dist_t.std()
    pe = np.zeros((n_sc, nr.N_SYMB, n_ue, 2))
    s = np.arange(n_sc)
    for u in range(n_ue):
        dist_f = ((s - nr.cdm_group(u)) % 2).astype(np.float64)
        pe[:, :, u, 0] = pe_t[None, :]
        pe[:, :, u, 1] = (2.0 * dist_f - 1.0)[:, None]
    return pe


def conv3x3(x, w, b):
    """out[s,t,...,o] = b_o + sum_{i,j in 0..2} sum_c w[i,j,c,o] x[s+i-1, t+j-1, ..., c]; zero outside."""
    S, T = x.shape[0], x.shape[1]
    xp = np.zeros((S + 2, T + 2) + x.shape[2:])
    xp[1:-1, 1:-1] = x
    out = np.zeros(x.shape[:-1] + (w.shape[-1],)) + b
    for i in range(3):
        for j in range(3):
            out += xp[i:i + S, j:j + T] @ w[i, j]
    return out


def conv3x3_backward(x, w, dout):
    S, T = x.shape[0], x.shape[1]
    xp = np.zeros((S + 2, T + 2) + x.shape[2:])
    xp[1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for i in range(3):
        for j in range(3):
            dxp[i:i + S, j:j + T] += dout @ w[i, j].T
            xs = xp[i:i + S, j:j + T].reshape(-1, x.shape[-1])
            dw[i, j] = xs.T @ dout.reshape(-1, dout.shape[-1])
    db = dout.reshape(-1, dout.shape[-1]).sum(axis=0)
    return dxp[1:-1, 1:-1], dw, db


def layer_norm(z, g, b):
    mu = z.mean(axis=-1, keepdims=True)
    var = ((z - mu) ** 2).mean(axis=-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + EPS_LN)
    zhat = (z - mu) * rstd
    return zhat * g + b, (zhat, rstd)


def layer_norm_backward(dy, g, cache):
    zhat, rstd = cache
    dg = (dy * zhat).reshape(-1, zhat.shape[-1]).sum(axis=0)
    db = dy.reshape(-1, zhat.shape[-1]).sum(axis=0)
    dzhat = dy * g
    n = zhat.shape[-1]
    dz = rstd * (dzhat - dzhat.mean(axis=-1, keepdims=True)
                 - zhat * (dzhat * zhat).mean(axis=-1, keepdims=True))
    return dz, dg, db


def relu(x):
    return np.maximum(x, 0.0)


def aggregate_others(m):
    """agg[..., u, :] = sum over u' != u of m[..., u', :]  (axis -2 is the UE axis)."""
    U = m.shape[-2]
    agg = np.zeros_like(m)
    for u in range(U):
        for v in range(U):
            if v != u:
                agg[..., u, :] += m[..., v, :]
    return agg


# -------------------------------------------------------------------- model ---

def nrx_inputs(y, h_ls, cfg):
    """X[s, t, u, 4B+2] = [Re y, Im y, Re Ĥ_u, Im Ĥ_u, pe_t, pe_f]; antennas beyond the slot's are zero."""
    S, T, Bs = y.shape
    U = h_ls.shape[2]
    B = cfg.B
    X = np.zeros((S, T, U, 4 * B + 2))
    X[:, :, :, 0:Bs] = y.real[:, :, None, :]
    X[:, :, :, B:B + Bs] = y.imag[:, :, None, :]
    X[:, :, :, 2 * B:2 * B + Bs] = h_ls.real
    X[:, :, :, 3 * B:3 * B + Bs] = h_ls.imag
    X[:, :, :, 4 * B:] = positional_encoding(S, U)
    return X


def iteration_ends(cfg):
    """Number of conv blocks completed at the end of each CGNN iteration.  An iteration is one
    message-passing round followed by the state-update blocks up to the next round (Sec. II-A), so
    iteration r ends where round r + 1 begins; a network without message passing is one iteration."""
    if cfg.R == 0:
        return [cfg.C]
    return [((r + 1) * cfg.C) // cfg.R for r in range(cfg.R)]


def readout_weights(cfg, m):
    """Names of the ReadoutLLRs tensors that serve a UE with m bits per symbol (Var-IO: its modulation's own)."""
    p = f"readout.m{m}." if cfg.var_io else "readout."
    return p + "w1", p + "b1", p + "w2", p + "b2"


def readout(W, cfg, h, mask):
    """ReadoutLLRs on the state h [S, T, U, d] -> masked llr [U, T, S, m_max] and (h, r1, q).  Under Var-IO each UE
    goes through the readout of its modulation (m_u outputs; the rest of the m_max are zero)."""
    if not cfg.var_io:
        r1 = h @ W["readout.w1"] + W["readout.b1"]
        q = relu(r1)
        out = q @ W["readout.w2"] + W["readout.b2"]          # [S, T, U, m_max]
        return np.transpose(out, (2, 1, 0, 3)) * mask[:, None, None, :], (h, r1, q)
    S, T, U, d = h.shape
    r1 = np.zeros_like(h)
    out = np.zeros((S, T, U, cfg.m_max))
    for u in range(U):
        m = int(mask[u].sum())
        w1, b1, w2, b2 = readout_weights(cfg, m)
        r1[:, :, u] = h[:, :, u] @ W[w1] + W[b1]
        out[:, :, u, :m] = relu(r1[:, :, u]) @ W[w2] + W[b2]
    return np.transpose(out, (2, 1, 0, 3)), (h, r1, relu(r1))


def readout_chest(W, h, n_ant):
    """ReadoutChEst on the state h [S, T, U, d] -> channel estimate [S, T, U, n_ant] (complex) and
    (h, r1, q); outputs 2b and 2b + 1 are the real and imaginary part for antenna b."""
    r1 = h @ W["readout_ch.w1"] + W["readout_ch.b1"]
    q = relu(r1)
    out = q @ W["readout_ch.w2"] + W["readout_ch.b2"]    # [S, T, U, 2B]
    return out[..., 0:2 * n_ant:2] + 1j * out[..., 1:2 * n_ant:2], (h, r1, q)


def forward(W, cfg, y, h_ls, bits_per_sym, keep=False, n_iter=None, all_iters=False):
    """One slot. y [S,T,Bs], h_ls [S,T,U,Bs] -> llr [U, T, S, m_max] (masked) (+ cache)."""
    return forward_x(W, cfg, nrx_inputs(y, h_ls, cfg), bits_per_sym, keep, n_iter, all_iters, y.shape[2])


def forward_x(W, cfg, X, bits_per_sym, keep=False, n_iter=None, all_iters=False, n_ant=None):
    """Same as forward() from the stacked input features X[s, t, u, 4B+2].

    n_iter runs only the first n_iter CGNN iterations and reads out after the last of them
    (inference-time depth control, Sec. IV-B); all_iters returns the list of LLRs read out after
    every iteration run (the multi-loss of Sec. II-B uses all of them), the readout layers shared.
    With cfg.chest every readout also applies ReadoutChEst; its estimates for the slot's n_ant
    antennas are in cache["hests"] (one per readout)."""
    U = X.shape[2]
    n_ant = cfg.B if n_ant is None else n_ant
    ends = iteration_ends(cfg)
    n_iter = len(ends) if n_iter is None else n_iter
    assert 1 <= n_iter <= len(ends)
    c_run = ends[n_iter - 1]
    mask = np.zeros((U, cfg.m_max))
    for u in range(U):
        mask[u, :bits_per_sym[u]] = 1.0
    pe = X[..., 4 * cfg.B:]
    cache = {"X": X, "mask": mask, "c_run": c_run, "readouts": [], "hests": [], "chest": []}
    if cfg.var_io:
        # Var-IO input layers: every UE's state starts from its modulation's own StateInit
        h = np.zeros(X.shape[:3] + (cfg.d,))
        for m in sorted(set(bits_per_sym[:U])):
            us = [u for u in range(U) if bits_per_sym[u] == m]
            h[:, :, us] = conv3x3(X[:, :, us], W[f"conv_in.m{m}.w"], W[f"conv_in.m{m}.b"])
    else:
        h = conv3x3(X, W["conv_in.w"], W["conv_in.b"])
    cache["h0"] = h
    mpb = cfg.mp_blocks()
    llrs = []
    for i in range(c_run):
        if i in mpb:
            r = mpb.index(i)
            a1 = h @ W[f"mp{r}.w1"] + W[f"mp{r}.b1"]
            m1 = relu(a1)
            msg = m1 @ W[f"mp{r}.w2"] + W[f"mp{r}.b2"]
            agg = aggregate_others(msg)
            xin = np.concatenate([h, agg, pe], axis=-1)
            cache[f"mp{r}"] = (h, a1, m1)
        else:
            xin = h
        z = conv3x3(xin, W[f"blk{i}.conv_a.w"], W[f"blk{i}.conv_a.b"])
        n, lnc = layer_norm(z, W[f"blk{i}.ln.g"], W[f"blk{i}.ln.b"])
        a = relu(n)
        h_new = h + conv3x3(a, W[f"blk{i}.conv_b.w"], W[f"blk{i}.conv_b.b"])
        cache[f"blk{i}"] = (xin, n, lnc, a)
        h = h_new
        if (all_iters and i + 1 in ends) or i + 1 == c_run:
            llr, rc = readout(W, cfg, h, mask)
            llrs.append(llr)
            cache["readouts"].append((i + 1, rc))
            if cfg.chest:
                he, cc = readout_chest(W, h, n_ant)
                cache["hests"].append(he)
                cache["chest"].append(cc)
    cache["readout"] = cache["readouts"][-1][1]
    res = llrs if all_iters else llrs[-1]
    return (res, cache) if keep else res


def backward(W, cfg, cache, dllr, dhest=None):
    """Gradients of sum_k sum(dllr_k * llr_k) w.r.t. every weight tensor (dict), over the readouts the
    forward took (dllr is one array for a single readout, or a list aligned with them).  dhest (same
    form, complex [S, T, U, n_ant]: real part the gradient w.r.t. Re ĥ, imaginary part w.r.t. Im ĥ)
    adds the term sum(Re dhest * Re ĥ + Im dhest * Im ĥ) of the ReadoutChEst outputs."""
    G = {k: np.zeros_like(v) for k, v in W.items()}
    dl = dllr if isinstance(dllr, list) else [dllr]
    at = [c for c, _ in cache["readouts"]]
    assert len(dl) == len(at)
    dhe = None if dhest is None else (dhest if isinstance(dhest, list) else [dhest])
    assert dhe is None or len(dhe) == len(at)

    def chest_back(k):
        h, r1, q = cache["chest"][k]
        nb = dhe[k].shape[-1]
        dout = np.zeros(q.shape[:-1] + (2 * cfg.B,))
        dout[..., 0:2 * nb:2] = dhe[k].real
        dout[..., 1:2 * nb:2] = dhe[k].imag
        G["readout_ch.w2"] += q.reshape(-1, q.shape[-1]).T @ dout.reshape(-1, dout.shape[-1])
        G["readout_ch.b2"] += dout.reshape(-1, dout.shape[-1]).sum(axis=0)
        dr1 = (dout @ W["readout_ch.w2"].T) * (r1 > 0)
        G["readout_ch.w1"] += h.reshape(-1, h.shape[-1]).T @ dr1.reshape(-1, dr1.shape[-1])
        G["readout_ch.b1"] += dr1.reshape(-1, dr1.shape[-1]).sum(axis=0)
        return dr1 @ W["readout_ch.w1"].T

    def readout_back(k):
        dout = np.transpose(dl[k] * cache["mask"][:, None, None, :], (2, 1, 0, 3))   # [S, T, U, m]
        h, r1, q = cache["readouts"][k][1]
        if cfg.var_io:
            dh_ = np.zeros_like(h)
            for u in range(h.shape[2]):
                m = int(cache["mask"][u].sum())
                w1, b1, w2, b2 = readout_weights(cfg, m)
                du = dout[:, :, u, :m].reshape(-1, m)
                qu, hu = q[:, :, u].reshape(-1, h.shape[-1]), h[:, :, u].reshape(-1, h.shape[-1])
                G[w2] += qu.T @ du
                G[b2] += du.sum(axis=0)
                dr1 = (du @ W[w2].T) * (r1[:, :, u].reshape(-1, h.shape[-1]) > 0)
                G[w1] += hu.T @ dr1
                G[b1] += dr1.sum(axis=0)
                dh_[:, :, u] = (dr1 @ W[w1].T).reshape(h.shape[0], h.shape[1], -1)
            return dh_
        G["readout.w2"] += q.reshape(-1, q.shape[-1]).T @ dout.reshape(-1, dout.shape[-1])
        G["readout.b2"] += dout.reshape(-1, dout.shape[-1]).sum(axis=0)
        dq = dout @ W["readout.w2"].T
        dr1 = dq * (r1 > 0)
        G["readout.w1"] += h.reshape(-1, h.shape[-1]).T @ dr1.reshape(-1, dr1.shape[-1])
        G["readout.b1"] += dr1.reshape(-1, dr1.shape[-1]).sum(axis=0)
        return dr1 @ W["readout.w1"].T

    d = cfg.d
    mpb = cfg.mp_blocks()
    dh = 0.0
    for i in reversed(range(cache["c_run"])):
        if i + 1 in at:
            dh = dh + readout_back(at.index(i + 1))
            if dhe is not None:
                dh = dh + chest_back(at.index(i + 1))
        xin, n, lnc, a = cache[f"blk{i}"]
        # h_new = h + conv_b(a)
        da, G[f"blk{i}.conv_b.w"], G[f"blk{i}.conv_b.b"] = conv3x3_backward(a, W[f"blk{i}.conv_b.w"], dh)
        dn = da * (n > 0)
        dz, G[f"blk{i}.ln.g"], G[f"blk{i}.ln.b"] = layer_norm_backward(dn, W[f"blk{i}.ln.g"], lnc)
        dxin, G[f"blk{i}.conv_a.w"], G[f"blk{i}.conv_a.b"] = conv3x3_backward(xin, W[f"blk{i}.conv_a.w"], dz)
        if i in mpb:
            r = mpb.index(i)
            hprev, a1, m1 = cache[f"mp{r}"]
            dh = dh + dxin[..., :d]
            dagg = dxin[..., d:2 * d]
            dmsg = aggregate_others(dagg)        # agg_u = sum_{v != u} m_v  =>  dm_v = sum_{u != v} dagg_u
            G[f"mp{r}.w2"] = m1.reshape(-1, d).T @ dmsg.reshape(-1, d)
            G[f"mp{r}.b2"] = dmsg.reshape(-1, d).sum(axis=0)
            dm1 = dmsg @ W[f"mp{r}.w2"].T
            da1 = dm1 * (a1 > 0)
            G[f"mp{r}.w1"] = hprev.reshape(-1, d).T @ da1.reshape(-1, d)
            G[f"mp{r}.b1"] = da1.reshape(-1, d).sum(axis=0)
            dh = dh + da1 @ W[f"mp{r}.w1"].T
        else:
            dh = dh + dxin
    if cfg.var_io:
        bps = [int(x) for x in cache["mask"].sum(axis=1)]
        for m in sorted(set(bps)):
            us = [u for u in range(len(bps)) if bps[u] == m]
            _, G[f"conv_in.m{m}.w"], G[f"conv_in.m{m}.b"] = conv3x3_backward(
                cache["X"][:, :, us], W[f"conv_in.m{m}.w"], dh[:, :, us])
    else:
        _, G["conv_in.w"], G["conv_in.b"] = conv3x3_backward(cache["X"], W["conv_in.w"], dh)
    return G


# --------------------------------------------------------------- training ---

def bit_labels_grid(bits, n_sc, m_max):
    """bits [U, n_data, m_max] -> labels [U, T, S, m_max] and a mask of the data REs."""
    U = bits.shape[0]
    lab = np.zeros((U, nr.N_SYMB, n_sc, m_max))
    msk = np.zeros((U, nr.N_SYMB, n_sc, 1))
    for k, t in enumerate(nr.data_symbols()):
        lab[:, t] = bits[:, k * n_sc:(k + 1) * n_sc, :]
        msk[:, t] = 1.0
    return lab, msk


def softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def bce_terms(llr, labels, valid):
    """Elementwise BCE with logits, softplus(l) - b*l, on valid entries (0 elsewhere)."""
    return (softplus(llr) - labels * llr) * valid


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def bce_grad(llr, labels, valid, n_total):
    return (sigmoid(llr) - labels) * valid / n_total


def mse_grad(hests, h_trues, gamma):
    """Channel-estimate loss of the double readout (Sec. II-B): MSE = mean over every complex entry of
    the batch (all slots, REs, UEs, antennas) of |ĥ - h|^2.  Returns MSE and, per slot, the gradient of
    gamma * MSE (real part w.r.t. Re ĥ, imaginary part w.r.t. Im ĥ: 2 gamma (ĥ - h) / N)."""
    n = sum(h.size for h in h_trues)
    err = [he - h for he, h in zip(hests, h_trues)]
    mse = sum(float(np.sum(np.abs(e) ** 2)) for e in err) / n
    return mse, [2.0 * gamma * e / n for e in err]


def adam_step(w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Kingma & Ba (2015), bias-corrected; step counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
