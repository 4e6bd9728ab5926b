"""Synthetic PUSCH slot generator (oracle side): the MU-MIMO OFDM model of Eq. (1).

TEST INFRASTRUCTURE ONLY (oracle).

Eq. (1): on every RE (s, t), y = sum_u H_{s,t,u} x_{s,t,u} + n with n ~ CN(0, N0 I),
valid when the cyclic prefix covers the channel (so the channel is a per-RE gain;
no inter-carrier interference).  Each UE sends one stream from one antenna
(Sec. II: one MIMO layer per UE).  The paper's channels (3GPP UMi, TDL, ray-traced)
are not reproducible here; the stand-in is a tapped-delay Rayleigh channel:

  H[s,t,u,b] = sum_l sqrt(p_l) * sum_{b'} Lc[b,b'] g_{l,b',u}(t) * exp(-j 2 pi s df tau_l)
  tau_l = l * spacing,  p_l ~ exp(-tau_l / decay) normalised to sum 1,
  g(t) = M^-1/2 sum_n exp(j(2 pi fD cos(alpha_n) t Tsym + phi_n)), alpha_n = 2 pi (n+theta)/M,
  Lc = lower Cholesky factor of R_ij = rho^|i-j| (exponential BS-array correlation).

All random quantities come from Philox4x32-10 with the counter layout below, so
the GPU generator (written separately) can draw the very same numbers:
  counter = (batch_index, slot, stream, element)
  bits    : stream 1, element (u << 16) | data_re, bit j = (word0 >> j) & 1
  channel : stream 2, element ((u*B + b')*L + l)*8 + k, k = 0..4 -> 20 words:
            word 0 -> theta, words 1..16 -> phi_n / (2 pi)
  noise   : stream 3, element (s*14 + t)*B + b, words 0,1 -> Box-Muller
  slot    : stream 4, element 0 word 0 -> SNR draw; element 1+u word 0 -> Doppler draw
"""
import numpy as np

from . import nr
from .philox import draw, uniform, STREAM_BITS, STREAM_CHANNEL, STREAM_NOISE, STREAM_SLOT

N_SIN = 16
T_SYM = 2192.0 / (2048.0 * 30e3)   # OFDM symbol + normal CP at 30 kHz SCS


class SimConfig:
    def __init__(self, n_taps=12, tap_spacing_ns=100, tap_decay_ns=487.42, doppler_max_hz=0.0,
                 rho=0.0, snr_db_lo=10.0, snr_db_hi=10.0, scs_khz=30):
        self.n_taps = n_taps
        self.tap_spacing_ns = tap_spacing_ns
        self.tap_decay_ns = tap_decay_ns
        self.doppler_max_hz = doppler_max_hz
        self.rho = rho
        self.snr_db_lo = snr_db_lo
        self.snr_db_hi = snr_db_hi
        self.scs_khz = scs_khz


class SlotDesc:
    def __init__(self, n_prb, n_ant, n_ue, bits_per_sym, slot_number=0, n_id=0, n_scid=0, snr_offset_db=0.0):
        self.n_prb = n_prb
        self.n_ant = n_ant
        self.n_ue = n_ue
        self.bits_per_sym = list(bits_per_sym)[:n_ue]
        self.slot_number = slot_number
        self.n_id = n_id
        self.n_scid = n_scid
        self.snr_offset_db = snr_offset_db   # added to the drawn SNR (mixed-MCS training offsets, Sec. III-A)

    @property
    def n_sc(self):
        return 12 * self.n_prb


def pdp(cfg):
    tau = np.arange(cfg.n_taps) * cfg.tap_spacing_ns * 1e-9
    p = np.exp(-tau / (cfg.tap_decay_ns * 1e-9))
    return tau, p / p.sum()


def spatial_factor(n_ant, rho):
    r = rho ** np.abs(np.arange(n_ant)[:, None] - np.arange(n_ant)[None, :])
    return np.linalg.cholesky(r)


def slot_params(seed, batch_index, slot, cfg, n_ue):
    w = draw(seed, batch_index, slot, STREAM_SLOT, np.arange(1 + n_ue))[:, 0]
    u = uniform(w)
    snr_db = cfg.snr_db_lo + (cfg.snr_db_hi - cfg.snr_db_lo) * u[0]
    fd = cfg.doppler_max_hz * u[1:]
    return snr_db, fd


def channel(seed, batch_index, slot, cfg, desc):
    """True channel H[s, t, u, b] (complex128) and per-UE Doppler."""
    S, B, U, L = desc.n_sc, desc.n_ant, desc.n_ue, cfg.n_taps
    _, fd = slot_params(seed, batch_index, slot, cfg, U)
    tau, p = pdp(cfg)
    lc = spatial_factor(B, cfg.rho)
    t = np.arange(nr.N_SYMB)
    H = np.zeros((S, nr.N_SYMB, U, B), dtype=np.complex128)
    s = np.arange(S)
    for u in range(U):
        g = np.zeros((L, B, nr.N_SYMB), dtype=np.complex128)
        for bp in range(B):
            for l in range(L):
                base = ((u * B + bp) * L + l) * 8
                words = draw(seed, batch_index, slot, STREAM_CHANNEL, base + np.arange(5)).reshape(-1)
                un = uniform(words)
                theta = un[0]
                phi = 2 * np.pi * un[1:1 + N_SIN]
                alpha = 2 * np.pi * (np.arange(N_SIN) + theta) / N_SIN
                ph = (2 * np.pi * fd[u] * np.cos(alpha)[None, :] * (t[:, None] * T_SYM)
                      + phi[None, :])
                g[l, bp] = np.exp(1j * ph).sum(axis=1) / np.sqrt(N_SIN)
        h = np.sqrt(p)[:, None, None] * np.einsum('bc,lct->lbt', lc, g)     # [L, B, T]
        steer = np.exp(-2j * np.pi * s[:, None] * cfg.scs_khz * 1e3 * tau[None, :])  # [S, L]
        H[:, :, u, :] = np.einsum('sl,lbt->stb', steer, h)
    return H


def bits(seed, batch_index, slot, desc, m_max):
    n_data = desc.n_sc * len(nr.data_symbols())
    out = np.zeros((desc.n_ue, n_data, m_max), dtype=np.uint8)
    e = np.arange(n_data, dtype=np.uint64)
    for u in range(desc.n_ue):
        w0 = draw(seed, batch_index, slot, STREAM_BITS, (np.uint64(u) << np.uint64(16)) | e)[:, 0]
        for j in range(desc.bits_per_sym[u]):
            out[u, :, j] = (w0 >> np.uint32(j)) & 1
    return out


def transmit_grid(desc, bitarr):
    """x[s, t, u]: Gray QAM on data REs (frequency-first order), DMRS on symbols 2 and 11."""
    S = desc.n_sc
    x = np.zeros((S, nr.N_SYMB, desc.n_ue), dtype=np.complex128)
    dsym = nr.data_symbols()
    for u in range(desc.n_ue):
        m = desc.bits_per_sym[u]
        sym = nr.qam_map(bitarr[u, :, :m], m)
        for k, t in enumerate(dsym):
            x[:, t, u] = sym[k * S:(k + 1) * S]
        for l in nr.DMRS_SYMBOLS:
            x[:, l, u] = nr.dmrs_grid(u, S, desc.slot_number, l, desc.n_id, desc.n_scid)
    return x


def noise(seed, batch_index, slot, desc, n0):
    S, B = desc.n_sc, desc.n_ant
    el = np.arange(S * nr.N_SYMB * B, dtype=np.uint64)
    w = draw(seed, batch_index, slot, STREAM_NOISE, el)
    u0 = uniform(w[:, 0])
    u1 = uniform(w[:, 1])
    r = np.sqrt(-2.0 * np.log(u0))
    n = r * np.cos(2 * np.pi * u1) + 1j * r * np.sin(2 * np.pi * u1)
    return (np.sqrt(n0 / 2.0) * n).reshape(S, nr.N_SYMB, B)


def simulate_slot(seed, batch_index, slot, cfg, desc, m_max):
    """Returns dict with y [S,T,B], h [S,T,U,B], bits [U,n_data,m_max], snr_db, n0."""
    snr_db, _ = slot_params(seed, batch_index, slot, cfg, desc.n_ue)
    snr_db += desc.snr_offset_db
    n0 = 10.0 ** (-snr_db / 10.0)
    H = channel(seed, batch_index, slot, cfg, desc)
    b = bits(seed, batch_index, slot, desc, m_max)
    x = transmit_grid(desc, b)
    y = np.einsum('stub,stu->stb', H, x) + noise(seed, batch_index, slot, desc, n0)
    return dict(y=y, h=H, bits=b, snr_db=snr_db, n0=n0, x=x)
