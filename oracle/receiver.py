"""Classical receiver front and judge (oracle side): LS + linear interpolation, LMMSE, max-log.

TEST INFRASTRUCTURE ONLY (oracle).

The paper's NRX takes, per UE stream, an initial LS channel estimate from the
DMRS (Sec. II-A, architecture description), and its classical baseline is LS
channel estimation with interpolation followed by LMMSE equalisation and
demapping (Sec. III-B comparison).  LLRs are logits, positive meaning bit 1,
Eq. (2).  Readings: despreading assumes equal channel on the two REs of an OCC
pair; interpolation is linear with flat extrapolation, in frequency between pair
centres and in time between the two DMRS symbols.
"""
import numpy as np

from . import nr


def ls_estimate(y, desc):
    """Ĥ[s, t, u, b] from y[s, t, b] for the desc.n_ue ports."""
    S, B, U = desc.n_sc, desc.n_ant, desc.n_ue
    out = np.zeros((S, nr.N_SYMB, U, B), dtype=np.complex128)
    n_pairs = S // 4
    for u in range(U):
        delta = nr.cdm_group(u)
        pos = 4 * np.arange(n_pairs) + 1 + delta
        est = {}
        for l in nr.DMRS_SYMBOLS:
            r = nr.dmrs_sequence(desc.slot_number, l, S // 2, desc.n_id, desc.n_scid)
            hp = np.zeros((n_pairs, B), dtype=np.complex128)
            for n in range(n_pairs):
                for kp in range(2):
                    k = 4 * n + 2 * kp + delta
                    pilot = nr.w_f(u, kp) * r[2 * n + kp]
                    hp[n] += 0.5 * y[k, l, :] * np.conj(pilot)
            full = np.zeros((S, B), dtype=np.complex128)
            for b in range(B):
                full[:, b] = (np.interp(np.arange(S), pos, hp[:, b].real)
                              + 1j * np.interp(np.arange(S), pos, hp[:, b].imag))
            est[l] = full
        l0, l1 = nr.DMRS_SYMBOLS
        for t in range(nr.N_SYMB):
            if t <= l0:
                out[:, t, u, :] = est[l0]
            elif t >= l1:
                out[:, t, u, :] = est[l1]
            else:
                out[:, t, u, :] = ((l1 - t) * est[l0] + (t - l0) * est[l1]) / (l1 - l0)
    return out


def lmmse_equalise(y, h, n0):
    """Per RE: G = H^H H + N0 I, z~ = G^-1 H^H y, d = 1 - N0 diag(G^-1), z = z~/d, var = (1-d)/d.
    y [..., B], h [..., U, B] -> z [..., U], var [..., U]."""
    hm = np.swapaxes(h, -1, -2)                       # [..., B, U]
    hh = np.conj(np.swapaxes(hm, -1, -2))             # [..., U, B]
    U = hm.shape[-1]
    G = hh @ hm + n0 * np.eye(U)
    Ginv = np.linalg.inv(G)
    zt = (Ginv @ (hh @ y[..., None]))[..., 0]
    d = 1.0 - n0 * np.real(np.diagonal(Ginv, axis1=-2, axis2=-1))
    z = zt / d
    var = np.maximum((1.0 - d) / d, 1e-12)
    return z, var


def maxlog_llr(z, var, m):
    """l_j = (min_{c: b_j=0} |z-c|^2 - min_{c: b_j=1} |z-c|^2) / var  (logit sign of Eq. (2))."""
    pts, lab = nr.constellation(m)
    dist = np.abs(z[..., None] - pts) ** 2            # [..., 2^m]
    out = np.zeros(z.shape + (m,))
    for j in range(m):
        d0 = np.where(lab[:, j] == 0, dist, np.inf).min(axis=-1)
        d1 = np.where(lab[:, j] == 1, dist, np.inf).min(axis=-1)
        out[..., j] = (d0 - d1) / var
    return out


def lmmse_demap(y, h, n0, desc, m_max):
    """LLRs in the [u][t][s][j] layout; DMRS symbols and j >= m_u are zero."""
    S, U = desc.n_sc, desc.n_ue
    llr = np.zeros((U, nr.N_SYMB, S, m_max))
    z, var = lmmse_equalise(y, h, n0)                 # [S, T, U]
    for u in range(U):
        m = desc.bits_per_sym[u]
        l = maxlog_llr(z[:, :, u], var[:, :, u], m)   # [S, T, m]
        for t in nr.data_symbols():
            llr[u, t, :, :m] = l[:, t, :]
    return llr
