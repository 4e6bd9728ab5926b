"""5G NR pieces the receiver depends on: Gold sequence, PUSCH DMRS, Gray QAM, RG order.

TEST INFRASTRUCTURE ONLY (oracle).  Plain fp64 / integer code, no blocking.

Paper basis: the pilots are mapping-type-A DMRS with one additional DMRS symbol
(Sec. III-B, simulation setup), known to the BS (Sec. II); constellations are Gray-labelled
QAM per the 5G NR MCS table (Sec. II), whose recursive labelling is what LLR
masking relies on (Sec. III).  The sequence, mapping and modulation formulas are
those of 3GPP TS 38.211 (Sec. 5.2.1 Gold sequence, 5.1 modulation, 6.4.1.1 PUSCH
DMRS type 1), restated below.  Readings (port map, N_ID, slot numbering) are
listed in the design notes.
"""
import numpy as np

NC = 1600
N_SYMB = 14
DMRS_SYMBOLS = (2, 11)   # type A, l0 = 2, one additional position, 14-symbol slot


def gold_sequence(c_init, length):
    """Bit-serial Gold sequence c(0..length-1) (TS 38.211 Sec. 5.2.1)."""
    n = NC + length + 31
    x1 = [0] * n
    x2 = [0] * n
    x1[0] = 1
    for i in range(31):
        x2[i] = (int(c_init) >> i) & 1
    for i in range(n - 31):
        x1[i + 31] = (x1[i + 3] + x1[i]) % 2
        x2[i + 31] = (x2[i + 3] + x2[i + 2] + x2[i + 1] + x2[i]) % 2
    return np.array([(x1[i + NC] + x2[i + NC]) % 2 for i in range(length)], dtype=np.uint8)


def dmrs_c_init(slot_number, symbol, n_id=0, n_scid=0):
    """PUSCH DMRS scrambling init, transform precoding disabled (TS 38.211 Sec. 6.4.1.1.1.1)."""
    return (2 ** 17 * (N_SYMB * slot_number + symbol + 1) * (2 * n_id + 1)
            + 2 * n_id + n_scid) % 2 ** 31


def dmrs_sequence(slot_number, symbol, length, n_id=0, n_scid=0):
    """r(n) = ((1-2c(2n)) + j(1-2c(2n+1)))/sqrt(2), n < length."""
    c = gold_sequence(dmrs_c_init(slot_number, symbol, n_id, n_scid), 2 * length).astype(np.float64)
    return ((1 - 2 * c[0::2]) + 1j * (1 - 2 * c[1::2])) / np.sqrt(2.0)


def cdm_group(port):
    """DMRS configuration type 1: ports 0,1 -> CDM group 0 (Delta=0); ports 2,3 -> group 1 (Delta=1)."""
    return port // 2


def w_f(port, kprime):
    """Frequency OCC of type-1 DMRS: +1,+1 for even ports, +1,-1 for odd ports."""
    return -1.0 if (port % 2 == 1 and kprime == 1) else 1.0


def dmrs_grid(port, n_sc, slot_number, symbol, n_id=0, n_scid=0):
    """Complex DMRS values of one port on one DMRS symbol, zero on the other CDM group's REs.
    a_k = w_f(k') r(2n+k') at k = 4n + 2k' + Delta (TS 38.211 Sec. 6.4.1.1.3), beta = 1."""
    delta = cdm_group(port)
    r = dmrs_sequence(slot_number, symbol, n_sc // 2, n_id, n_scid)
    a = np.zeros(n_sc, dtype=np.complex128)
    for n in range(n_sc // 4):
        for kp in range(2):
            k = 4 * n + 2 * kp + delta
            a[k] = w_f(port, kp) * r[2 * n + kp]
    return a


# ----------------------------------------------------------------- Gray QAM ---

def qam_map(bits, m):
    """bits: (..., m) of 0/1 -> complex symbols (TS 38.211 Sec. 5.1.3-5.1.7)."""
    b = np.asarray(bits, dtype=np.float64)
    if m == 2:
        re = (1 - 2 * b[..., 0])
        im = (1 - 2 * b[..., 1])
        return (re + 1j * im) / np.sqrt(2.0)
    if m == 4:
        re = (1 - 2 * b[..., 0]) * (2 - (1 - 2 * b[..., 2]))
        im = (1 - 2 * b[..., 1]) * (2 - (1 - 2 * b[..., 3]))
        return (re + 1j * im) / np.sqrt(10.0)
    if m == 6:
        re = (1 - 2 * b[..., 0]) * (4 - (1 - 2 * b[..., 2]) * (2 - (1 - 2 * b[..., 4])))
        im = (1 - 2 * b[..., 1]) * (4 - (1 - 2 * b[..., 3]) * (2 - (1 - 2 * b[..., 5])))
        return (re + 1j * im) / np.sqrt(42.0)
    if m == 8:
        re = (1 - 2 * b[..., 0]) * (8 - (1 - 2 * b[..., 2]) * (4 - (1 - 2 * b[..., 4]) * (2 - (1 - 2 * b[..., 6]))))
        im = (1 - 2 * b[..., 1]) * (8 - (1 - 2 * b[..., 3]) * (4 - (1 - 2 * b[..., 5]) * (2 - (1 - 2 * b[..., 7]))))
        return (re + 1j * im) / np.sqrt(170.0)
    raise ValueError("m must be 2, 4, 6 or 8")


def constellation(m):
    """All 2^m points with their labels; label integer i has bit j = (i >> j) & 1."""
    labels = np.arange(2 ** m)
    bits = (labels[:, None] >> np.arange(m)[None, :]) & 1
    return qam_map(bits, m), bits


def data_symbols(n_symb=N_SYMB):
    return [t for t in range(n_symb) if t not in DMRS_SYMBOLS]


def data_re_index(s, t, n_sc):
    """Position of RE (s, t) in the frequency-first, then time, data-RE order (TS 38.211 Sec. 6.3.1.6)."""
    return data_symbols().index(t) * n_sc + s
