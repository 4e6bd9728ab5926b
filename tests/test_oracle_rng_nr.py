"""Pins of the oracle's Philox generator and 5G NR building blocks (no GPU)."""
import os

import numpy as np
import pytest

from oracle import nr, philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt")) if not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(np.array(v[0:4]), v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_uniform_open_interval_exact():
    w = np.array([0, 1, 511, 512, 0xFFFFFFFF], dtype=np.uint64)
    u = philox.uniform(w)
    assert u[0] == 2.0 ** -24 and u[-1] == 1 - 2.0 ** -24
    assert np.all((u > 0) & (u < 1))
    assert np.all(u.astype(np.float32).astype(np.float64) == u)   # exact in fp32


# ---- Gold sequence: pinned by linear-recurrence theory, not by re-running the LFSR ----

def _polymulmod(a, b, p, deg):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> deg & 1:
            a ^= p
    return r


def _xpow(n, p, deg):
    """x^n mod p over GF(2), p including its x^deg term."""
    result, base = 1, 2
    while n:
        if n & 1:
            result = _polymulmod(result, base, p, deg)
        base = _polymulmod(base, base, p, deg)
        n >>= 1
    return result


P1 = (1 << 31) | (1 << 3) | 1                         # x^31 + x^3 + 1
P2 = (1 << 31) | (1 << 3) | (1 << 2) | (1 << 1) | 1   # x^31 + x^3 + x^2 + x + 1


@pytest.mark.parametrize("p", [P1, P2])
def test_gold_polynomials_primitive(p):
    # 2^31-1 is prime, so x has order 2^31-1 (maximal period) iff x^(2^31-1) = 1 and x != 1.
    assert _xpow(2 ** 31 - 1, p, 31) == 1
    assert _xpow(1, p, 31) != 1


def _jump(init_bits, p, n):
    """a(n) of the recurrence with characteristic polynomial p from a(0..30), via x^n mod p."""
    c = _xpow(n, p, 31)
    return sum(((c >> i) & 1) * init_bits[i] for i in range(31)) % 2


@pytest.mark.parametrize("c_init", [0, 1, 0x1234567, nr.dmrs_c_init(7, 11, 0, 0), 2 ** 31 - 1])
def test_gold_sequence_by_polynomial_jump(c_init):
    c = nr.gold_sequence(c_init, 64)
    x1_init = [1] + [0] * 30
    x2_init = [(c_init >> i) & 1 for i in range(31)]
    for n in [0, 1, 2, 5, 31, 63]:
        expect = (_jump(x1_init, P1, n + nr.NC) + _jump(x2_init, P2, n + nr.NC)) % 2
        assert c[n] == expect


def _berlekamp_massey(s):
    n = len(s)
    c, b = [1] + [0] * n, [1] + [0] * n
    L, m = 0, 1
    for i in range(n):
        d = s[i]
        for j in range(1, L + 1):
            d ^= c[j] & s[i - j]
        if d == 0:
            m += 1
        elif 2 * L <= i:
            t = c[:]
            for j in range(n + 1 - m):
                c[j + m] ^= b[j]
            L, b, m = i + 1 - L, t, 1
        else:
            for j in range(n + 1 - m):
                c[j + m] ^= b[j]
            m += 1
    return L, c[:L + 1]


def test_gold_linear_complexity():
    # c = x1 + x2 has linear complexity 62 with connection polynomial p1*p2 (reciprocal form).
    c = [int(v) for v in nr.gold_sequence(0x5A5A5A5, 200)]
    L, conn = _berlekamp_massey(c)
    assert L == 62
    prod = 0
    for i in range(32):
        if P1 >> i & 1:
            prod ^= P2 << i
    recip = [(prod >> (62 - j)) & 1 for j in range(63)]
    assert conn == recip


def test_gold_cinit_zero_is_pure_x1():
    c = nr.gold_sequence(0, 40)
    x1_init = [1] + [0] * 30
    assert all(c[n] == _jump(x1_init, P1, n + nr.NC) for n in range(40))


def test_dmrs_values_and_occ():
    r = nr.dmrs_sequence(3, 2, 100)
    assert np.allclose(np.abs(r), 1.0)
    assert set(np.round(r.real * np.sqrt(2)).astype(int)) <= {-1, 1}
    S = 48
    for port in range(4):
        g = nr.dmrs_grid(port, S, 3, 2)
        nz = np.nonzero(g)[0]
        assert np.all(nz % 2 == nr.cdm_group(port)) and len(nz) == S // 2
    # ports sharing a CDM group are orthogonal over each OCC pair
    g0, g1 = nr.dmrs_grid(0, S, 3, 2), nr.dmrs_grid(1, S, 3, 2)
    pair = (g0 * np.conj(g1)).reshape(-1, 4).sum(axis=1)
    assert np.allclose(pair, 0)


# ---- Gray QAM ----

@pytest.mark.parametrize("m,norm", [(2, 2), (4, 10), (6, 42), (8, 170)])
def test_qam_energy_and_levels(m, norm):
    pts, _ = nr.constellation(m)
    assert np.isclose(np.mean(np.abs(pts) ** 2), 1.0)
    lv = np.unique(np.round(pts.real * np.sqrt(norm)).astype(int))
    assert list(lv) == list(range(-(2 ** (m // 2) - 1), 2 ** (m // 2), 2))


@pytest.mark.parametrize("m", [2, 4, 6, 8])
def test_qam_gray_neighbours(m):
    pts, bits = nr.constellation(m)
    dmin = np.min(np.abs(pts[:, None] - pts[None, :]) + 10 * np.eye(len(pts)))
    for i in range(len(pts)):
        for k in range(len(pts)):
            if i != k and np.isclose(abs(pts[i] - pts[k]), dmin):
                assert np.sum(bits[i] != bits[k]) == 1


@pytest.mark.parametrize("m", [4, 6, 8])
def test_qam_recursive_labels(m):
    # The first two bits of a higher-order Gray QAM point are the QPSK label of its quadrant.
    pts, bits = nr.constellation(m)
    q = nr.qam_map(bits[:, :2], 2)
    assert np.all(np.sign(q.real) == np.sign(pts.real))
    assert np.all(np.sign(q.imag) == np.sign(pts.imag))


def test_qpsk_example_point():
    # b = (0, 0) -> (1 + j)/sqrt(2); b = (1, 0) -> (-1 + j)/sqrt(2)
    assert np.isclose(nr.qam_map(np.array([0, 0]), 2), (1 + 1j) / np.sqrt(2))
    assert np.isclose(nr.qam_map(np.array([1, 0]), 2), (-1 + 1j) / np.sqrt(2))
    # 16-QAM b = (0,0,0,0) -> (1 + j)/sqrt(10)
    assert np.isclose(nr.qam_map(np.array([0, 0, 0, 0]), 4), (1 + 1j) / np.sqrt(10))


def test_re_order():
    assert nr.data_symbols() == [0, 1, 3, 4, 5, 6, 7, 8, 9, 10, 12, 13]
    assert nr.data_re_index(5, 3, 48) == 2 * 48 + 5
