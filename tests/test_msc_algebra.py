"""The multispin sweep's bit-sliced Creutz move against the rule it encodes.

The multispin sweeps decide 64 sites per word with boolean algebra: the
one-sweep kernel with msc_move (csrc/msc_kernels.hpp), the two-sweep pass
with msc_move_fused (csrc/msc2_kernels.hpp), whose gates are fused further.
Their three-input gates are single gfx950 v_bitop3 instructions given by an
8-bit truth table.  This test restates that algebra on the CPU, emulating
v_bitop3 from its table, and checks it site by site against the move of
Sec. 2.3 with the 2-bit daemon of Sec. 2.5.  A site with u unsatisfied bonds has local energy 2u - 6, and
flipping it changes the energy by dH = 12 - 4u.  The daemon holds n = 4m,
m in 0..3, and the flip is accepted iff 0 <= n - dH <= 12, i.e. iff
3 <= m + u <= 6, leaving m' = m + u - 3.  The check covers every (m, u) and
every placement of the unsatisfied bonds among the six.
"""
import itertools

import pytest

MASK = (1 << 64) - 1


def bitop3(a, b, c, table, msb_first=True):
    """v_bitop3 on Python ints: bit i of the result is bit k of the table,
    k formed from bit i of the operands (first operand as the high bit of k,
    or, with msb_first=False, as the low bit)."""
    out = 0
    for i in range(64):
        x, y, z = (a >> i) & 1, (b >> i) & 1, (c >> i) & 1
        k = (x << 2 | y << 1 | z) if msb_first else (z << 2 | y << 1 | x)
        out |= ((table >> k) & 1) << i
    return out


def move(s, a, m0, m1, msb_first=True):
    """The kernel's move: a[0..5] already s ^ neighbour ^ coupling (the
    unsatisfied-bond bits); returns (new s, new m0, new m1, accepted)."""
    xor3 = lambda x, y, z: bitop3(x, y, z, 0x96, msb_first)
    maj3 = lambda x, y, z: bitop3(x, y, z, 0xE8, msb_first)
    s1, c1 = xor3(a[0], a[1], a[2]), maj3(a[0], a[1], a[2])
    s2, c2 = xor3(a[3], a[4], a[5]), maj3(a[3], a[4], a[5])
    u0, k0 = s1 ^ s2, s1 & s2
    u1, u2 = xor3(c1, c2, k0), maj3(c1, c2, k0)
    w0, cw0 = m0 ^ u0, m0 & u0
    w1, cw1 = xor3(m1, u1, cw0), maj3(m1, u1, cw0)
    w2, w3 = u2 ^ cw1, u2 & cw1
    acc = ~w3 & (w2 ^ (w1 & w0)) & MASK
    n0 = ((acc & ~w0) | (~acc & m0)) & MASK
    n1 = ((acc & (w2 & (w1 | w0))) | (~acc & m1)) & MASK
    return s ^ acc, n0, n1, acc


def cases():
    """One lane per (m, placement of unsatisfied bonds, spin): 4 x 64 x 2 =
    512 cases, packed 64 to a word."""
    all_cases = [(m, bits, sp) for m in range(4) for bits in range(64) for sp in (0, 1)]
    for start in range(0, len(all_cases), 64):
        yield all_cases[start:start + 64]


@pytest.mark.parametrize("msb_first", [True, False], ids=["table-msb-first", "table-lsb-first"])
def test_bit_sliced_move_matches_the_creutz_rule(msb_first):
    seen = set()
    for chunk in cases():
        s = m0 = m1 = 0
        a = [0] * 6
        for lane, (m, bits, sp) in enumerate(chunk):
            s |= sp << lane
            m0 |= (m & 1) << lane
            m1 |= (m >> 1) << lane
            for d in range(6):
                a[d] |= ((bits >> d) & 1) << lane
        ns, n0, n1, acc = move(s, a, m0, m1, msb_first)
        for lane, (m, bits, sp) in enumerate(chunk):
            u = bin(bits).count("1")
            dH = 12 - 4 * u
            ok = 0 <= 4 * m - dH <= 12
            got_acc = (acc >> lane) & 1
            got_m = ((n0 >> lane) & 1) | (((n1 >> lane) & 1) << 1)
            assert got_acc == int(ok), (m, u)
            assert ((ns >> lane) & 1) == sp ^ int(ok), (m, u)
            assert got_m == (m + u - 3 if ok else m), (m, u)
            # the energy tally adds 4 (m - m'), which is dH when accepted
            assert 4 * (m - got_m) == (dH if ok else 0), (m, u)
            seen.add((m, u))
    assert seen == {(m, u) for m in range(4) for u in range(7)}


def test_symmetric_truth_tables_do_not_depend_on_operand_order():
    for t, f in ((0x96, lambda x, y, z: x ^ y ^ z), (0xE8, lambda x, y, z: (x & y) | (z & (x | y)))):
        for x, y, z in itertools.product((0, 1), repeat=3):
            k_msb, k_lsb = x << 2 | y << 1 | z, z << 2 | y << 1 | x
            assert (t >> k_msb) & 1 == (t >> k_lsb) & 1 == f(x, y, z)


def move_fused(s, a, m0, m1, msb_first=True):
    """The two-sweep pass's form of the move (csrc/msc2_kernels.hpp,
    msc_move_fused): the same decision with the gates of each 32-bit half
    fused into three-input v_bitop3 tables, each symmetric in its first and
    third operands, and two-way selects (v_bfi)."""
    b3 = lambda x, y, z, t: bitop3(x, y, z, t, msb_first)
    xor3 = lambda x, y, z: b3(x, y, z, 0x96)
    maj3 = lambda x, y, z: b3(x, y, z, 0xE8)
    sel = lambda c, x, y: ((c & x) | (~c & y)) & MASK
    s1, c1 = xor3(a[0], a[1], a[2]), maj3(a[0], a[1], a[2])
    s2, c2 = xor3(a[3], a[4], a[5]), maj3(a[3], a[4], a[5])
    k0 = s1 & s2
    u1, u2 = xor3(c1, c2, k0), maj3(c1, c2, k0)
    x0 = b3(s1, m0, s2, 0x69)    # ~(m0 ^ s1 ^ s2)
    cw0 = b3(s1, m0, s2, 0x48)   # m0 & (s1 ^ s2)
    w1, cw1 = xor3(m1, u1, cw0), maj3(m1, u1, cw0)
    p = b3(w1, x0, w1, 0x30)     # w1 & ~x0
    r = b3(w1, x0, w1, 0xF3)     # w1 | ~x0
    acc = b3(u2, p, cw1, 0x16)   # ~(u2 & cw1) & (u2 ^ cw1 ^ p)
    v = b3(u2, r, cw1, 0x48)     # (u2 ^ cw1) & r
    return s ^ acc, sel(acc, x0, m0), sel(acc, v, m1), acc


@pytest.mark.parametrize("msb_first", [True, False], ids=["table-msb-first", "table-lsb-first"])
def test_fused_gate_move_equals_the_move(msb_first):
    """Every (level, placement of unsatisfied bonds, spin): the fused form
    gives the same new spin, levels and acceptance as the move above, under
    either operand order of the truth tables."""
    for chunk in cases():
        s = m0 = m1 = 0
        a = [0] * 6
        for lane, (m, bits, sp) in enumerate(chunk):
            s |= sp << lane
            m0 |= (m & 1) << lane
            m1 |= (m >> 1) << lane
            for d in range(6):
                a[d] |= ((bits >> d) & 1) << lane
        assert move_fused(s, a, m0, m1, msb_first) == move(s, a, m0, m1, True)
