"""Pins of the oracle's corner turn (F-engine packets -> X-stage input order),
against the packet order written out sample by sample and the 4-bit
two's-complement definition (Sec. 2.3, Sec. 2.4 and its packet-format figure)."""
import numpy as np

import oracle


def packetize_loops(x, F, J, S):
    """Packets built one sample at a time from an X-stage array x[c][t][i]:
    packet (b, f) carries, for each of its S spectra, every channel's J
    inputs of F-engine f, the spectra one after another."""
    C, T, N = x.shape
    B = T // S
    out = np.zeros((B, F, S, C, J), dtype=np.uint8)
    for b in range(B):
        for f in range(F):
            for s in range(S):
                for c in range(C):
                    for j in range(J):
                        out[b, f, s, c, j] = x[c, b * S + s, f * J + j]
    return out


def test_corner_turn_inverts_the_packet_order():
    rng = np.random.default_rng(3)
    F, J, C, S, B = 3, 4, 5, 2, 4
    x = rng.integers(0, 256, size=(C, B * S, F * J), dtype=np.uint8)
    p = packetize_loops(x, F, J, S)
    np.testing.assert_array_equal(oracle.corner_turn(p, F, J, C, S), x)


def test_lost_packets_give_zeros_and_nothing_else_changes():
    rng = np.random.default_rng(4)
    F, J, C, S, B = 4, 8, 3, 3, 5
    x = rng.integers(0, 256, size=(C, B * S, F * J), dtype=np.uint8)
    p = packetize_loops(x, F, J, S)
    valid = np.ones((B, F), dtype=np.uint8)
    valid[1, 2] = 0
    valid[4, 0] = 0
    y = oracle.corner_turn(p, F, J, C, S, valid=valid)
    expect = x.copy()
    for (b, f) in [(1, 2), (4, 0)]:
        expect[:, b * S:(b + 1) * S, f * J:(f + 1) * J] = 0
    np.testing.assert_array_equal(y, expect)


def nibble(v):
    return v - 16 if v >= 8 else v


def test_unpack_every_byte():
    # all 256 byte values: high nibble -> real, low nibble -> imaginary,
    # each a 4-bit two's-complement integer
    x = np.arange(256, dtype=np.uint8).reshape(1, 1, 256)    # C=1, T=1, N=256 (F=16, J=16, S=1)
    p = packetize_loops(x, 16, 16, 1)
    y = oracle.corner_turn(p, 16, 16, 1, 1, out_fmt="ci8")
    assert y.shape == (1, 1, 256, 2) and y.dtype == np.int8
    for v in range(256):
        assert (int(y[0, 0, v, 0]), int(y[0, 0, v, 1])) == (nibble(v >> 4), nibble(v & 15)), v


def test_unpacked_visibilities_match_the_packed_ones():
    # the X-stage result does not depend on whether the 4-bit samples were
    # promoted to 8 bits first
    rng = np.random.default_rng(5)
    F, J, C, S, B = 2, 8, 2, 4, 8
    x = rng.integers(0, 256, size=(C, B * S, F * J), dtype=np.uint8)
    p = packetize_loops(x, F, J, S)
    v4 = oracle.correlate(oracle.corner_turn(p, F, J, C, S), "ci4")
    v8 = oracle.correlate(oracle.corner_turn(p, F, J, C, S, out_fmt="ci8"), "ci8")
    np.testing.assert_array_equal(v4, v8)
