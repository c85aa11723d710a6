"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle (oracle/) is the plain definition of the X-stage: for every channel
V_ij = sum_t x_i conj(x_j), i >= j (Sec. 1, Sec. 2.4).  Each test below checks
it against something other than itself:

  * exhaustive 4-bit domain with Python complex arithmetic on values built by
    the encoder (pins nibble order, sign extension and the conjugate side);
  * pure-Python complex loops and exact int64 numpy matrix products;
  * invariants of a sum of outer products (Hermitian, positive autos,
    Cauchy-Schwarz, additivity in time, conjugation, phase rotation);
  * the closed-form visibility of a common tone with per-antenna delays;
  * the beam-power identity w^H V w = sum_t |w^H x_t|^2;
  * closed forms for constant worst-case inputs past the int32 range.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1401_8288_amd import synth


def np_(t):
    return t.cpu().numpy()


# ------------------------------------------------------------ exhaustive / brute

def test_exhaustive_ci4_pairs():
    # all 16^4 (re0, im0, re1, im1) combinations, 2 inputs, 1 sample: V =
    # (x0 conj x0, x1 conj x0, x1 conj x1)
    vals = list(itertools.product(range(-8, 8), repeat=4))
    a = torch.tensor(vals, dtype=torch.int32)             # [65536][4]
    re = torch.stack([a[:, 0], a[:, 2]], 1)[:, None, :]  # [C][1][2]
    im = torch.stack([a[:, 1], a[:, 3]], 1)[:, None, :]
    x = np_(synth.pack_ci4(re, im))
    v = oracle.correlate(x, "ci4")
    assert v.shape == (65536, 3, 2)
    exp = np.empty_like(v)
    for k, (r0, i0, r1, i1) in enumerate(vals):
        x0, x1 = complex(r0, i0), complex(r1, i1)
        for b, z in enumerate((x0 * x0.conjugate(), x1 * x0.conjugate(), x1 * x1.conjugate())):
            exp[k, b] = (int(z.real), int(z.imag))
    np.testing.assert_array_equal(v, exp)


def test_ci8_corner_values():
    corner = [-128, -127, -1, 0, 1, 127]
    vals = list(itertools.product(corner, repeat=4))
    a = torch.tensor(vals, dtype=torch.int32)
    re = torch.stack([a[:, 0], a[:, 2]], 1)[:, None, :]
    im = torch.stack([a[:, 1], a[:, 3]], 1)[:, None, :]
    x = np_(synth.pack_ci8(re, im))
    v = oracle.correlate(x, "ci8")
    for k, (r0, i0, r1, i1) in enumerate(vals):
        x0, x1 = complex(r0, i0), complex(r1, i1)
        for b, z in enumerate((x0 * x0.conjugate(), x1 * x0.conjugate(), x1 * x1.conjugate())):
            assert tuple(v[k, b]) == (int(z.real), int(z.imag))


def test_ci8_random_pairs():
    g = np.random.default_rng(11)
    n = 200_000
    comp = g.integers(-128, 128, size=(n, 4))
    re = torch.tensor(comp[:, [0, 2]])[:, None, :]
    im = torch.tensor(comp[:, [1, 3]])[:, None, :]
    x = np_(synth.pack_ci8(re, im))
    v = oracle.correlate(x, "ci8")
    r0, i0, r1, i1 = (comp[:, k].astype(np.int64) for k in range(4))
    np.testing.assert_array_equal(v[:, 0, 0], r0 * r0 + i0 * i0)
    np.testing.assert_array_equal(v[:, 0, 1], 0)
    # x1 conj(x0) = (r1 r0 + i1 i0) + i (i1 r0 - r1 i0)
    np.testing.assert_array_equal(v[:, 1, 0], r1 * r0 + i1 * i0)
    np.testing.assert_array_equal(v[:, 1, 1], i1 * r0 - r1 * i0)
    np.testing.assert_array_equal(v[:, 2, 0], r1 * r1 + i1 * i1)


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 16, 5), (3, 7, 8), (1, 13, 3)])
def test_brute_force_tiny(fmt, shape):
    c, t, n = shape
    x = np_(synth.random_input(c, t, n, fmt, seed=sum(shape) + len(fmt),
                               lo=-8 if fmt == "ci4" else -128))
    v = oracle.correlate(x, fmt)
    bf = oracle.brute_force(x, fmt)
    np.testing.assert_array_equal(v, np.array(bf, dtype=np.int64).reshape(v.shape))


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_matmul_form(fmt):
    x = np_(synth.random_input(3, 100, 37, fmt, seed=5))
    np.testing.assert_array_equal(oracle.correlate(x, fmt), oracle.matmul_form(x, fmt))


def test_channel_range_matches_full_run():
    x = np_(synth.random_input(6, 40, 20, "ci4", seed=6))
    full = oracle.correlate(x, "ci4")
    np.testing.assert_array_equal(oracle.correlate(x, "ci4", channels=(2, 3)), full[2:5])


def test_delta_input_gives_single_entry():
    # one nonzero sample on input 5 only -> only the autocorrelation (5,5)
    re = torch.zeros(1, 9, 8, dtype=torch.int32)
    im = torch.zeros(1, 9, 8, dtype=torch.int32)
    re[0, 4, 5], im[0, 4, 5] = 3, -2
    v = oracle.correlate(np_(synth.pack_ci4(re, im)), "ci4")
    nz = np.argwhere(v[0] != 0)
    assert [tuple(r) for r in nz] == [(5 * 6 // 2 + 5, 0)]
    assert v[0, 5 * 6 // 2 + 5, 0] == 13
    # two inputs -> cross term x7 conj(x2) at tri(7, 2)
    re[0, 4, 5], im[0, 4, 5] = 0, 0
    re[0, 1, 7], im[0, 1, 7] = 1, 2
    re[0, 1, 2], im[0, 1, 2] = 3, -1
    v = oracle.correlate(np_(synth.pack_ci4(re, im)), "ci4")
    z = complex(1, 2) * complex(3, -1).conjugate()
    assert tuple(v[0, 7 * 8 // 2 + 2]) == (int(z.real), int(z.imag))


# ------------------------------------------------------------------ invariants

def _full(v, n):
    """Packed triangle -> full Hermitian complex matrix per channel."""
    i, j = oracle.tri_index(n)
    m = np.zeros((v.shape[0], n, n), dtype=np.complex128)
    z = v[..., 0] + 1j * v[..., 1]
    m[:, i, j] = z
    m[:, j, i] = np.conj(z)
    return m


def test_autocorrelations_real_nonnegative():
    x = np_(synth.random_input(4, 64, 24, "ci4", seed=7))
    v = oracle.correlate(x, "ci4")
    i, j = oracle.tri_index(24)
    auto = v[:, i == j]
    assert (auto[..., 1] == 0).all()
    assert (auto[..., 0] >= 0).all()


def test_cauchy_schwarz():
    x = np_(synth.random_input(4, 64, 24, "ci8", seed=8))
    v = oracle.correlate(x, "ci8")
    i, j = oracle.tri_index(24)
    k = np.arange(24)
    d = k * (k + 1) // 2 + k                    # tri(k, k)
    vii = v[:, d, 0][:, i].astype(object)
    vjj = v[:, d, 0][:, j].astype(object)
    mag2 = v[..., 0].astype(object) ** 2 + v[..., 1].astype(object) ** 2
    assert (mag2 <= vii * vjj).all()


def test_input_reversal_gives_conjugate_transpose():
    n = 19
    x = np_(synth.random_input(2, 33, n, "ci4", seed=9))
    a = _full(oracle.correlate(x, "ci4"), n)
    b = _full(oracle.correlate(np.ascontiguousarray(x[:, :, ::-1]), "ci4"), n)
    # reversed order: V'[p][q] = V[n-1-p][n-1-q]
    np.testing.assert_array_equal(b, a[:, ::-1, ::-1])
    # and the full matrix is Hermitian by construction of the triangle
    np.testing.assert_array_equal(a, np.conj(np.swapaxes(a, 1, 2)))


def test_time_additivity():
    x = np_(synth.random_input(3, 90, 16, "ci4", seed=10))
    whole = oracle.correlate(x, "ci4")
    parts = sum(oracle.correlate(np.ascontiguousarray(x[:, s]), "ci4")
                for s in (slice(0, 1), slice(1, 40), slice(40, 90)))
    np.testing.assert_array_equal(whole, parts)


def test_conjugating_inputs_conjugates_v():
    g = torch.Generator().manual_seed(12)
    re = torch.randint(-7, 8, (2, 20, 11), generator=g)
    im = torch.randint(-7, 8, (2, 20, 11), generator=g)
    v = oracle.correlate(np_(synth.pack_ci4(re, im)), "ci4")
    vc = oracle.correlate(np_(synth.pack_ci4(re, -im)), "ci4")
    np.testing.assert_array_equal(vc[..., 0], v[..., 0])
    np.testing.assert_array_equal(vc[..., 1], -v[..., 1])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_common_phase_rotation_leaves_v_unchanged(k):
    g = torch.Generator().manual_seed(13)
    re = torch.randint(-7, 8, (2, 20, 11), generator=g)
    im = torch.randint(-7, 8, (2, 20, 11), generator=g)
    v = oracle.correlate(np_(synth.pack_ci4(re, im)), "ci4")
    r, i = re, im
    for _ in range(k):                     # multiply by i: (r, i) -> (-i, r)
        r, i = -i, r
    np.testing.assert_array_equal(oracle.correlate(np_(synth.pack_ci4(r, i)), "ci4"), v)


def test_zero_input():
    x = np.zeros((2, 50, 9), dtype=np.uint8)
    assert not oracle.correlate(x, "ci4").any()


# -------------------------------------------------------- closed-form tone (exact)

def test_exact_tone_closed_form():
    # x_i[c,t] = i^k[c,t] q_i[c] -> V_ij[c] = N_t q_i conj(q_j) exactly
    w = synth.scaled(synth.WORKLOADS["paper_exact"], n_channels=24, n_time=128, n_inputs=40)
    x = np_(synth.generate(w))
    v = oracle.correlate(x, "ci4")
    qr, qi = synth.exact_tone_amplitudes(w)
    q = qr.numpy() + 1j * qi.numpy()                     # [C][N], exact small ints
    i, j = oracle.tri_index(w.n_inputs)
    exp = w.n_time * q[:, i] * np.conj(q[:, j])
    np.testing.assert_array_equal(v[..., 0], exp.real.astype(np.int64))
    np.testing.assert_array_equal(v[..., 1], exp.imag.astype(np.int64))


def test_exact_tone_fringe_phase_follows_delay():
    # arg V_ij[c] tracks -2 pi nu_c (d_i - d_j) within the 4-bit rounding bound
    w = synth.scaled(synth.WORKLOADS["paper_exact"], n_channels=64, n_time=16, n_inputs=8)
    v = oracle.correlate(np_(synth.generate(w)), "ci4")
    d = synth.delays_ns(w).numpy() * 1e-9
    nu = np.arange(w.n_channels) * synth.CHANNEL_WIDTH_HZ
    i, j = oracle.tri_index(w.n_inputs)
    bound = 2 * math.asin(math.sqrt(2) / 2 / 7) + 1e-9
    for b in range(len(i)):
        ai, aj = i[b] // 2, j[b] // 2
        phase = np.angle(v[:, b, 0] + 1j * v[:, b, 1])
        model = -2 * np.pi * nu * (d[ai] - d[aj])
        err = np.angle(np.exp(1j * (phase - model)))
        assert np.abs(err).max() <= bound


def test_noisy_tone_fringe_slope():
    # noisy PAPER-like recipe: the least-squares fringe slope over channels
    # recovers the delay difference of a baseline (statistical physics check)
    w = synth.scaled(synth.WORKLOADS["paper"], n_channels=128, n_time=512, n_inputs=8)
    v = oracle.correlate(np_(synth.generate(w)), "ci4")
    d = synth.delays_ns(w).numpy() * 1e-9
    nu = np.arange(w.n_channels) * synth.CHANNEL_WIDTH_HZ
    b = 6 * 7 // 2 + 0          # baseline (input 6 = ant 3 X, input 0 = ant 0 X)
    z = v[:, b, 0] + 1j * v[:, b, 1]
    ph = np.unwrap(np.angle(z))
    slope = np.polyfit(nu, ph, 1)[0]
    expect = -2 * np.pi * (d[3] - d[0])
    assert slope == pytest.approx(expect, rel=0.05, abs=2 * np.pi * 2e-9)


# ------------------------------------------------------------- beam-power identity

@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_beam_power_identity(fmt):
    x = np_(synth.random_input(5, 77, 29, fmt, seed=14))
    v = oracle.correlate(x, fmt)
    g = np.random.default_rng(15)
    for _ in range(3):
        w = g.integers(-3, 4, size=(29, 2))
        np.testing.assert_array_equal(oracle.hermitian_form(v, w), oracle.beam_power(x, fmt, w))


def test_beam_power_detects_a_single_wrong_entry():
    x = np_(synth.random_input(2, 30, 12, "ci4", seed=16))
    v = oracle.correlate(x, "ci4")
    w = np.random.default_rng(17).integers(-3, 4, size=(12, 2))
    w[w == 0] = 1
    p = oracle.beam_power(x, "ci4", w)
    bad = v.copy()
    bad[1, 40, 1] += 1
    assert (oracle.hermitian_form(bad, w) != p).any()


# ------------------------------------------------------------ overflow closed form

@pytest.mark.parametrize("fmt,re,im,per_sample", [("ci4", -8, -8, 128), ("ci8", 127, 127, 32258),
                                                  ("ci8", -128, -128, 32768)])
def test_constant_input_past_int32(fmt, re, im, per_sample):
    # every sample equal to x: V_ij = N_t |x|^2 for all i >= j; N_t chosen so
    # that the sums pass 2^31
    n_t = (2 ** 31) // per_sample + 3
    x = np_(synth.constant_input(1, n_t, 2, fmt, re, im))
    v = oracle.correlate(x, fmt)
    assert (v[..., 0] == n_t * per_sample).all()
    assert (v[..., 1] == 0).all()
    assert v[0, 0, 0] > 2 ** 31


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_row_range_matches_full_channel(fmt):
    x = np_(synth.random_input(3, 50, 23, fmt, seed=18))
    full = oracle.correlate(x, fmt)
    for r0, rc in ((0, 1), (5, 7), (22, 1), (0, 23)):
        a = r0 * (r0 + 1) // 2
        b = (r0 + rc) * (r0 + rc + 1) // 2
        np.testing.assert_array_equal(oracle.correlate_rows(x, fmt, 2, r0, rc), full[2, a:b])
