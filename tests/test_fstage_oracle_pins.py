"""Pins of the F-stage oracle (Sec. 2.3; Sec. 4: 8-bit real samples at 200 MHz,
2-tap 8192-point PFB, 24.4 kHz channels, 4+4-bit requantisation, a contiguous
sub-band of channels) against things other than itself:

  * the filter-bank sum written as sample-by-sample Python loops;
  * a direct O(N^2) DFT in Python complex arithmetic (pins the sign of the
    exponent and which N/2 bins are the channels);
  * the tap order (a prototype that keeps only one tap is a plain DFT of
    that frame);
  * a tone at the centre frequency of channel k (the paper's clock and
    transform size) lands in channel k, with the closed-form amplitude;
  * rounding and saturation of the requantiser, and the nibble encoding the
    X-stage decodes;
  * the output layout, gains and channel selection, from tones placed in
    known channels of known inputs.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1401_8288_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_numbers.json")


def rng(seed):
    return np.random.default_rng(seed)


def test_pfb_frames_match_sample_loops():
    N, P, A, S = 8, 2, 3, 50
    x = rng(1).integers(-128, 128, (A, S)).astype(np.int8)
    h = rng(2).normal(size=P * N)
    y = oracle.pfb_frames(x, h, N, P)
    n_spec = S // N - P + 1
    assert y.shape == (A, n_spec, N)
    for a in range(A):
        for m in range(n_spec):
            for j in range(N):
                ref = 0.0
                for p in range(P):
                    ref += float(h[p * N + j]) * int(x[a, (m + p) * N + j])
                assert abs(y[a, m, j] - ref) < 1e-9


@pytest.mark.parametrize("P", [1, 2])
def test_spectra_match_direct_dft(P):
    N, A, S = 16, 2, 80
    x = rng(3 + P).integers(-128, 128, (A, S)).astype(np.int8)
    h = rng(5).normal(size=P * N)
    X = oracle.pfb_spectra(x, h, N, P)
    n_spec = S // N - P + 1
    assert X.shape == (A, n_spec, N // 2)
    for a in range(A):
        for m in range(n_spec):
            y = [sum(float(h[p * N + j]) * int(x[a, (m + p) * N + j]) for p in range(P)) for j in range(N)]
            for k in range(N // 2):
                ref = sum(y[j] * cmath.exp(-2j * math.pi * j * k / N) for j in range(N))
                assert abs(X[a, m, k] - ref) < 1e-9 * (1 + abs(ref))


def test_a_prototype_with_one_tap_is_the_dft_of_that_frame():
    N, S = 32, 32 * 6
    x = rng(7).integers(-128, 128, (1, S)).astype(np.int8)
    first = np.concatenate([np.ones(N), np.zeros(N)])
    second = np.concatenate([np.zeros(N), np.ones(N)])
    X1 = oracle.pfb_spectra(x, first, N, 2)
    X2 = oracle.pfb_spectra(x, second, N, 2)
    for m in range(X1.shape[1]):
        for k in (0, 1, 5, N // 2 - 1):
            f0 = sum(int(x[0, m * N + j]) * cmath.exp(-2j * math.pi * j * k / N) for j in range(N))
            f1 = sum(int(x[0, (m + 1) * N + j]) * cmath.exp(-2j * math.pi * j * k / N) for j in range(N))
            assert abs(X1[0, m, k] - f0) < 1e-8 and abs(X2[0, m, k] - f1) < 1e-8


def test_channel_zero_is_real_for_real_samples():
    x = rng(9).integers(-128, 128, (2, 64 * 5)).astype(np.int8)
    X = oracle.pfb_spectra(x, rng(10).normal(size=128), 64, 2)
    assert np.abs(X[..., 0].imag).max() < 1e-9


def test_tone_at_a_channel_centre_lands_in_that_channel():
    g = json.load(open(GOLDEN))
    N = synth.PFB_POINTS
    spacing = synth.ADC_CLOCK_HZ / N
    assert round(spacing / 1e3, 1) == g["channel_spacing_khz"]["value"]
    k0, amp = 1234, 100.0
    t = np.arange(3 * N)
    x = np.clip(np.rint(amp * np.cos(2 * math.pi * k0 * spacing / synth.ADC_CLOCK_HZ * t + 0.3)),
                -128, 127).astype(np.int8)[None, :]
    # rectangular single-tap prototype: X[k0] = N A / 2 e^{i phi}, the rest is
    # the rounding noise of the 8-bit samples
    X = oracle.pfb_spectra(x, np.ones(N), N, 1)
    for m in range(X.shape[1]):
        assert np.argmax(np.abs(X[0, m])) == k0
        assert abs(X[0, m, k0] - N * amp / 2 * cmath.exp(0.3j)) < 0.002 * N * amp / 2
    # the paper's 2-tap prototype: the same channel, gain sum of the sinc lobe
    h = synth.pfb_coefficients(2, N).numpy().astype(np.float64)
    X2 = oracle.pfb_spectra(x, h, N, 2)
    assert all(np.argmax(np.abs(X2[0, m])) == k0 for m in range(X2.shape[1]))
    # 1628 channels of 24.4 kHz are the ~40 MHz sub-band of the demonstration
    assert round(g["subband_mhz"]["channels"] * spacing / 1e6) == g["subband_mhz"]["value"]


def test_requantiser_rounds_half_to_even_and_saturates_symmetrically():
    v = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 6.49, 6.5, 7.5, 100.0, -6.5, -7.5, -100.0])
    assert oracle.requantise4(v).tolist() == [0, 2, 2, 0, -2, -2, 6, 6, 7, 7, -6, -7, -7]


def test_fstage_layout_gain_and_selection():
    # input a carries a tone at the centre of channel 10 + 3a; with a
    # single-tap rectangular prototype X = N A / 2 there, and the gain
    # 5 / (N A / 2) makes the requantised sample exactly 5 + 0i (0x50)
    N, A_in, amp = 64, 4, 100.0
    n_spec = 3
    t = np.arange(n_spec * N)
    x = np.stack([np.rint(amp * np.cos(2 * math.pi * (10 + 3 * a) * t / N)) for a in range(A_in)]).astype(np.int8)
    ch0, n_ch = 8, 16
    gain = np.full((A_in, n_ch), 5.0 / (N * amp / 2))
    gain[2, :] *= -1.0                       # input 2: -5 + 0i (0xB0)
    out = oracle.fstage(x, np.ones(N), gain, N, 1, ch0, n_ch)
    assert out.shape == (n_ch, n_spec, A_in) and out.dtype == np.uint8
    for a in range(A_in):
        c = 10 + 3 * a - ch0
        want = 0xB0 if a == 2 else 0x50
        assert (out[c, :, a] == want).all()
        others = np.delete(out[:, :, a], c, axis=0)
        assert (others == 0).all()
    # the 8-bit rounding of the tone moves X by at most N / 2 (1 % here)
    v = oracle.fstage(x, np.ones(N), gain, N, 1, ch0, n_ch, out="c128")
    assert abs(v[10 - ch0, 0, 0] - 5.0) < 5.0 * 0.01


def test_no_full_spectrum_gives_empty_output():
    x = np.zeros((2, 8192 + 100), dtype=np.int8)
    assert oracle.fstage(x, np.ones(16384), np.ones((2, 4)), 8192, 2, 0, 4).shape == (4, 0, 2)
