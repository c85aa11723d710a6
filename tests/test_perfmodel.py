"""The paper's sizing equations against the numbers it prints (Sec. 2.2-4)."""
import json
import math
import os

import pytest

from paper_1401_8288_amd import perfmodel as pm
from paper_1401_8288_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


T1 = _load("table1_datarate.json")
# The table is evaluated at a ~100 MHz band (Sec. 4: 200 MHz clock -> 100 MHz).
BAND = 100e6


@pytest.mark.parametrize("k", range(5))
def test_eq1_matches_table_tflops(k):
    n = T1["inputs"][k]
    printed = T1["gpu_tflops_required"][k]
    r = pm.eq1_flops_per_bandwidth(n, BAND) / 1e12
    # printed values carry 2-3 significant digits for small N
    assert r == pytest.approx(printed, rel=1e-2)


@pytest.mark.parametrize("k", range(5))
def test_gpu_counts_from_eq1(k):
    # Every GPU-count cell equals floor(R / F) + 1 for the printed R and the
    # per-GPU rate F (at 512 inputs R/3 = 35.0 is printed as 36 GPUs, so the
    # count is not a plain ceiling).
    printed = T1["gpu_tflops_required"][k]
    assert math.floor(printed / 3.0) + 1 == T1["gpus_at_3tflops"][k]
    assert math.floor(printed / 24.0) + 1 == T1["gpus_at_24tflops_read"][k]


def test_garbled_cell_is_only_the_19000_input_column():
    printed = T1["gpus_at_24tflops_printed"]
    read = T1["gpus_at_24tflops_read"]
    diff = [k for k in range(5) if printed[k] != read[k]]
    assert diff == [4]
    # the data-rate cell of that column pins the reading 6014
    n = T1["inputs"][4]
    assert 8 * n * BAND / read[4] / 1e9 == pytest.approx(T1["gbps_per_gpu_at_24tflops"][4],
                                                          rel=5e-3)
    assert 8 * n * BAND / printed[4] / 1e9 > 5 * T1["gbps_per_gpu_at_24tflops"][4]


@pytest.mark.parametrize("k", range(5))
def test_eq2_data_rate_per_gpu(k):
    n = T1["inputs"][k]
    for gpus, col in ((T1["gpus_at_3tflops"], "gbps_per_gpu_at_3tflops"),
                      (T1["gpus_at_24tflops_read"], "gbps_per_gpu_at_24tflops")):
        d = pm.eq2_bits(n, 1, 1.0 / BAND) / gpus[k] / 1e9
        assert d == pytest.approx(T1[col][k], rel=5e-3)


def test_channel_spacing_and_tau():
    w = _load("worked_numbers.json")
    assert synth.CHANNEL_WIDTH_HZ / 1e3 == pytest.approx(w["channel_spacing_khz"]["value"],
                                                         abs=0.05)
    assert synth.SPECTRUM_INTERVAL_S == pytest.approx(40.96e-6, rel=1e-12)
    sub = w["subband_mhz"]
    assert sub["channels"] * synth.CHANNEL_WIDTH_HZ / 1e6 == pytest.approx(sub["value"], rel=0.01)


def test_capture_rate_32_inputs():
    w = _load("worked_numbers.json")["capture_gbps_32_inputs"]
    d = pm.eq2_bits(32, 1628, synth.SPECTRUM_INTERVAL_S) / 1e9
    assert d == pytest.approx(w["value"], rel=0.03)


def test_output_averaging_time():
    w = _load("worked_numbers.json")["integration_seconds"]
    t = w["gpu_spectra"] * w["cpu_dumps"] * synth.SPECTRUM_INTERVAL_S
    assert t == pytest.approx(w["value"], abs=0.005)


def test_max_inputs_one_channel():
    w = _load("worked_numbers.json")["max_inputs_3tflops_one_channel"]
    n = pm.max_inputs_per_channel(3e12, synth.SPECTRUM_INTERVAL_S)
    assert n == pytest.approx(w["value"], rel=0.02)
    assert pm.eq1_flops(n, 1, synth.SPECTRUM_INTERVAL_S) == pytest.approx(3e12, rel=1e-9)


def test_optimal_inputs_at_2p6mhz():
    w = _load("worked_numbers.json")["optimal_inputs_2p6mhz"]
    for tf, expect in zip(w["tflops"], w["value"]):
        n = pm.optimal_inputs(tf * 1e12, 2.6e6)
        assert n == pytest.approx(expect, rel=0.1)


def test_eq3_reduces_to_eq2_for_one_server():
    # all inputs and all channels into one server: D_I = D
    assert pm.eq3_bits_per_server(4, 8, 0, 1628, 1, 40.96e-6) == \
        pytest.approx(pm.eq2_bits(32, 1628, 40.96e-6))
    # N servers split the band evenly
    assert pm.eq3_bits_per_server(4, 8, 0, 1628, 2, 40.96e-6) == \
        pytest.approx(pm.eq2_bits(32, 1628, 40.96e-6) / 2)


def test_eq4_counts_station_blocks():
    # Eq. 4 with N_s = N_i / 2 stations is N_c N_s (N_s/2 + 1) N_pol^2: the
    # N_s (N_s + 1) / 2 station pairs of the triangle packed into N_s/2 + 1
    # columns of 2x2 polarisation blocks, N_s/2 pairs more than the triangle.
    # Per channel that is N_i (N_i + 4) / 2 entries: 1.5 N_i more than the
    # input triangle N_i (N_i + 1) / 2 that the X-stage here returns.
    for n in (32, 64, 512, 2048):
        ns = n // 2
        assert pm.eq4_output_size(1, n) == n * (n + 4) / 2
        assert pm.eq4_output_size(1, n) == 4 * (ns * (ns + 1) / 2 + ns / 2)
        assert pm.eq4_output_size(1, n) - n * (n + 1) / 2 == 1.5 * n


def test_cmac_unit_is_eq1_over_8():
    n, c, tau = 512, 4096, synth.SPECTRUM_INTERVAL_S
    cmac = pm.cmac_per_s(n, c, 1, tau)
    assert cmac * pm.FLOP_PER_CMAC == pytest.approx(pm.eq1_flops(n, c, tau))
