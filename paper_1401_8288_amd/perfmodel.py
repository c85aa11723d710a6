"""The paper's sizing equations (Sec. 2.2 and Sec. 2.4) and the metric units.

Eq. 1  R    = 4 N_i (N_i + 1) N_c / tau          single-precision flop/s
Eq. 2  D    = 8 N_i N_c / tau                    bit/s into the X-stage
Eq. 3  D_I  = 8 N_r N_a (High_ch - Low_ch) / (N_serv tau)   bit/s per server
Eq. 4  D_cc = N_c (N_i/4 + 1)(N_i/2) N_pol^2     size of the output matrix

Eq. 1 counts 8 flop per baseline (N_i (N_i+1)/2 baselines incl. autos) per
channel per spectrum, i.e. 8 flop per complex multiply-accumulate (CMAC):
CMAC/s = R / 8.  The paper notes 4 flop per fused complex multiply-add on
GPUs and divides Eq. 1 by four for a fixed-point comparison (Sec. 2.2).
"""
from __future__ import annotations

import math

FLOP_PER_CMAC = 8
# MI355X dense peaks (vendor figures): int8 MFMA, fp16 MFMA, fp32 vector.
PEAK_INT8_OPS = 5.0e15
PEAK_FP16_FLOPS = 2.5e15
PEAK_FP32_FLOPS = 157.3e12
PEAK_FP32_UNPACKED_FLOPS = 78.6e12
PEAK_HBM_BYTES = 8.0e12


def eq1_flops(n_inputs: float, n_channels: float, tau_s: float) -> float:
    """R = 4 N_i (N_i + 1) N_c / tau (flop/s)."""
    return 4.0 * n_inputs * (n_inputs + 1) * n_channels / tau_s


def eq1_flops_per_bandwidth(n_inputs: float, bandwidth_hz: float) -> float:
    """Eq. 1 with N_c / tau = bandwidth (one spectrum per channel per tau)."""
    return 4.0 * n_inputs * (n_inputs + 1) * bandwidth_hz


def eq2_bits(n_inputs: float, n_channels: float, tau_s: float) -> float:
    """D = 8 N_i N_c / tau (bit/s): 8 bits per complex 4+4-bit sample."""
    return 8.0 * n_inputs * n_channels / tau_s


def eq3_bits_per_server(n_nodes: float, inputs_per_node: float, low_ch: float, high_ch: float,
                        n_servers: float, tau_s: float) -> float:
    """D_I = 8 N_r N_a (High_ch - Low_ch) / (N_serv tau) (bit/s)."""
    return 8.0 * n_nodes * inputs_per_node * (high_ch - low_ch) / (n_servers * tau_s)


def eq4_output_size(n_channels: float, n_inputs: float, n_pol: int = 2) -> float:
    """D_cc = N_c (N_i/4 + 1)(N_i/2) N_pol^2 (elements, as printed)."""
    return n_channels * (n_inputs / 4.0 + 1.0) * (n_inputs / 2.0) * n_pol ** 2


def cmac_per_s(n_inputs: int, n_channels: int, n_time: int, seconds: float) -> float:
    """Useful complex MACs per second: N_b N_c N_t / t (lower triangle with autos)."""
    return n_inputs * (n_inputs + 1) // 2 * n_channels * n_time / seconds


def gpus_required(n_inputs: float, bandwidth_hz: float, per_gpu_flops: float) -> int:
    return int(math.ceil(eq1_flops_per_bandwidth(n_inputs, bandwidth_hz) / per_gpu_flops))


def data_rate_per_gpu_bits(n_inputs: float, bandwidth_hz: float, per_gpu_flops: float) -> float:
    """Eq. 2 total divided over the GPUs of `gpus_required`."""
    return 8.0 * n_inputs * bandwidth_hz / gpus_required(n_inputs, bandwidth_hz, per_gpu_flops)


def max_inputs_per_channel(per_gpu_flops: float, tau_s: float) -> float:
    """Largest N_i one GPU can correlate for a single channel in real time (Eq. 1)."""
    # 4 N (N + 1) / tau = F  ->  N = (-1 + sqrt(1 + F tau)) / 2
    return (-1.0 + math.sqrt(1.0 + per_gpu_flops * tau_s)) / 2.0


def optimal_inputs(per_gpu_flops: float, bandwidth_hz: float) -> float:
    """N_i at which Eq. 1 for `bandwidth_hz` equals the GPU's rate."""
    # 4 N (N + 1) B = F
    return (-1.0 + math.sqrt(1.0 + per_gpu_flops / bandwidth_hz)) / 2.0
