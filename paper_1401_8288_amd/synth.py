"""Seeded synthetic channelised voltages shaped like the paper's arrays.

This module only draws random numbers, quantises them and packs them into the
X-stage input layout.  It holds none of the correlation arithmetic, and both
the HIP path and the CPU oracle take their inputs from it.

Shapes and statistics
  * Channel spacing 200 MHz / 8192 = 24.414 kHz, so one spectrum every
    40.96 us (Sec. 4: 200 MHz ADC clock, 8192-point PFB).
  * Inputs = 2 x antennas (two polarisations, Sec. 2.2); input index
    i = 2 * antenna + pol.
  * Samples are requantised to 4 bits real + 4 bits imaginary (Sec. 2.3,
    Sec. 4) because channel data are noise-like; here Q(v) rounds half to
    even and then clips each component.
  * Geometric delays d_ant ~ U[-300, 300] ns, the scale of the 5-98 m
    spacings of the field demonstration (Sec. 4); the sky signal then has the
    fringe phase -2 pi nu_c d_ant, linear in channel (Sec. 4, fringes figure).

Layout: ci4 -> uint8 [channel][time][input] (high nibble = real, low nibble =
imaginary, two's complement); ci8 -> int8 [channel][time][input][2].
Large workloads are generated on the device in fixed 16-channel chunks, each
from its own seeded generator, so a given (workload, seed, device) always
yields the same bytes whatever the caller's chunking.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

ADC_CLOCK_HZ = 200e6
PFB_POINTS = 8192
CHANNEL_WIDTH_HZ = ADC_CLOCK_HZ / PFB_POINTS      # 24414.0625 Hz
SPECTRUM_INTERVAL_S = 1.0 / CHANNEL_WIDTH_HZ      # 40.96 us
CHUNK_CHANNELS = 16


@dataclass(frozen=True)
class Workload:
    name: str
    n_inputs: int
    n_channels: int
    n_time: int
    fmt: str            # "ci4" | "ci8"
    recipe: str
    seed: int
    params: dict = field(default_factory=dict, hash=False, compare=False)

    @property
    def n_antennas(self) -> int:
        return self.n_inputs // 2

    @property
    def bytes_per_sample(self) -> int:
        return 1 if self.fmt == "ci4" else 2

    @property
    def n_baselines(self) -> int:
        return self.n_inputs * (self.n_inputs + 1) // 2

    @property
    def cmac(self) -> int:
        """Useful complex multiply-accumulates per integration."""
        return self.n_baselines * self.n_channels * self.n_time

    @property
    def input_bytes(self) -> int:
        return self.n_inputs * self.n_channels * self.n_time * self.bytes_per_sample

    @property
    def output_bytes(self) -> int:
        return self.n_baselines * self.n_channels * 16


WORKLOADS = {
    # 32 antennas x 2 pol, 64 channels, 1024 samples; uniform integers in [-7, 7].
    "tiny": Workload("tiny", 64, 64, 1024, "ci4", "uniform", 1),
    # 64 antennas x 2 pol (PAPER-like), 1024 channels, 2048 samples; noise plus a
    # common constant-envelope tone with per-antenna delay.
    "paper": Workload("paper", 128, 1024, 2048, "ci4", "tone", 2,
                      {"noise_sigma": 2.5, "tone_gain": 1.5}),
    # Noise-free variant whose visibilities have a closed form.
    "paper_exact": Workload("paper_exact", 128, 1024, 2048, "ci4", "exact_tone", 2,
                            {"amplitude": 7.0}),
    # 256 antennas x 2 pol (LWA-scale), 4096 channels, 4096 samples; Gaussian
    # noise plus a point source of correlation coefficient 0.05.
    "lwa": Workload("lwa", 512, 4096, 4096, "ci4", "point_source", 3,
                    {"scale": 2.5, "rho": 0.05}),
    # 1024 antennas x 2 pol, 256 channels, 8192 samples; 8+8-bit Gaussian.
    "large_n": Workload("large_n", 2048, 256, 8192, "ci8", "gauss8", 4, {"sigma": 32.0}),
}

# Five concurrent subarrays (antennas, channels) of the batched streaming case.
SUBARRAYS = [(16, 512), (48, 1024), (96, 2048), (200, 256), (352, 128)]


def subarray_workload(k: int, n_time: int) -> Workload:
    ant, ch = SUBARRAYS[k]
    return Workload("sub%d" % k, 2 * ant, ch, n_time, "ci4", "tone", 5 + 100 * k,
                    {"noise_sigma": 2.5, "tone_gain": 0.0})


def scaled(w: Workload, **kw) -> Workload:
    """Same recipe and seed at another shape (tests use this for small cases)."""
    d = dict(name=w.name, n_inputs=w.n_inputs, n_channels=w.n_channels, n_time=w.n_time,
             fmt=w.fmt, recipe=w.recipe, seed=w.seed, params=dict(w.params))
    d.update(kw)
    return Workload(**d)


# ------------------------------------------------------------------ helpers

def quantise(v: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    """Round half to even, then clip (per component)."""
    return torch.clamp(torch.round(v), lo, hi)


def pack_ci4(re: torch.Tensor, im: torch.Tensor) -> torch.Tensor:
    """Pack integer components in [-8, 7] into bytes: high nibble re, low im."""
    r = re.to(torch.int32) & 0xF
    i = im.to(torch.int32) & 0xF
    return ((r << 4) | i).to(torch.uint8)


def pack_ci8(re: torch.Tensor, im: torch.Tensor) -> torch.Tensor:
    return torch.stack([re.to(torch.int8), im.to(torch.int8)], dim=-1)


def delays_ns(w: Workload) -> torch.Tensor:
    """Per-antenna geometric delay (ns), always drawn on the CPU."""
    g = torch.Generator(device="cpu").manual_seed(1000 + w.seed)
    return (torch.rand(w.n_antennas, generator=g, dtype=torch.float64) * 600.0 - 300.0)


def channel_freq_hz(n_channels: int, device) -> torch.Tensor:
    return torch.arange(n_channels, device=device, dtype=torch.float64) * CHANNEL_WIDTH_HZ


def geometric_phasor(w: Workload, c0: int, c1: int, device):
    """exp(-2 pi i nu_c d_ant) for channels [c0, c1), shape [C][ant] (re, im) float64."""
    nu = channel_freq_hz(w.n_channels, device)[c0:c1]
    d = delays_ns(w).to(device) * 1e-9
    ph = -2.0 * math.pi * nu[:, None] * d[None, :]
    return torch.cos(ph), torch.sin(ph)


def exact_tone_amplitudes(w: Workload, c0: int = 0, c1: int | None = None, device="cpu"):
    """q_i[c] = Q(A exp(-2 pi i nu_c d_ant(i))) as int64 (re, im), [C][n_inputs]."""
    c1 = w.n_channels if c1 is None else c1
    amp = float(w.params.get("amplitude", 7.0))
    cr, ci = geometric_phasor(w, c0, c1, device)
    qr = quantise(amp * cr, -7, 7).to(torch.int64)
    qi = quantise(amp * ci, -7, 7).to(torch.int64)
    # both polarisations of an antenna see the same tone
    return qr.repeat_interleave(2, dim=1), qi.repeat_interleave(2, dim=1)


def _chunk_generator(w: Workload, chunk: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((w.seed * 1_000_003 + chunk * 7919 + 17) % (2 ** 63))
    return g


def _gen_chunk(w: Workload, c0: int, c1: int, device):
    """Integer (re, im) components for channels [c0, c1), shape [C][T][N]."""
    C, T, N = c1 - c0, w.n_time, w.n_inputs
    g = _chunk_generator(w, c0 // CHUNK_CHANNELS, device)
    p = w.params
    if w.recipe == "uniform":
        re = torch.randint(-7, 8, (C, T, N), generator=g, device=device)
        im = torch.randint(-7, 8, (C, T, N), generator=g, device=device)
        return re, im
    if w.recipe == "gauss8":
        s = float(p.get("sigma", 32.0))
        re = quantise(torch.randn((C, T, N), generator=g, device=device) * s, -127, 127)
        im = quantise(torch.randn((C, T, N), generator=g, device=device) * s, -127, 127)
        return re, im
    if w.recipe == "exact_tone":
        qr, qi = exact_tone_amplitudes(w, c0, c1, device)          # [C][N]
        k = torch.randint(0, 4, (C, T, 1), generator=g, device=device)
        # multiply q by i^k: k=1 -> (-im, re); k=2 -> (-re, -im); k=3 -> (im, -re)
        qr = qr[:, None, :].expand(C, T, N)
        qi = qi[:, None, :].expand(C, T, N)
        re = torch.where(k == 0, qr, torch.where(k == 1, -qi, torch.where(k == 2, -qr, qi)))
        im = torch.where(k == 0, qi, torch.where(k == 1, qr, torch.where(k == 2, -qi, -qr)))
        return re, im
    cr, ci = geometric_phasor(w, c0, c1, device)                    # [C][ant]
    cr = cr.to(torch.float32).repeat_interleave(2, dim=1)[:, None, :]
    ci = ci.to(torch.float32).repeat_interleave(2, dim=1)[:, None, :]
    if w.recipe == "tone":
        sig = float(p.get("noise_sigma", 2.5))
        gain = float(p.get("tone_gain", 1.5))
        nr = torch.randn((C, T, N), generator=g, device=device) * sig
        ni = torch.randn((C, T, N), generator=g, device=device) * sig
        # unit-modulus tone, independent phase per (channel, time, pol)
        psi = torch.rand((C, T, 2), generator=g, device=device) * (2.0 * math.pi)
        sr = torch.cos(psi).repeat(1, 1, N // 2)
        si = torch.sin(psi).repeat(1, 1, N // 2)
        # s * phasor
        tr = sr * cr - si * ci
        ti = sr * ci + si * cr
        re = quantise(nr + gain * tr, -7, 7)
        im = quantise(ni + gain * ti, -7, 7)
        return re, im
    if w.recipe == "point_source":
        scale = float(p.get("scale", 2.5))
        rho = float(p.get("rho", 0.05))
        nr = torch.randn((C, T, N), generator=g, device=device)
        ni = torch.randn((C, T, N), generator=g, device=device)
        s = torch.randn((C, T, 2, 2), generator=g, device=device)    # [.., pol, re/im]
        sr = s[..., 0].repeat(1, 1, N // 2)
        si = s[..., 1].repeat(1, 1, N // 2)
        tr = sr * cr - si * ci
        ti = sr * ci + si * cr
        a, b = math.sqrt(1.0 - rho), math.sqrt(rho)
        re = quantise(scale * (a * nr + b * tr), -7, 7)
        im = quantise(scale * (a * ni + b * ti), -7, 7)
        return re, im
    raise ValueError("unknown recipe %r" % w.recipe)


def generate(w: Workload, device="cpu", out: torch.Tensor | None = None) -> torch.Tensor:
    """The packed input buffer of a workload, generated on `device`."""
    shape = (w.n_channels, w.n_time, w.n_inputs) if w.fmt == "ci4" else \
        (w.n_channels, w.n_time, w.n_inputs, 2)
    dtype = torch.uint8 if w.fmt == "ci4" else torch.int8
    if out is None:
        out = torch.empty(shape, dtype=dtype, device=device)
    elif tuple(out.shape) != shape or out.dtype != dtype:
        raise ValueError("output buffer has the wrong shape or dtype")
    for c0 in range(0, w.n_channels, CHUNK_CHANNELS):
        c1 = min(w.n_channels, c0 + CHUNK_CHANNELS)
        re, im = _gen_chunk(w, c0, c1, out.device)
        out[c0:c1] = pack_ci4(re, im) if w.fmt == "ci4" else pack_ci8(re, im)
    return out


def constant_input(n_channels: int, n_time: int, n_inputs: int, fmt: str, re: int, im: int,
                   device="cpu") -> torch.Tensor:
    """Every sample equal to re + i im (worst-case and closed-form cases)."""
    shape = (n_channels, n_time, n_inputs)
    r = torch.full(shape, re, dtype=torch.int32, device=device)
    i = torch.full(shape, im, dtype=torch.int32, device=device)
    return pack_ci4(r, i) if fmt == "ci4" else pack_ci8(r, i)


def random_input(n_channels: int, n_time: int, n_inputs: int, fmt: str, seed: int,
                 lo: int | None = None, hi: int | None = None, device="cpu") -> torch.Tensor:
    """Uniform integer components over the full range of a format (edge-case tests)."""
    lo = (-8 if fmt == "ci4" else -127) if lo is None else lo
    hi = (7 if fmt == "ci4" else 127) if hi is None else hi
    g = torch.Generator(device=device).manual_seed(seed)
    shape = (n_channels, n_time, n_inputs)
    re = torch.randint(lo, hi + 1, shape, generator=g, device=device)
    im = torch.randint(lo, hi + 1, shape, generator=g, device=device)
    return pack_ci4(re, im) if fmt == "ci4" else pack_ci8(re, im)


# ------------------------------------------------------------------ F-stage inputs
#
# The F-stage of Sec. 2.3 takes 8-bit real ADC samples (Sec. 4: 200 MHz clock)
# through a 2-tap, 8192-point PFB.  The prototype filter and the equaliser
# gains are inputs of that stage, drawn here like the samples.

def pfb_coefficients(n_taps: int = 2, n_points: int = PFB_POINTS) -> torch.Tensor:
    """Prototype filter of P taps x N points: a sinc whose main lobe spans one
    channel, times a Hamming window over the P N coefficients (float32, CPU).
    The paper gives the taps and points only; this shape is the usual one for
    critically sampled PFBs."""
    P, N = n_taps, n_points
    k = torch.arange(P * N, dtype=torch.float64)
    u = (k + 0.5) / N - P / 2.0
    ham = 0.54 - 0.46 * torch.cos(2.0 * math.pi * k / max(P * N - 1, 1))
    return (torch.sinc(u) * ham).to(torch.float32)


def adc_input(n_inputs: int, n_samples: int, seed: int, sigma: float = 16.0, rho: float = 0.05,
              tone_amp: float = 0.0, tone_hz: float = 0.0, device="cpu", out: torch.Tensor | None = None):
    """Real int8 ADC streams [n_inputs][n_samples]: per input, independent
    Gaussian noise plus a common sky signal (fraction rho of the power) delayed
    by 0..15 samples per input, plus an optional common tone, rounded half to
    even and clipped to [-128, 127]."""
    if out is None:
        out = torch.empty((n_inputs, n_samples), dtype=torch.int8, device=device)
    elif tuple(out.shape) != (n_inputs, n_samples) or out.dtype != torch.int8:
        raise ValueError("output buffer has the wrong shape or dtype")
    dev = out.device
    g = torch.Generator(device=dev).manual_seed(seed * 7_654_321 + 11)
    common = torch.randn(n_samples + 16, generator=g, device=dev, dtype=torch.float32)
    gd = torch.Generator(device="cpu").manual_seed(seed + 99)
    delays = torch.randint(0, 16, (n_inputs,), generator=gd)
    t = torch.arange(n_samples, device=dev, dtype=torch.float64)
    tone = (tone_amp * torch.cos(2.0 * math.pi * tone_hz / ADC_CLOCK_HZ * t)).to(torch.float32) \
        if tone_amp else None
    a_n, a_c = sigma * math.sqrt(1.0 - rho), sigma * math.sqrt(rho)
    for a in range(n_inputs):
        ga = torch.Generator(device=dev).manual_seed(seed * 1_000_003 + 31 * a + 5)
        v = a_n * torch.randn(n_samples, generator=ga, device=dev, dtype=torch.float32)
        d = int(delays[a])
        v += a_c * common[16 - d:16 - d + n_samples]
        if tone is not None:
            v += tone
        out[a] = torch.clamp(torch.round(v), -128, 127).to(torch.int8)
    return out


def fstage_gains(n_inputs: int, n_chan: int, coeff: torch.Tensor, sigma: float = 16.0,
                 target: float = 2.5, seed: int = 0) -> torch.Tensor:
    """Equaliser gains [n_inputs][n_chan] (float32, CPU) that bring white
    noise of rms sigma to rms `target` per component after the PFB, with a
    +-10 % spread per input and channel (a bandpass to flatten)."""
    norm = sigma * math.sqrt(float((coeff.double() ** 2).sum()) / 2.0)
    g = torch.Generator(device="cpu").manual_seed(seed + 4242)
    spread = 1.0 + 0.1 * (2.0 * torch.rand((n_inputs, n_chan), generator=g, dtype=torch.float64) - 1.0)
    return (target / norm * spread).to(torch.float32)
