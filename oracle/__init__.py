"""CPU oracle for the X-stage cross-multiply-accumulate.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product package never imports this
module, and this module never imports the product package; the two share
nothing but the layout convention of their buffers.

Contents
  correlate      -- the plain int64 definition (C, OpenMP over channels).
                    V[c][i][j] = sum_t x_i[c,t] conj(x_j[c,t]) for i >= j
                    (Sec. 1: outer product per time and frequency; Sec. 2.4:
                    cross multiplication into a lower-triangular matrix per
                    channel; Sec. 2.1: integration on the GPU).
  beam_power     -- sum_t |sum_i conj(w_i) x_i|^2 per channel, the O(N T)
                    side of the identity  w^H V w = beam power  used to check
                    full-size results.
  hermitian_form -- w^H V w evaluated from a lower-triangle result.
  brute_force    -- pure-Python integer loops for tiny inputs.
  matmul_form    -- the same sums as exact int64 numpy matrix products.
  corner_turn    -- F-engine packet order -> X-stage input order, with the
                    4 -> 8 bit promotion and zeros for lost packets (Sec. 2.4:
                    packets placed by sequence number and F-engine; the
                    unpacker pads 4 to 8 bits and reorders the channels of
                    the F-engines next to each other; packet-format figure:
                    the spectra of a packet follow one another).
  pfb_frames,    -- the F-stage of Sec. 2.3 (and Sec. 4: 2 taps, 8192
  pfb_spectra,      points, 8-bit real ADC samples): polyphase filter bank
  requantise4,      (weighted sum of consecutive frames, then a real DFT
  fstage            whose first N/2 bins are the channels), equalisation by
                    a real gain per input and channel, requantisation to 4+4
                    bits, and selection of a contiguous run of channels,
                    written in X-stage order.

Formats: "ci4" = one byte per sample, high nibble real, low nibble imaginary,
two's complement (Sec. 2.3: 4 bits real and 4 bits imaginary); "ci8" = two
signed bytes per sample, real then imaginary (the 8-bit form of Sec. 2.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xcorr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FORMATS = {"ci4": 0, "ci8": 1}


# The library is built where the tests run and then copied to the machine
# that runs it, whose host CPU may differ: x86-64-v3 (AVX2) is the widest
# target both are known to have, so the loops may auto-vectorise to AVX2.
CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def compiler() -> str:
    """The compiler and flags the C oracle is built with."""
    try:
        v = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        v = "gcc (version unknown)"
    return "%s, %s" % (v, " ".join(CFLAGS[:3]))


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc"] + CFLAGS + ["-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        L.xo_correlate.argtypes = [ctypes.c_void_p, ctypes.c_int, i64, i64, i64, i64, i64,
                                   ctypes.c_void_p]
        L.xo_correlate.restype = ctypes.c_int
        L.xo_correlate_rows.argtypes = [ctypes.c_void_p, ctypes.c_int, i64, i64, i64, i64, i64,
                                        i64, ctypes.c_void_p]
        L.xo_correlate_rows.restype = ctypes.c_int
        L.xo_beam_power.argtypes = [ctypes.c_void_p, ctypes.c_int, i64, i64, i64,
                                    ctypes.c_void_p, ctypes.c_void_p]
        L.xo_beam_power.restype = ctypes.c_int
        L.xo_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(lib().xo_threads())


def _shape(x: np.ndarray, fmt: str):
    if fmt == "ci4":
        if x.dtype != np.uint8 or x.ndim != 3:
            raise ValueError("ci4 input must be uint8 [channel][time][input]")
        n_ch, n_t, n_in = x.shape
    elif fmt == "ci8":
        if x.dtype != np.int8 or x.ndim != 4 or x.shape[3] != 2:
            raise ValueError("ci8 input must be int8 [channel][time][input][2]")
        n_ch, n_t, n_in, _ = x.shape
    else:
        raise ValueError("unknown format %r" % fmt)
    return n_ch, n_t, n_in


def n_baselines(n_in: int) -> int:
    return n_in * (n_in + 1) // 2


def correlate(x: np.ndarray, fmt: str, channels=None) -> np.ndarray:
    """Exact visibilities, int64 [len(channels)][n_in(n_in+1)/2][2] (re, im).

    `channels` is None (all) or a (begin, count) range.
    """
    n_ch, n_t, n_in = _shape(x, fmt)
    x = np.ascontiguousarray(x)
    begin, count = (0, n_ch) if channels is None else channels
    out = np.empty((count, n_baselines(n_in), 2), dtype=np.int64)
    rc = lib().xo_correlate(x.ctypes.data, FORMATS[fmt], n_ch, n_t, n_in, begin, count,
                            out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def correlate_rows(x: np.ndarray, fmt: str, channel: int, row_begin: int, row_count: int):
    """Rows [row_begin, row_begin+row_count) of one channel's triangle.

    Returns int64 [sum of (i+1) over the rows][2], the same entries in the same
    order as the packed triangle of a full result.
    """
    n_ch, n_t, n_in = _shape(x, fmt)
    x = np.ascontiguousarray(x)
    r0, r1 = row_begin, row_begin + row_count
    n = r1 * (r1 + 1) // 2 - r0 * (r0 + 1) // 2
    out = np.empty((n, 2), dtype=np.int64)
    rc = lib().xo_correlate_rows(x.ctypes.data, FORMATS[fmt], n_ch, n_t, n_in, channel, r0,
                                 row_count, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def beam_power(x: np.ndarray, fmt: str, w: np.ndarray) -> np.ndarray:
    """Per-channel beamformed power sum_t |sum_i conj(w_i) x_i|^2 (int64)."""
    n_ch, n_t, n_in = _shape(x, fmt)
    x = np.ascontiguousarray(x)
    w = np.ascontiguousarray(w, dtype=np.int64)
    if w.shape != (n_in, 2):
        raise ValueError("weights must be int64 [n_in][2]")
    out = np.empty(n_ch, dtype=np.int64)
    rc = lib().xo_beam_power(x.ctypes.data, FORMATS[fmt], n_ch, n_t, n_in, w.ctypes.data,
                             out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def tri_index(n_in: int):
    """Row and column index of every entry of the packed lower triangle."""
    i = np.repeat(np.arange(n_in), np.arange(1, n_in + 1))
    j = np.concatenate([np.arange(k + 1) for k in range(n_in)]) if n_in else np.zeros(0, int)
    return i, j


def hermitian_form(v: np.ndarray, w: np.ndarray) -> np.ndarray:
    """w^H V w for every channel of a packed lower-triangle result.

    v: [n_ch][n_b][2] integer; w: [n_in][2] integer.  Uses
    w^H V w = sum_i |w_i|^2 V_ii + 2 Re sum_{i>j} conj(w_i) V_ij w_j,
    which holds because V is Hermitian.  Exact in int64 for the sizes used.
    """
    v = np.asarray(v)
    n_b = v.shape[1]
    n_in = int((np.sqrt(8 * n_b + 1) - 1) // 2)
    if n_in * (n_in + 1) // 2 != n_b:
        raise ValueError("not a packed triangle")
    i, j = tri_index(n_in)
    wr = np.asarray(w[:, 0], dtype=np.int64)
    wi = np.asarray(w[:, 1], dtype=np.int64)
    # c = conj(w_i) * w_j = (wr_i wr_j + wi_i wi_j) + 1j (wr_i wi_j - wi_i wr_j)
    cr = wr[i] * wr[j] + wi[i] * wi[j]
    ci = wr[i] * wi[j] - wi[i] * wr[j]
    scale = np.where(i == j, 1, 2).astype(np.int64)
    # Re(c * V) = cr Vr - ci Vi
    alpha = scale * cr
    beta = -scale * ci
    vr = v[:, :, 0].astype(np.int64)
    vi = v[:, :, 1].astype(np.int64)
    return vr @ alpha + vi @ beta


# ---------------------------------------------------------------- tiny forms

def _decode_py(x, fmt):
    """Independent pure-Python decoder -> nested lists of (re, im) ints."""
    if fmt == "ci4":
        def nib(v):
            v &= 0xF
            return v - 16 if v >= 8 else v
        return [[[(nib(int(b) >> 4), nib(int(b))) for b in row] for row in ch] for ch in x]
    return [[[(int(s[0]), int(s[1])) for s in row] for row in ch] for ch in x]


def brute_force(x: np.ndarray, fmt: str):
    """Pure-Python loops over Python complex numbers: list[channel][tri] of (re, im).

    Exact for the tiny inputs it is meant for (all partial sums are small
    integers, which float64 represents exactly).
    """
    n_ch, n_t, n_in = _shape(x, fmt)
    d = _decode_py(x, fmt)
    out = []
    for c in range(n_ch):
        acc = []
        for i in range(n_in):
            for j in range(i + 1):
                s = 0j
                for t in range(n_t):
                    xi = complex(*d[c][t][i])
                    xj = complex(*d[c][t][j])
                    s += xi * xj.conjugate()   # exact: small integers in float64
                acc.append((int(s.real), int(s.imag)))
        out.append(acc)
    return out


def matmul_form(x: np.ndarray, fmt: str) -> np.ndarray:
    """Re = A A^T + B B^T, Im = B A^T - A B^T per channel (exact int64 matmul)."""
    n_ch, n_t, n_in = _shape(x, fmt)
    if fmt == "ci4":
        b = x.astype(np.int64)
        hi = (b >> 4) & 0xF
        lo = b & 0xF
        re = np.where(hi >= 8, hi - 16, hi)
        im = np.where(lo >= 8, lo - 16, lo)
    else:
        re = x[..., 0].astype(np.int64)
        im = x[..., 1].astype(np.int64)
    i, j = tri_index(n_in)
    out = np.empty((n_ch, n_baselines(n_in), 2), dtype=np.int64)
    for c in range(n_ch):
        A = re[c].T  # [n_in][n_t]
        B = im[c].T
        vr = A @ A.T + B @ B.T
        vi = B @ A.T - A @ B.T
        out[c, :, 0] = vr[i, j]
        out[c, :, 1] = vi[i, j]
    return out


def corner_turn(packets: np.ndarray, n_fengines: int, inputs_per_feng: int, n_channels: int,
                spectra_per_packet: int, valid: np.ndarray | None = None, out_fmt: str = "ci4") -> np.ndarray:
    """X-stage input from captured F-engine packets.

    packets: uint8 [n_blocks][n_fengines][spectra_per_packet][n_channels][inputs_per_feng],
    one 4+4-bit sample per byte; block b, spectrum s is time b * S + s and
    F-engine f, input j is X-stage input f * J + j.  valid[b][f] == 0 marks a
    lost packet, whose samples are zero.  Returns ci4 bytes
    [n_channels][time][inputs] or, for out_fmt "ci8", int8 [..][inputs][2]
    (real, imaginary) with each nibble sign-extended.
    """
    F, J, C, S = n_fengines, inputs_per_feng, n_channels, spectra_per_packet
    p = np.asarray(packets, dtype=np.uint8).reshape(-1, F, S, C, J)
    B = p.shape[0]
    if valid is not None:
        p = p * (np.asarray(valid).reshape(B, F)[:, :, None, None, None] != 0).astype(np.uint8)
    x = np.ascontiguousarray(p.transpose(3, 0, 2, 1, 4)).reshape(C, B * S, F * J)
    if out_fmt == "ci4":
        return x
    re = x.view(np.int8) >> 4
    im = (x << 4).view(np.int8) >> 4
    return np.stack([re, im], axis=-1).astype(np.int8)


# ---------------------------------------------------------------- F-stage

def pfb_frames(adc: np.ndarray, coeff: np.ndarray, n_points: int, n_taps: int) -> np.ndarray:
    """Polyphase filter-bank front end (Sec. 2.3: the first F-stage operation).

    adc: int8 [n_inputs][n_samples] real samples; coeff: [n_taps * n_points]
    prototype filter.  Spectrum m of an input uses frames m .. m + P - 1 of N
    samples: y_m[j] = sum_p coeff[p N + j] * x[(m + p) N + j] (fp64).
    Returns [n_inputs][n_spectra][N], n_spectra = n_samples // N - P + 1.
    """
    N, P = n_points, n_taps
    x = np.asarray(adc).astype(np.float64)
    n_spec = x.shape[1] // N - P + 1
    if n_spec <= 0:
        return np.zeros((x.shape[0], 0, N))
    frames = x[:, :(n_spec + P - 1) * N].reshape(x.shape[0], n_spec + P - 1, N)
    h = np.asarray(coeff, dtype=np.float64).reshape(P, N)
    y = np.zeros((x.shape[0], n_spec, N))
    for p in range(P):
        y += frames[:, p:p + n_spec, :] * h[p]
    return y


def pfb_spectra(adc: np.ndarray, coeff: np.ndarray, n_points: int, n_taps: int) -> np.ndarray:
    """Channelised spectra: X_m[k] = sum_j y_m[j] exp(-2 pi i j k / N) for the
    N/2 channels k = 0 .. N/2 - 1 of the real input (Sec. 2.3; Sec. 4: an
    8192-point transform of the 200 MHz samples gives 24.4 kHz channels).
    complex128 [n_inputs][n_spectra][N/2]."""
    y = pfb_frames(adc, coeff, n_points, n_taps)
    return np.fft.fft(y, axis=-1)[..., :n_points // 2]


def requantise4(v: np.ndarray) -> np.ndarray:
    """4-bit requantisation of one component (Sec. 2.3): round half to even,
    then saturate to the symmetric range [-7, 7] (int8 result)."""
    return np.clip(np.rint(v), -7, 7).astype(np.int8)


def fstage(adc: np.ndarray, coeff: np.ndarray, gain: np.ndarray, n_points: int, n_taps: int,
           chan_begin: int, n_chan: int, out: str = "ci4") -> np.ndarray:
    """The F-stage feeding the X-stage (Sec. 2.3): PFB spectra, equalisation
    v = gain[a][c - chan_begin] * X_m[c] for the selected channels
    c = chan_begin .. chan_begin + n_chan - 1, then 4+4-bit requantisation.

    out "ci4": uint8 [n_chan][n_spectra][n_inputs], high nibble = real, low
    nibble = imaginary (the X-stage input layout); out "c128": the equalised
    values before requantisation, complex128 [n_chan][n_spectra][n_inputs].
    """
    X = pfb_spectra(adc, coeff, n_points, n_taps)[..., chan_begin:chan_begin + n_chan]
    v = X * np.asarray(gain, dtype=np.float64)[:, None, :]
    v = np.ascontiguousarray(v.transpose(2, 1, 0))
    if out == "c128":
        return v
    re = requantise4(v.real).astype(np.uint8)
    im = requantise4(v.imag).astype(np.uint8)
    return ((re & 0xF) << 4) | (im & 0xF)
