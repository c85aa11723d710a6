"""GPU parity of the HIP X-stage against the CPU oracle, through the C ABI.

Bar: the int8-MFMA path is bit-exact (int64).  The fp16-MFMA and fp32 paths
are exact whenever every fp32 partial sum stays below 2^24 (all CI4 cases
here: |x|^2 <= 128 per sample, N_t <= 131072); for the 8-bit large-N case
their error is measured and bounded (see test_large_n_fp_paths_error_bound).

Small cases are compared element by element; the full-size workloads are
checked on sampled channels (or sampled rows of a channel) that the oracle
computes directly, plus the beam-power identity w^H V w = sum_t |w^H x_t|^2 on
every channel.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1401_8288_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def xc():
    from paper_1401_8288_amd import xcorr
    return xcorr


def run(x, fmt, path, **kw):
    p = xc().Plan(x.shape[2], x.shape[0], fmt, path, **kw)
    out, info = p.accumulate_dump(x)
    torch.cuda.synchronize()
    p.close()
    return out.cpu().numpy(), info


def weights(n_in, seed):
    g = np.random.default_rng(seed)
    w = g.integers(-3, 4, size=(n_in, 2))
    w[(w == 0).all(axis=1)] = (1, 0)
    return w


# ------------------------------------------------------------------ small cases

@pytest.mark.parametrize("path", ["i8", "f16", "f32"])
def test_tiny_workload_all_paths(path):
    w = synth.WORKLOADS["tiny"]
    say("tiny workload", path, w.n_inputs, w.n_channels, w.n_time)
    x = synth.generate(w, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), w.fmt)
    got, info = run(x, w.fmt, path)
    if path == "i8":
        np.testing.assert_array_equal(got, ref)
    else:
        np.testing.assert_array_equal(got, ref.astype(np.float32))
    assert info.samples_accumulated == w.n_time


SHAPES = [  # (n_in, n_ch, n_t): ragged inputs, ragged time, channel groups
    (4, 3, 1), (4, 5, 64), (8, 6, 65), (36, 5, 100), (64, 9, 129), (100, 2, 129),
    (128, 3, 64), (192, 2, 65), (256, 2, 200), (400, 2, 77), (516, 1, 70),
    # input counts that are not a multiple of 4 (rows zero padded for the
    # kernels' loads; 160 and more to 16 for the LDS-DMA kernels)
    (1, 2, 5), (2, 3, 7), (3, 2, 64), (6, 4, 100), (66, 3, 130), (130, 2, 65), (161, 2, 70), (514, 1, 70)]


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("path", ["i8", "f16", "f32"])
def test_ragged_shapes_full_range(fmt, shape, path):
    n_in, n_ch, n_t = shape
    say("ragged", fmt, shape, path)
    x = synth.random_input(n_ch, n_t, n_in, fmt, seed=n_in * 7 + n_t, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), fmt)
    got, _ = run(x, fmt, path)
    if path == "i8":
        np.testing.assert_array_equal(got, ref)
    elif fmt == "ci4":
        np.testing.assert_array_equal(got, ref.astype(np.float32))
    else:
        # 8-bit: exact while partial sums < 2^24 (n_t * 2 * 128^2 < 2^24 here)
        assert n_t * 2 * 128 * 128 < 2 ** 24
        np.testing.assert_array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_launch_modes_give_the_same_result(fmt):
    # persistent or one workgroup per item, XCD-aware or plain order: the
    # same exact sums (both LDS-DMA variants)
    X = xc()
    x = synth.random_input(6, 333, 128, fmt, seed=17, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), fmt)
    for flags in (0, X.FLAG_NO_PERSIST, X.FLAG_NO_XCD_MAP, X.FLAG_NO_PERSIST | X.FLAG_NO_XCD_MAP):
        got, _ = run(x, fmt, "i8", flags=flags)
        np.testing.assert_array_equal(got, ref, err_msg="flags %#x" % flags)


def test_no_xcd_map_gives_the_same_result():
    x = synth.random_input(20, 70, 256, "ci4", seed=3, device=DEV)
    a, _ = run(x, "ci4", "i8")
    b, _ = run(x, "ci4", "i8", flags=xc().FLAG_NO_XCD_MAP)
    np.testing.assert_array_equal(a, b)


def test_repeated_runs_identical():
    # integer results are unique: any race shows up as a difference
    x = synth.random_input(64, 256, 192, "ci4", seed=4, device=DEV)
    a, _ = run(x, "ci4", "i8")
    for _ in range(2):
        b, _ = run(x, "ci4", "i8")
        np.testing.assert_array_equal(a, b)


# ------------------------------------------------------- accumulate / dump protocol

def test_split_accumulation_equals_one_window():
    n_in, n_ch = 128, 6
    x = synth.random_input(n_ch, 2048, n_in, "ci4", seed=5, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), "ci4")
    p = xc().Plan(n_in, n_ch, "ci4", "i8")
    for a, b in ((0, 1), (1, 100), (100, 1000), (1000, 2048)):
        p.accumulate(x[:, a:b].contiguous())
    out, info = p.dump(reset=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    assert (info.samples_accumulated, info.start_sample, info.n_dumps) == (2048, 0, 1)
    # after a reset the next dump without data is zero
    out, info = p.dump(reset=True)
    torch.cuda.synchronize()
    assert not out.cpu().numpy().any()
    assert (info.samples_accumulated, info.start_sample, info.n_dumps) == (0, 2048, 2)
    p.close()


def test_dump_without_reset_keeps_integrating():
    n_in, n_ch = 64, 4
    x1 = synth.random_input(n_ch, 300, n_in, "ci8", seed=6, device=DEV)
    x2 = synth.random_input(n_ch, 200, n_in, "ci8", seed=7, device=DEV)
    r1 = oracle.correlate(x1.cpu().numpy(), "ci8")
    r2 = oracle.correlate(x2.cpu().numpy(), "ci8")
    p = xc().Plan(n_in, n_ch, "ci8", "i8")
    o1, i1 = p.accumulate_dump(x1, reset=False)
    o2, i2 = p.accumulate_dump(x2, reset=False)
    o3, i3 = p.dump(reset=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o1.cpu().numpy(), r1)
    np.testing.assert_array_equal(o2.cpu().numpy(), r1 + r2)
    np.testing.assert_array_equal(o3.cpu().numpy(), r1 + r2)
    assert (i2.samples_accumulated, i3.samples_accumulated) == (500, 500)
    p.close()


@pytest.mark.parametrize("path", ["f16", "f32"])
def test_fp_paths_accumulate_across_calls(path):
    x = synth.random_input(3, 500, 96, "ci4", seed=8, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), "ci4")
    p = xc().Plan(96, 3, "ci4", path)
    p.accumulate(x[:, :123].contiguous())
    out, _ = p.accumulate_dump(x[:, 123:].contiguous())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.astype(np.float32))
    p.close()


@pytest.mark.parametrize("shape", [(36, 3, 100), (128, 2, 129), (400, 1, 77)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("path", ["i8", "f16", "f32"])
def test_ci8_with_minus_128(shape, path):
    # components over the whole int8 range [-128, 127]
    n_in, n_ch, n_t = shape
    say("ci8 -128..127", shape, path)
    x = synth.random_input(n_ch, n_t, n_in, "ci8", seed=n_in + 3 * n_t, lo=-128, hi=127, device=DEV)
    assert int(x.min()) == -128
    ref = oracle.correlate(x.cpu().numpy(), "ci8")
    got, _ = run(x, "ci8", path)
    if path == "i8":
        np.testing.assert_array_equal(got, ref)
    else:
        assert n_t * 2 * 128 * 128 < 2 ** 24
        np.testing.assert_array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("shape", [(64, 3, 1000), (512, 1, 333), (112, 5, 64), (16, 7, 129), (48, 5, 300),
                                   (192, 2, 65), (400, 2, 77)], ids=lambda s: "x".join(map(str, s)))
def test_int8_tile_variants(tile, shape):
    n_in, n_ch, n_t = shape
    say("tile", tile, shape)
    x = synth.random_input(n_ch, n_t, n_in, "ci4", seed=tile + n_in, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), "ci4")
    got, _ = run(x, "ci4", "i8", tile=tile)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("shape", [(6, 3, 100), (36, 2, 129), (99, 2, 70), (514, 1, 65)],
                         ids=lambda s: "x".join(map(str, s)))
def test_dma_tiles_on_padded_rows(tile, shape):
    # an LDS-DMA tile asked for rows that are not a multiple of 16 inputs:
    # each chunk is staged zero padded; int64 and int32 output, and a window
    # split over calls (the second call adds)
    n_in, n_ch, n_t = shape
    say("dma tile on padded rows", tile, shape)
    x = synth.random_input(n_ch, n_t, n_in, "ci4", seed=tile * 7 + n_in, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), "ci4")
    got, _ = run(x, "ci4", "i8", tile=tile)
    np.testing.assert_array_equal(got, ref)
    got32, _ = run(x, "ci4", "i8", tile=tile, flags=xc().FLAG_OUT_I32)
    np.testing.assert_array_equal(got32.astype(np.int64), ref)
    p = xc().Plan(n_in, n_ch, "ci4", "i8", tile=tile)
    p.accumulate(x[:, : n_t // 2].contiguous())
    out, _ = p.accumulate_dump(x[:, n_t // 2:].contiguous())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    p.close()
    if tile == 2:
        x8 = synth.random_input(n_ch, n_t, n_in, "ci8", seed=tile * 5 + n_in, lo=-128, hi=127, device=DEV)
        got, _ = run(x8, "ci8", "i8", tile=tile)
        np.testing.assert_array_equal(got, oracle.correlate(x8.cpu().numpy(), "ci8"))


@pytest.mark.parametrize("tile", [2, 3])
@pytest.mark.parametrize("shape", [(64, 3, 1000), (512, 1, 333), (112, 5, 64), (16, 7, 129), (48, 5, 300),
                                   (192, 2, 65), (400, 2, 77)], ids=lambda s: "x".join(map(str, s)))
def test_int8_tile_variants_8bit(tile, shape):
    # 8-bit samples: the LDS-DMA tile (interleaved rows transposed by 16-bit
    # LDS reads) and the register tile, full value range
    n_in, n_ch, n_t = shape
    say("tile ci8", tile, shape)
    x = synth.random_input(n_ch, n_t, n_in, "ci8", seed=tile + 3 * n_in, lo=-128, hi=127, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), "ci8")
    got, _ = run(x, "ci8", "i8", tile=tile)
    np.testing.assert_array_equal(got, ref)


def test_8bit_dma_plan_over_windows_of_changing_length():
    # windows of growing and shrinking length through one 8-bit LDS-DMA plan
    X = xc()
    p = X.Plan(64, 3, "ci8", "i8", tile=2)
    total = None
    xs = [synth.random_input(3, n_t, 64, "ci8", seed=n_t, device=DEV) for n_t in (100, 700, 300)]
    for x in xs:
        p.accumulate(x)
    out, info = p.dump()
    torch.cuda.synchronize()
    ref = sum(oracle.correlate(x.cpu().numpy(), "ci8") for x in xs)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    assert info.samples_accumulated == 1100
    p.close()


@pytest.mark.parametrize("fmt,re,im,per_sample", [("ci4", -8, -8, 128), ("ci8", -128, -128, 32768),
                                                  ("ci8", 127, -128, 127 * 127 + 128 * 128)])
def test_int32_fold_past_two_to_the_31(fmt, re, im, per_sample):
    # constant worst-case samples for longer than one int32 window: every
    # entry is n_t |x|^2.  The kernel's int32 partial of this sum (scaled by
    # 256 for 4-bit samples, whose nibbles are used as 16 x value) would pass
    # 2^31 - 1 without the 65535-sample fold.
    n_t = 70000
    scale = 256 if fmt == "ci4" else 1
    assert n_t * per_sample * scale > 2 ** 31
    say("fold", fmt, re, im, n_t)
    x = synth.constant_input(2, n_t, 64, fmt, re, im, device=DEV)
    got, _ = run(x, fmt, "i8")
    assert (got[..., 0] == n_t * per_sample).all()
    assert (got[..., 1] == 0).all()


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_int32_accumulator_folds_across_calls(fmt):
    # xcorr_accumulate of an int64 plan adds into an int32 accumulator that
    # is folded into the int64 one before it passes the fold bound: calls of
    # uneven length that cross the bound several times (within a call and
    # between calls), dumps without reset in between, a tile dump with
    # restart, then a fused accumulate_dump; worst-case constant samples
    # make every int32 partial reach its limit
    say("int32 accumulator folds", fmt)
    X = xc()
    lo = -8 if fmt == "ci4" else -128
    n_in, n_ch = 72, 3
    lens = [40000, 30000, 70000, 1, 65535, 20000]
    xs = [synth.constant_input(n_ch, n, n_in, fmt, lo, lo, device=DEV) if k % 2 == 0 else
          synth.random_input(n_ch, n, n_in, fmt, seed=300 + k, device=DEV) for k, n in enumerate(lens)]
    refs = [oracle.correlate(x.cpu().numpy(), fmt) for x in xs]
    p = X.Plan(n_in, n_ch, fmt, "i8")
    total = np.zeros_like(refs[0])
    for k, (x, r) in enumerate(zip(xs[:-1], refs[:-1])):
        p.accumulate(x)
        total = total + r
        if k in (1, 3):
            out, info = p.dump(reset=False)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), total, err_msg="dump after call %d" % k)
            assert info.samples_accumulated == sum(lens[:k + 1])
    # restart tile (1, 0) only: its baselines start again from zero
    sel = [0, 1, 0]
    out = p.new_output()
    out.fill_(-1)
    p.dump_tiles(out, sel, reset=True)
    torch.cuda.synchronize()
    i, j = oracle.tri_index(n_in)
    in_tile = (i >= 64) & (j < 64)
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[:, in_tile], total[:, in_tile])
    assert (got[:, ~in_tile] == -1).all()
    total[:, in_tile] = 0
    out, info = p.accumulate_dump(xs[-1])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), total + refs[-1])
    p.close()


def test_error_paths_enqueue_nothing():
    X = xc()
    x = synth.random_input(2, 64, 64, "ci4", seed=9, device=DEV)
    p = X.Plan(64, 2, "ci4", "i8")
    out = p.new_output()
    base = int(x.data_ptr())
    import ctypes
    assert X.lib.xcorr_accumulate(p._h, ctypes.c_void_p(base + 1), 64) == -1   # misaligned
    assert X.lib.xcorr_accumulate(p._h, None, 64) == -1
    assert X.lib.xcorr_accumulate(p._h, ctypes.c_void_p(base), -1) == -1
    assert X.lib.xcorr_accumulate(p._h, None, 0) == 0                          # no-op
    assert X.lib.xcorr_dump(p._h, None, 1, None) == -1
    o, info = p.dump()
    torch.cuda.synchronize()
    assert not o.cpu().numpy().any() and info.samples_accumulated == 0
    with pytest.raises(ValueError):
        p.accumulate(x[:, :, :32])
    q = p.query()
    assert q.fold_bound == 65535 and q.output_bytes == out.numel() * 8
    p.close()


# ------------------------------------------------------------ full-size workloads

def _beam_check(x_np, fmt, out, seeds=(101, 102, 103)):
    for s in seeds:
        w = weights(x_np.shape[2], s)
        np.testing.assert_array_equal(oracle.hermitian_form(out, w), oracle.beam_power(x_np, fmt, w))


def test_paper_workload_full_size():
    w = synth.WORKLOADS["paper"]
    say("paper workload", w)
    x = synth.generate(w, device=DEV)
    x_np = x.cpu().numpy()
    got, _ = run(x, w.fmt, "i8")
    ch = np.random.default_rng(21).choice(w.n_channels, 24, replace=False)
    for c in sorted(ch):
        np.testing.assert_array_equal(got[c], oracle.correlate(x_np, w.fmt, (int(c), 1))[0])
    _beam_check(x_np, w.fmt, got)
    for path in ("f16", "f32"):
        f, _ = run(x, w.fmt, path)
        for c in sorted(ch)[:8]:
            np.testing.assert_array_equal(
                f[c], oracle.correlate(x_np, w.fmt, (int(c), 1))[0].astype(np.float32))


def test_paper_exact_tone_closed_form():
    w = synth.WORKLOADS["paper_exact"]
    say("paper exact tone", w)
    x = synth.generate(w, device=DEV)
    got, _ = run(x, w.fmt, "i8")
    qr, qi = synth.exact_tone_amplitudes(w)
    q = qr.numpy() + 1j * qi.numpy()
    i, j = oracle.tri_index(w.n_inputs)
    exp = w.n_time * q[:, i] * np.conj(q[:, j])
    np.testing.assert_array_equal(got[..., 0], exp.real.astype(np.int64))
    np.testing.assert_array_equal(got[..., 1], exp.imag.astype(np.int64))


@pytest.fixture(scope="module")
def lwa():
    w = synth.WORKLOADS["lwa"]
    say("generating lwa workload", w)
    x = synth.generate(w, device=DEV)
    torch.cuda.synchronize()
    yield w, x
    del x
    torch.cuda.empty_cache()


def test_lwa_workload_full_size_int8(lwa):
    w, x = lwa
    say("lwa int8 accumulate_dump")
    got, info = run(x, w.fmt, "i8")
    assert info.samples_accumulated == w.n_time
    x_np = x.cpu().numpy()
    ch = sorted(np.random.default_rng(31).choice(w.n_channels, 6, replace=False))
    for c in list(ch) + [0, w.n_channels - 1]:
        np.testing.assert_array_equal(got[c], oracle.correlate(x_np, w.fmt, (int(c), 1))[0])
    say("lwa beam-power identity on all channels")
    _beam_check(x_np, w.fmt, got, seeds=(201, 202))
    del got
    # the configuration the benchmark times: int32 (re, im) output, the
    # persistent LDS-DMA kernel writing the dump directly
    say("lwa int8 accumulate_dump, int32 output")
    got32, info = run(x, w.fmt, "i8", flags=xc().FLAG_OUT_I32)
    assert info.samples_accumulated == w.n_time and got32.dtype == np.int32
    for c in list(ch) + [0, 1, w.n_channels - 1]:
        np.testing.assert_array_equal(got32[c].astype(np.int64), oracle.correlate(x_np, w.fmt, (int(c), 1))[0])
    say("lwa int32 output: beam-power identity on all channels")
    _beam_check(x_np, w.fmt, got32, seeds=(203, 204))


def test_lwa_workload_fp16_exact_on_sampled_channels(lwa):
    w, x = lwa
    got, _ = run(x, w.fmt, "f16")
    x_np = x.cpu().numpy()
    for c in (0, 1777, w.n_channels - 1):
        np.testing.assert_array_equal(
            got[c], oracle.correlate(x_np, w.fmt, (c, 1))[0].astype(np.float32))


def test_large_n_workload_sampled_rows():
    w = synth.WORKLOADS["large_n"]
    say("large-N workload", w)
    x = synth.generate(w, device=DEV)
    got, _ = run(x, w.fmt, "i8")
    x_np = x.cpu().numpy()
    for c in (0, 137, w.n_channels - 1):
        for r0, rc in ((0, 4), (1023, 3), (2040, 8)):
            a = r0 * (r0 + 1) // 2
            b = (r0 + rc) * (r0 + rc + 1) // 2
            np.testing.assert_array_equal(got[c, a:b], oracle.correlate_rows(x_np, w.fmt, c, r0, rc))
    say("large-N beam-power identity on all channels")
    _beam_check(x_np, w.fmt, got, seeds=(301,))
    del got
    # the configuration the benchmark's large-N line times: int32 output
    say("large-N int32 output")
    got32, info = run(x, w.fmt, "i8", flags=xc().FLAG_OUT_I32)
    assert info.samples_accumulated == w.n_time and got32.dtype == np.int32
    for c in (0, 99, w.n_channels - 1):
        for r0, rc in ((0, 3), (777, 2), (2045, 3)):
            a = r0 * (r0 + 1) // 2
            b = (r0 + rc) * (r0 + rc + 1) // 2
            np.testing.assert_array_equal(got32[c, a:b].astype(np.int64), oracle.correlate_rows(x_np, w.fmt, c, r0, rc))
    _beam_check(x_np, w.fmt, got32, seeds=(302,))
    del x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("path", ["f16", "f32"])
def test_large_n_fp_paths_error_bound(path):
    # 8-bit Gaussian (sigma 32) over 8192 samples: autocorrelations reach
    # ~2^24, so fp32 accumulation rounds.  Each partial sum is rounded at
    # most once per added term with relative error 2^-24, so the error of an
    # entry is below n_t * 2^-24 * sum_t |x_i x_j| <= n_t * 2^-24 * sqrt(V_ii V_jj).
    w = synth.scaled(synth.WORKLOADS["large_n"], n_channels=4)
    say("large-N fp error", path)
    x = synth.generate(w, device=DEV)
    got, _ = run(x, w.fmt, path)
    x_np = x.cpu().numpy()
    ref = oracle.correlate(x_np, w.fmt, (0, 1))[0]
    i, j = oracle.tri_index(w.n_inputs)
    k = np.arange(w.n_inputs)
    auto = ref[k * (k + 1) // 2 + k, 0].astype(np.float64)
    scale = np.sqrt(auto[i] * auto[j])
    err = np.abs(got[0].astype(np.float64) - ref.astype(np.float64)).max(axis=1)
    bound = w.n_time * 2.0 ** -24 * scale
    say("%s: max abs err %.1f, max err / sqrt(Vii Vjj) %.3e" % (path, err.max(), (err / scale).max()))
    assert (err <= bound).all()


@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_many_inputs_one_channel(fmt):
    # 4096 inputs: 64 row blocks, 2080 tiles per channel (8.4 M baselines)
    say("many inputs", fmt)
    x = synth.random_input(1, 70, 4096, fmt, seed=41, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), fmt)
    got, info = run(x, fmt, "i8")
    np.testing.assert_array_equal(got, ref)
    got32, _ = run(x, fmt, "i8", flags=xc().FLAG_OUT_I32)
    np.testing.assert_array_equal(got32.astype(np.int64), ref)


@pytest.mark.parametrize("fmt,tile", [("ci4", 0), ("ci4", 1), ("ci4", 3), ("ci8", 0), ("ci8", 3)])
@pytest.mark.parametrize("shape", [(128, 1, 200), (192, 3, 129), (320, 5, 64), (256, 2, 300), (448, 7, 70),
                                   (100, 3, 90)], ids=lambda s: "x".join(map(str, s)))
def test_int8_items_pair_diagonals_of_two_channels(fmt, tile, shape):
    # int8 plans put the diagonal tiles of two channels into one work item;
    # odd channel counts leave the second channel of the last group empty,
    # odd row-block counts end with a single-block diagonal item
    n_in, n_ch, n_t = shape
    if tile == 1 and n_in % 16:
        pytest.skip("the LDS-DMA tiles need n_inputs % 16 == 0")
    say("paired diagonal items", fmt, shape, "tile", tile)
    x = synth.random_input(n_ch, n_t, n_in, fmt, seed=n_in + n_ch, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), fmt)
    p = xc().Plan(n_in, n_ch, fmt, "i8", tile=tile)
    assert p.query().channels_per_group == 2
    p.close()
    got, _ = run(x, fmt, "i8", tile=tile)
    np.testing.assert_array_equal(got, ref)
    got32, _ = run(x, fmt, "i8", tile=tile, flags=xc().FLAG_OUT_I32)
    np.testing.assert_array_equal(got32.astype(np.int64), ref)
    # launches that add to the accumulator take the single-channel items,
    # launches that write their result the paired ones: mix both in a window
    k = n_t // 3
    p = xc().Plan(n_in, n_ch, fmt, "i8", tile=tile)
    p.accumulate(x[:, :k].contiguous())
    p.accumulate(x[:, k:2 * k].contiguous())
    out, info = p.accumulate_dump(x[:, 2 * k:].contiguous())
    torch.cuda.synchronize()
    assert info.samples_accumulated == n_t
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    out, _ = p.accumulate_dump(x)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    p.close()


@pytest.mark.parametrize("n_in,n_ch,n_t", [(16, 40, 70000), (32, 33, 300), (64, 128, 129), (2048, 2, 200)])
def test_8bit_dma_many_channels_and_chunks(n_in, n_ch, n_t):
    # the 8-bit LDS-DMA kernel over many channels (odd counts leave the
    # last channel group half empty), over two chunks (70000 samples pass
    # the 65535-sample fold bound; the second chunk adds to the first) and
    # over 32 row blocks
    say("8-bit dma channels and chunks", n_in, n_ch, n_t)
    x = synth.random_input(n_ch, n_t, n_in, "ci8", seed=n_ch, device=DEV)
    ref = oracle.correlate(x.cpu().numpy(), "ci8")
    got, info = run(x, "ci8", "i8")
    assert info.samples_accumulated == n_t
    np.testing.assert_array_equal(got, ref)
    p = xc().Plan(n_in, n_ch, "ci8", "i8")
    k = n_t // 2
    p.accumulate(x[:, :k].contiguous())
    out, _ = p.accumulate_dump(x[:, k:].contiguous())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    p.close()


def test_clock_probe_reports_a_plausible_shader_clock():
    # measurement support: one wave waits 2 ms of wall-clock time; the
    # shader clock it reports lies within what the chip can run at
    X = xc()
    probe = X.ClockProbe(DEV)
    assert probe.wall_khz > 0
    s = torch.cuda.Stream(device=DEV)
    probe.start(2.0, s)
    torch.cuda.synchronize()
    r0, r1, c0, c1 = (int(v) for v in probe.buf.cpu())
    assert (r1 - r0) >= 2.0 * probe.wall_khz
    mhz = probe.mhz()
    say("shader clock %.0f MHz (wall clock %d kHz)" % (mhz, probe.wall_khz))
    assert 100.0 < mhz < 3000.0
