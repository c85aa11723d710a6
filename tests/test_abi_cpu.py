"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad descriptors before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xcorr.h")
LIB = os.path.join(ROOT, "paper_1401_8288_amd", "libxcorr.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xcorr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1401_8288_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("xcorr_plan", "xcorr_accumulate", "xcorr_dump", "xcorr_accumulate_dump",
              "xcorr_query", "xcorr_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_exports_match_header():
    import torch  # noqa: F401  (the binding loads after torch)
    from paper_1401_8288_amd import xcorr
    assert sorted(xcorr.EXPORTS) == declared()


def test_version_and_strerror(lib):
    lib.xcorr_version.restype = ctypes.c_int32
    assert lib.xcorr_version() >= 100
    lib.xcorr_strerror.restype = ctypes.c_char_p
    lib.xcorr_strerror.argtypes = [ctypes.c_int]
    assert lib.xcorr_strerror(0) == b"ok"
    assert lib.xcorr_strerror(-1) == b"invalid argument"
    assert lib.xcorr_strerror(-99) == b"unknown status"


def _desc(**kw):
    import torch  # noqa: F401
    from paper_1401_8288_amd import xcorr
    d = dict(n_inputs=64, n_channels=4, fmt="ci4", path="i8")
    d.update(kw)
    return xcorr.make_desc(**d)


@pytest.mark.parametrize("kw,status", [
    (dict(n_inputs=0), -1), (dict(n_channels=0), -1), (dict(n_inputs=-4), -1),
    (dict(n_inputs=40000), -6),
    (dict(flags=0x100), -1), (dict(tile=7), -1),
    (dict(tile=1, fmt="ci8"), -6),      # DMA8 takes 4-bit samples only
    (dict(tile=4), -1),
    (dict(tile=3, path="f32"), -6)])    # tile variants exist for the int8 path only
def test_bad_descriptors_rejected_before_any_device_call(kw, status):
    from paper_1401_8288_amd import xcorr
    h = ctypes.c_void_p()
    d = _desc(**kw)
    assert xcorr.lib.xcorr_plan(ctypes.byref(h), ctypes.byref(d)) == status
    assert h.value is None
    assert xcorr.lib.xcorr_last_error()


@pytest.mark.parametrize("n_in,fmt", [(1, "ci4"), (2, "ci4"), (6, "ci4"), (66, "ci4"), (130, "ci4"),
                                      (514, "ci4"), (1, "ci8"), (5, "ci8"), (129, "ci8")])
def test_every_input_count_is_accepted(n_in, fmt):
    # rows of any width are zero padded to what the kernels read; the plan's
    # accumulators are those of n_in inputs (the padding is a staging buffer
    # grown on use, outside the plan's bytes)
    from paper_1401_8288_amd import xcorr
    nb = n_in * (n_in + 1) // 2
    for path in ("i8", "f16", "f32"):
        acc = nb * 7 * 2 * (8 + 4 if path == "i8" else 4)
        assert acc <= xcorr.plan_bytes(n_in, 7, fmt, path) < acc + 65536


def test_bad_enums_rejected():
    from paper_1401_8288_amd import xcorr
    d = _desc()
    d.format = 7
    h = ctypes.c_void_p()
    assert xcorr.lib.xcorr_plan(ctypes.byref(h), ctypes.byref(d)) == -1
    d = _desc()
    d.path = 9
    assert xcorr.lib.xcorr_plan(ctypes.byref(h), ctypes.byref(d)) == -1
    assert xcorr.lib.xcorr_plan(None, ctypes.byref(_desc())) == -1
    assert xcorr.lib.xcorr_plan(ctypes.byref(h), None) == -1


def test_calls_on_invalid_handles():
    from paper_1401_8288_amd import xcorr
    bogus = ctypes.c_void_p(0x1234)
    assert xcorr.lib.xcorr_accumulate(bogus, None, 0) == -4
    assert xcorr.lib.xcorr_dump(bogus, None, 1, None) == -4
    assert xcorr.lib.xcorr_accumulate_dump(bogus, None, 0, None, 1, None) == -4
    assert xcorr.lib.xcorr_query(bogus, None) == -4
    assert xcorr.lib.xcorr_destroy(None) == -4
    assert xcorr.lib.xcorr_destroy(bogus) == -4


@pytest.mark.parametrize("n_in,fmt,path", [(64, "ci4", "i8"), (512, "ci4", "i8"),
                                           (2048, "ci8", "i8"), (512, "ci4", "f32")])
def test_plan_bytes_is_the_accumulator(n_in, fmt, path):
    from paper_1401_8288_amd import xcorr
    nb = n_in * (n_in + 1) // 2
    got = xcorr.plan_bytes(n_in, 4096, fmt, path)
    acc = nb * 4096 * 2 * (8 if path == "i8" else 4)
    if path == "i8":
        acc += nb * 4096 * 2 * 4        # the int32 accumulator beside the int64 one
    assert acc <= got < acc + 65536


def test_batch_and_graph_calls_on_invalid_handles():
    from paper_1401_8288_amd import xcorr
    L = xcorr.lib
    bogus = ctypes.c_void_p(0x1234)
    h = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 1)(0x1234)
    assert L.xcorr_batch_create(None, plans, 1, None) == -1
    assert L.xcorr_batch_create(ctypes.byref(h), None, 1, None) == -1
    assert L.xcorr_batch_create(ctypes.byref(h), plans, 0, None) == -1
    assert L.xcorr_batch_create(ctypes.byref(h), plans, 65, None) == -1
    assert L.xcorr_batch_create(ctypes.byref(h), plans, 1, None) == -4   # not a plan
    assert h.value is None
    assert L.xcorr_batch_run(bogus, None, None, None, None, None) == -4
    assert L.xcorr_batch_get_config(bogus, None) == -4
    assert L.xcorr_batch_set_config(bogus, None) == -4
    assert L.xcorr_batch_autotune(bogus, None, None, 1, None, None) == -4
    assert L.xcorr_batch_capture(bogus, None, None, None, None) == -4
    assert L.xcorr_graph_launch(bogus) == -4
    assert L.xcorr_graph_destroy(bogus) == -4
    assert L.xcorr_graph_destroy(None) == -4
    assert L.xcorr_batch_destroy(bogus) == -4
    assert L.xcorr_batch_destroy(None) == -4


def test_server_calls_on_invalid_handles_and_arguments():
    from paper_1401_8288_amd import xcorr
    L = xcorr.lib
    bogus = ctypes.c_void_p(0x1234)
    h = ctypes.c_void_p()
    for budget, streams, inflight in ((0, 4, 2), (1 << 30, 0, 2), (1 << 30, 65, 2), (1 << 30, 4, 0), (1 << 30, 4, 9)):
        d = xcorr.ServerDesc(budget, streams, inflight, None, None)
        assert L.xcorr_server_create(ctypes.byref(h), ctypes.byref(d)) == -1
        assert h.value is None
    assert L.xcorr_server_create(None, None) == -1
    sid = ctypes.c_int32(0)
    t = ctypes.c_int64(0)
    done = ctypes.c_int32(0)
    assert L.xcorr_server_open(bogus, None, ctypes.byref(sid)) == -4
    assert L.xcorr_server_submit(bogus, 1, None, 1, None, ctypes.byref(t)) == -4
    assert L.xcorr_server_poll(bogus, 1, ctypes.byref(done), None, None) == -4
    assert L.xcorr_server_wait(bogus, 1, None, None) == -4
    assert L.xcorr_server_close(bogus, 1) == -4
    assert L.xcorr_server_set_deadline(bogus, 1, 1e-3) == -4
    assert L.xcorr_server_query(bogus, None) == -4
    assert L.xcorr_server_destroy(bogus) == -4
    assert L.xcorr_server_destroy(None) == -4


def test_accumulate_variants_on_invalid_handles():
    from paper_1401_8288_amd import xcorr
    L = xcorr.lib
    bogus = ctypes.c_void_p(0x1234)
    plans = (ctypes.c_void_p * 2)(0x1234, 0x5678)
    sel = (ctypes.c_uint8 * 1)(1)
    assert L.xcorr_dump_tiles(bogus, None, ctypes.cast(sel, ctypes.c_void_p), 1, None) == -4
    assert L.xcorr_accumulate_gated(None, 1, None, 0, None) == -1
    assert L.xcorr_accumulate_gated(plans, 0, None, 0, None) == -1
    assert L.xcorr_accumulate_gated(plans, 65, None, 0, None) == -1
    assert L.xcorr_accumulate_gated(plans, 2, None, 0, None) == -4
    lay = xcorr.PacketLayout(0, 1, 4, 1, 1)
    assert L.xcorr_corner_turn(None, None, ctypes.byref(lay), 0, None, None) == -1
    lay = xcorr.PacketLayout(1, 1, 6, 1, 1)
    assert L.xcorr_corner_turn(None, None, ctypes.byref(lay), 0, None, None) == -6
    assert L.xcorr_corner_turn(None, None, None, 0, None, None) == -1


def test_fstage_argument_checks():
    from paper_1401_8288_amd import xcorr
    L = xcorr.lib
    n = ctypes.c_int64(-1)

    def call(d, stride=16384, n_samples=16384):
        return L.xcorr_fstage(ctypes.byref(d) if d is not None else None, None, stride, n_samples,
                              None, None, None, None, ctypes.byref(n), None)

    ok = dict(n_inputs=4, n_points=8192, n_taps=2, chan_begin=0, n_chan=16, out_kind=0)
    assert call(None) == -1
    assert call(xcorr.FstageDesc(**dict(ok, n_points=4096))) == -6
    assert call(xcorr.FstageDesc(**dict(ok, n_taps=3))) == -6
    assert call(xcorr.FstageDesc(**dict(ok, chan_begin=4090))) == -1
    assert call(xcorr.FstageDesc(**dict(ok, n_chan=0))) == -1
    assert call(xcorr.FstageDesc(**dict(ok, out_kind=7))) == -1
    assert call(xcorr.FstageDesc(**ok), stride=16383, n_samples=100) == -1      # odd stride
    assert call(xcorr.FstageDesc(**ok), stride=100, n_samples=16384) == -1      # stride < samples
    # fewer than P frames: no spectrum, nothing touched, pointers not needed
    assert call(xcorr.FstageDesc(**ok), n_samples=16383) == 0 and n.value == 0
    # a full spectrum needs the device buffers
    assert call(xcorr.FstageDesc(**ok)) == -1 and n.value == 1
    nb = ctypes.c_size_t(0)
    assert L.xcorr_fstage_work_bytes(ctypes.byref(xcorr.FstageDesc(**dict(ok, chan_begin=5, n_chan=20))),
                                     3 * 8192, ctypes.byref(nb)) == 0
    assert nb.value == 4 * 2 * 32                     # channels 5..24 -> rows of 0..31
    assert L.xcorr_fstage_work_bytes(ctypes.byref(xcorr.FstageDesc(**dict(ok, out_kind=1))),
                                     3 * 8192, ctypes.byref(nb)) == 0 and nb.value == 0


def test_int32_output_flag_checks():
    from paper_1401_8288_amd import xcorr
    full = xcorr.plan_bytes(512, 64, "ci4", "i8")
    half = xcorr.plan_bytes(512, 64, "ci4", "i8", flags=xcorr.FLAG_OUT_I32)
    nb = 512 * 513 // 2 * 64 * 2
    assert full - half == nb * 8                     # int32 pairs only, not int64 + int32
    for path, tile in (("f16", 0), ("f32", 0)):
        with pytest.raises(xcorr.XcorrError) as e:
            xcorr.plan_bytes(512, 64, "ci4", path, flags=xcorr.FLAG_OUT_I32, tile=tile)
        assert e.value.status == -6


def test_clock_probe_argument_checks():
    from paper_1401_8288_amd import xcorr
    L = xcorr.lib
    khz = ctypes.c_int32(0)
    assert L.xcorr_clock_probe(None, 100, ctypes.byref(khz), None) == -1
    assert L.xcorr_clock_probe(ctypes.c_void_p(0x1004), 100, None, None) == -1     # misaligned
    assert L.xcorr_clock_probe(ctypes.c_void_p(0x1000), 0, None, None) == -1
    assert L.xcorr_clock_probe(ctypes.c_void_p(0x1000), 1 << 32, None, None) == -1


def test_noalloc_argument_checks_before_any_device_call():
    from paper_1401_8288_amd import xcorr
    L = xcorr.lib
    p = ctypes.c_void_p(0x1000)
    assert L.xcorr_correlate_noalloc(None, p, 64, p) == -1
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc(path="f32")), p, 64, p) == -6
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc(n_inputs=6)), p, 64, p) == -6
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc(tile=1)), p, 64, p) == -6
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc(flags=0x100)), p, 64, p) == -1
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc()), p, 0, p) == -1           # empty window
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc()), p, 65536, p) == -1       # past the fold bound
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc()), None, 64, p) == -1
    assert L.xcorr_correlate_noalloc(ctypes.byref(_desc()), ctypes.c_void_p(0x1008), 64, p) == -1
