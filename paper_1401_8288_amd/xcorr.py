"""Python binding of libxcorr (include/xcorr.h): argument marshalling only.

Every step of the X-stage runs in the HIP library; this module checks tensor
shapes, passes device pointers and the current torch stream across the C ABI
and turns status codes into exceptions.  torch is imported first so that the
library binds to the HIP runtime torch has already loaded.  There is no
fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxcorr.so")

CI4, CI8 = 0, 1
PATH_I8, PATH_F16, PATH_F32 = 0, 1, 2
FLAG_NO_XCD_MAP = 0x2
FLAG_NO_PERSIST = 0x4
FLAG_OUT_I32 = 0x8
TILE_DEFAULT, TILE_DMA8, TILE_DMA4, TILE_REGS = 0, 1, 2, 3

FORMATS = {"ci4": CI4, "ci8": CI8}
PATHS = {"i8": PATH_I8, "f16": PATH_F16, "f32": PATH_F32}

EXPORTS = ("xcorr_plan", "xcorr_accumulate", "xcorr_dump", "xcorr_accumulate_dump",
           "xcorr_query", "xcorr_plan_bytes", "xcorr_destroy", "xcorr_strerror",
           "xcorr_last_error", "xcorr_version",
           "xcorr_batch_create", "xcorr_batch_run", "xcorr_batch_get_config",
           "xcorr_batch_set_config", "xcorr_batch_autotune", "xcorr_batch_capture",
           "xcorr_graph_launch", "xcorr_graph_destroy", "xcorr_batch_destroy",
           "xcorr_server_create", "xcorr_server_open", "xcorr_server_submit", "xcorr_server_poll",
           "xcorr_server_wait", "xcorr_server_close", "xcorr_server_query", "xcorr_server_destroy",
           "xcorr_corner_turn", "xcorr_dump_tiles", "xcorr_accumulate_gated", "xcorr_fstage",
           "xcorr_fstage_work_bytes", "xcorr_clock_probe", "xcorr_correlate_noalloc",
           "xcorr_server_set_deadline")


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("format", ctypes.c_int32), ("path", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("tile", ctypes.c_int32)]


class DumpInfo(ctypes.Structure):
    _fields_ = [("samples_accumulated", ctypes.c_int64), ("start_sample", ctypes.c_int64),
                ("n_dumps", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_size_t), ("output_bytes", ctypes.c_size_t),
                ("input_bytes_per_sample", ctypes.c_size_t), ("fold_bound", ctypes.c_int64),
                ("tile", ctypes.c_int32), ("work_items", ctypes.c_int32),
                ("items_per_group", ctypes.c_int32), ("channels_per_group", ctypes.c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("grid", ctypes.c_int32), ("balance", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"tile": self.tile, "grid": self.grid, "balance": self.balance}


class ServerDesc(ctypes.Structure):
    _fields_ = [("device_budget", ctypes.c_size_t), ("max_streams", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("stream", ctypes.c_void_p), ("tune_path", ctypes.c_char_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("windows_done", ctypes.c_int64), ("launches", ctypes.c_int64), ("cmac", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("latency_p50_ms", ctypes.c_double),
                ("latency_p99_ms", ctypes.c_double), ("latency_max_ms", ctypes.c_double),
                ("mean_batch", ctypes.c_double), ("streams_admitted", ctypes.c_int32),
                ("streams_waiting", ctypes.c_int32), ("device_bytes", ctypes.c_size_t),
                ("mixes_tuned", ctypes.c_int32), ("mixes_tuning", ctypes.c_int32),
                ("deadline_misses", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PacketLayout(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("n_fengines", ctypes.c_int32),
                ("inputs_per_feng", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("spectra_per_packet", ctypes.c_int32)]


class FstageDesc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_points", ctypes.c_int32), ("n_taps", ctypes.c_int32),
                ("chan_begin", ctypes.c_int32), ("n_chan", ctypes.c_int32), ("out_kind", ctypes.c_int32)]


FSTAGE_CI4, FSTAGE_F32 = 0, 1


class XcorrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("xcorr status %d: %s" % (status, message))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libxcorr.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1401_8288_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.xcorr_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc)]
    L.xcorr_accumulate.argtypes = [vp, vp, i64]
    L.xcorr_dump.argtypes = [vp, vp, i32, ctypes.POINTER(DumpInfo)]
    L.xcorr_accumulate_dump.argtypes = [vp, vp, i64, vp, i32, ctypes.POINTER(DumpInfo)]
    L.xcorr_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.xcorr_plan_bytes.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_size_t)]
    L.xcorr_destroy.argtypes = [vp]
    L.xcorr_strerror.argtypes = [i32]
    L.xcorr_strerror.restype = ctypes.c_char_p
    L.xcorr_last_error.restype = ctypes.c_char_p
    L.xcorr_version.restype = ctypes.c_int32
    P = ctypes.POINTER
    L.xcorr_batch_create.argtypes = [P(vp), P(vp), i32, vp]
    L.xcorr_batch_run.argtypes = [vp, P(vp), P(i64), P(vp), P(ctypes.c_int32), P(DumpInfo)]
    L.xcorr_batch_get_config.argtypes = [vp, P(BatchConfig)]
    L.xcorr_batch_set_config.argtypes = [vp, P(BatchConfig)]
    L.xcorr_batch_autotune.argtypes = [vp, P(vp), P(i64), i32, P(BatchConfig), P(ctypes.c_float)]
    L.xcorr_batch_capture.argtypes = [vp, P(vp), P(i64), P(vp), P(vp)]
    L.xcorr_graph_launch.argtypes = [vp]
    L.xcorr_graph_destroy.argtypes = [vp]
    L.xcorr_batch_destroy.argtypes = [vp]
    L.xcorr_server_create.argtypes = [P(vp), P(ServerDesc)]
    L.xcorr_server_open.argtypes = [vp, P(PlanDesc), P(ctypes.c_int32)]
    L.xcorr_server_submit.argtypes = [vp, ctypes.c_int32, vp, i64, vp, P(i64)]
    L.xcorr_server_poll.argtypes = [vp, i64, P(ctypes.c_int32), P(DumpInfo), P(ctypes.c_double)]
    L.xcorr_server_wait.argtypes = [vp, i64, P(DumpInfo), P(ctypes.c_double)]
    L.xcorr_server_close.argtypes = [vp, ctypes.c_int32]
    L.xcorr_server_set_deadline.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    L.xcorr_server_query.argtypes = [vp, P(ServerStats)]
    L.xcorr_server_destroy.argtypes = [vp]
    L.xcorr_corner_turn.argtypes = [vp, vp, P(PacketLayout), i32, vp, vp]
    L.xcorr_dump_tiles.argtypes = [vp, vp, vp, i32, P(DumpInfo)]
    L.xcorr_accumulate_gated.argtypes = [P(vp), i32, vp, i64, vp]
    L.xcorr_fstage.argtypes = [P(FstageDesc), vp, i64, i64, vp, vp, vp, vp, P(i64), vp]
    L.xcorr_fstage_work_bytes.argtypes = [P(FstageDesc), i64, P(ctypes.c_size_t)]
    L.xcorr_clock_probe.argtypes = [vp, i64, P(ctypes.c_int32), vp]
    L.xcorr_correlate_noalloc.argtypes = [P(PlanDesc), vp, i64, vp]
    for name in EXPORTS:
        if name not in ("xcorr_strerror", "xcorr_last_error", "xcorr_version"):
            getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(status: int):
    if status != 0:
        raise XcorrError(status, lib.xcorr_last_error().decode())


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def make_desc(n_inputs, n_channels, fmt="ci4", path="i8", stream=None, flags=0, tile=0,
              stream_ptr: int | None = None) -> PlanDesc:
    sp = stream_ptr if stream_ptr is not None else (
        int(stream.cuda_stream) if stream is not None else 0)
    return PlanDesc(int(n_inputs), int(n_channels), FORMATS[fmt], PATHS[path],
                    ctypes.c_void_p(sp), int(flags), int(tile))


def plan_bytes(n_inputs, n_channels, fmt="ci4", path="i8", flags=0, tile=0) -> int:
    out = ctypes.c_size_t(0)
    _check(lib.xcorr_plan_bytes(ctypes.byref(make_desc(n_inputs, n_channels, fmt, path, flags=flags, tile=tile)),
                                ctypes.byref(out)))
    return int(out.value)


@dataclass
class Dump:
    samples_accumulated: int
    start_sample: int
    n_dumps: int


class Plan:
    """One X-stage plan: device accumulators for n_channels x n_inputs.

    Calls are enqueued on `stream` (default: torch's current stream at plan
    creation) and return without waiting.
    """

    def __init__(self, n_inputs: int, n_channels: int, fmt: str = "ci4", path: str = "i8",
                 stream: torch.cuda.Stream | None = None, flags: int = 0, tile: int = 0):
        self.n_inputs, self.n_channels, self.fmt, self.path = n_inputs, n_channels, fmt, path
        self.out32 = bool(flags & FLAG_OUT_I32)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        desc = make_desc(n_inputs, n_channels, fmt, path, self.stream, flags, tile)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.xcorr_plan(ctypes.byref(h), ctypes.byref(desc)))
        self._h = h
        self.n_baselines = n_inputs * (n_inputs + 1) // 2

    # ---------------------------------------------------------------- helpers
    @property
    def out_dtype(self):
        if self.path != "i8":
            return torch.float32
        return torch.int32 if self.out32 else torch.int64

    def out_shape(self):
        return (self.n_channels, self.n_baselines, 2)

    def new_output(self) -> torch.Tensor:
        return torch.empty(self.out_shape(), dtype=self.out_dtype, device=self.device)

    def _check_input(self, x: torch.Tensor) -> int:
        if not isinstance(x, torch.Tensor) or x.device != self.device:
            raise ValueError("input must be a tensor on %s" % self.device)
        if not x.is_contiguous():
            raise ValueError("input must be contiguous")
        if self.fmt == "ci4":
            if x.dtype != torch.uint8 or x.dim() != 3:
                raise ValueError("ci4 input must be uint8 [channel][time][input]")
            c, t, n = x.shape
        else:
            if x.dtype != torch.int8 or x.dim() != 4 or x.shape[3] != 2:
                raise ValueError("ci8 input must be int8 [channel][time][input][2]")
            c, t, n, _ = x.shape
        if c != self.n_channels or n != self.n_inputs:
            raise ValueError("input shape %s does not match the plan" % (tuple(x.shape),))
        return t

    def _check_output(self, out: torch.Tensor):
        if (out.device != self.device or out.dtype != self.out_dtype or
                tuple(out.shape) != self.out_shape() or not out.is_contiguous()):
            raise ValueError("output must be a contiguous %s tensor %s on %s"
                             % (self.out_dtype, self.out_shape(), self.device))

    def _ptr(self, t: torch.Tensor) -> int:
        return int(t.data_ptr())

    # ------------------------------------------------------------------- calls
    def accumulate(self, x: torch.Tensor):
        t = self._check_input(x)
        _check(lib.xcorr_accumulate(self._h, ctypes.c_void_p(self._ptr(x) if t else 0), t))

    def dump(self, out: torch.Tensor | None = None, reset: bool = True):
        out = self.new_output() if out is None else out
        self._check_output(out)
        info = DumpInfo()
        _check(lib.xcorr_dump(self._h, ctypes.c_void_p(self._ptr(out)), int(bool(reset)),
                              ctypes.byref(info)))
        return out, Dump(info.samples_accumulated, info.start_sample, info.n_dumps)

    def accumulate_dump(self, x: torch.Tensor, out: torch.Tensor | None = None,
                        reset: bool = True):
        t = self._check_input(x)
        out = self.new_output() if out is None else out
        self._check_output(out)
        info = DumpInfo()
        _check(lib.xcorr_accumulate_dump(self._h, ctypes.c_void_p(self._ptr(x) if t else 0), t,
                                         ctypes.c_void_p(self._ptr(out)), int(bool(reset)),
                                         ctypes.byref(info)))
        return out, Dump(info.samples_accumulated, info.start_sample, info.n_dumps)

    def dump_tiles(self, out: torch.Tensor, tile_select, reset: bool = True):
        """Dump (and restart) only the selected 64 x 64 tiles; tile_select is a
        sequence of nr (nr + 1) / 2 flags in lower-triangle tile order."""
        self._check_output(out)
        nr = (self.n_inputs + 63) // 64
        sel = bytes(1 if v else 0 for v in tile_select)
        if len(sel) != nr * (nr + 1) // 2:
            raise ValueError("tile_select needs %d flags" % (nr * (nr + 1) // 2))
        info = DumpInfo()
        buf = (ctypes.c_uint8 * len(sel)).from_buffer_copy(sel)
        _check(lib.xcorr_dump_tiles(self._h, ctypes.c_void_p(self._ptr(out)), ctypes.cast(buf, ctypes.c_void_p),
                                    int(bool(reset)), ctypes.byref(info)))
        return out, Dump(info.samples_accumulated, info.start_sample, info.n_dumps)

    def query(self) -> PlanInfo:
        info = PlanInfo()
        _check(lib.xcorr_query(self._h, ctypes.byref(info)))
        return info

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib.xcorr_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def correlate(x: torch.Tensor, fmt: str = "ci4", path: str = "i8") -> torch.Tensor:
    """One-shot: visibilities of one integration window (fused accumulate + dump)."""
    n_ch, n_in = x.shape[0], x.shape[2]
    with Plan(n_in, n_ch, fmt, path) as p:
        out, _ = p.accumulate_dump(x)
    return out


def correlate_noalloc(x: torch.Tensor, fmt: str = "ci4", out: torch.Tensor | None = None, flags: int = 0,
                      stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """One window through xcorr_correlate_noalloc (int8 path): the library
    allocates no device memory; `out` (int64, or int32 with FLAG_OUT_I32) is
    allocated here when not given."""
    if fmt == "ci4":
        if x.dtype != torch.uint8 or x.dim() != 3:
            raise ValueError("ci4 input must be uint8 [channel][time][input]")
    elif x.dtype != torch.int8 or x.dim() != 4 or x.shape[3] != 2:
        raise ValueError("ci8 input must be int8 [channel][time][input][2]")
    if not x.is_contiguous():
        raise ValueError("input must be contiguous")
    n_ch, n_t, n_in = x.shape[0], x.shape[1], x.shape[2]
    dtype = torch.int32 if flags & FLAG_OUT_I32 else torch.int64
    shape = (n_ch, n_in * (n_in + 1) // 2, 2)
    if out is None:
        out = torch.empty(shape, dtype=dtype, device=x.device)
    elif out.dtype != dtype or tuple(out.shape) != shape or not out.is_contiguous() or out.device != x.device:
        raise ValueError("output must be a contiguous %s tensor %s on %s" % (dtype, shape, x.device))
    stream = stream if stream is not None else torch.cuda.current_stream(x.device)
    desc = make_desc(n_in, n_ch, fmt, "i8", stream, flags)
    with torch.cuda.device(x.device):
        _check(lib.xcorr_correlate_noalloc(ctypes.byref(desc), ctypes.c_void_p(int(x.data_ptr())), int(n_t),
                                           ctypes.c_void_p(int(out.data_ptr()))))
    return out


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(int(p)) for p in ptrs])


class Batch:
    """Several int8 plans (subarrays) run as one persistent launch per step.

    The batch borrows the plans; they must stay open while it exists and must
    not be used on their own while the batch runs.  Work is enqueued on
    `stream` (default: torch's current stream).
    """

    def __init__(self, plans, stream: torch.cuda.Stream | None = None):
        self.plans = list(plans)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        hs = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.xcorr_batch_create(ctypes.byref(h), hs, len(self.plans),
                                      ctypes.c_void_p(int(self.stream.cuda_stream))))
        self._h = h

    def _inputs(self, xs):
        if len(xs) != len(self.plans):
            raise ValueError("one input per plan (None for no samples)")
        ptrs, nts = [], []
        for p, x in zip(self.plans, xs):
            if x is None:
                ptrs.append(0)
                nts.append(0)
            else:
                nts.append(p._check_input(x))
                ptrs.append(x.data_ptr())
        return _ptr_array(ptrs), (ctypes.c_int64 * len(nts))(*nts)

    def _outputs(self, outs):
        ptrs = []
        for p, o in zip(self.plans, outs):
            if o is None:
                ptrs.append(0)
            else:
                p._check_output(o)
                ptrs.append(o.data_ptr())
        return _ptr_array(ptrs)

    def run(self, xs, outs=None, reset=True):
        """One step: xs[k] samples for plan k; dump plan k into outs[k] when given."""
        d_in, nt = self._inputs(xs)
        outs = outs if outs is not None else [None] * len(self.plans)
        d_out = self._outputs(outs)
        rs = (ctypes.c_int32 * len(self.plans))(*([int(bool(reset))] * len(self.plans)))
        info = (DumpInfo * len(self.plans))()
        _check(lib.xcorr_batch_run(self._h, d_in, nt, d_out, rs, info))
        return [Dump(i.samples_accumulated, i.start_sample, i.n_dumps) if o is not None else None
                for i, o in zip(info, outs)]

    def config(self) -> dict:
        c = BatchConfig()
        _check(lib.xcorr_batch_get_config(self._h, ctypes.byref(c)))
        return c.as_dict()

    def set_config(self, tile=0, grid=256, balance=1):
        c = BatchConfig(int(tile), int(grid), int(balance), 0)
        _check(lib.xcorr_batch_set_config(self._h, ctypes.byref(c)))

    def autotune(self, xs, reps: int = 3):
        d_in, nt = self._inputs(xs)
        c = BatchConfig()
        ms = ctypes.c_float(0)
        _check(lib.xcorr_batch_autotune(self._h, d_in, nt, int(reps), ctypes.byref(c), ctypes.byref(ms)))
        return c.as_dict(), float(ms.value)

    def capture(self, xs, outs) -> "Graph":
        d_in, nt = self._inputs(xs)
        d_out = self._outputs(outs)
        g = ctypes.c_void_p()
        _check(lib.xcorr_batch_capture(self._h, d_in, nt, d_out, ctypes.byref(g)))
        return Graph(g, self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib.xcorr_batch_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured integration step of a Batch (one full window per plan)."""

    def __init__(self, h, batch):
        self._h, self.batch = h, batch

    def launch(self):
        _check(lib.xcorr_graph_launch(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib.xcorr_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Streaming server: streams admitted by device memory, windows batched
    continuously by a native worker thread (see include/xcorr.h).

    Inputs must be complete on the device when submitted (synchronise the
    producing stream first); outputs are valid once their ticket is done.
    """

    def __init__(self, device_budget: int, max_streams: int = 16, max_inflight: int = 2,
                 stream: torch.cuda.Stream | None = None, tune_path: str | None = None):
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self._tune_path = tune_path.encode() if tune_path else None
        d = ServerDesc(int(device_budget), int(max_streams), int(max_inflight),
                       ctypes.c_void_p(int(self.stream.cuda_stream)), self._tune_path)
        h = ctypes.c_void_p()
        _check(lib.xcorr_server_create(ctypes.byref(h), ctypes.byref(d)))
        self._h = h
        self._streams = {}

    def open(self, n_inputs: int, n_channels: int, fmt: str = "ci4", tile: int = 0, flags: int = 0) -> int:
        desc = make_desc(n_inputs, n_channels, fmt, "i8", tile=tile, flags=flags)
        sid = ctypes.c_int32(0)
        _check(lib.xcorr_server_open(self._h, ctypes.byref(desc), ctypes.byref(sid)))
        self._streams[sid.value] = (n_inputs, n_channels, fmt, torch.int32 if flags & FLAG_OUT_I32 else torch.int64)
        return sid.value

    def new_output(self, sid: int) -> torch.Tensor:
        n, c, _, dt = self._streams[sid]
        return torch.empty((c, n * (n + 1) // 2, 2), dtype=dt, device=self.stream.device)

    def submit(self, sid: int, x: torch.Tensor, out: torch.Tensor) -> int:
        n, c, fmt, dt = self._streams[sid]
        if not x.is_contiguous() or x.shape[0] != c or x.shape[2] != n:
            raise ValueError("input does not match stream %d" % sid)
        if fmt == "ci4" and (x.dtype != torch.uint8 or x.dim() != 3):
            raise ValueError("ci4 input must be uint8 [channel][time][input]")
        if fmt == "ci8" and (x.dtype != torch.int8 or x.dim() != 4):
            raise ValueError("ci8 input must be int8 [channel][time][input][2]")
        if (out.dtype != dt or not out.is_contiguous()
                or tuple(out.shape) != (c, n * (n + 1) // 2, 2)):
            raise ValueError("output does not match stream %d" % sid)
        t = ctypes.c_int64(0)
        _check(lib.xcorr_server_submit(self._h, int(sid), ctypes.c_void_p(x.data_ptr()), int(x.shape[1]),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int32(0)
        info = DumpInfo()
        lat = ctypes.c_double(0)
        _check(lib.xcorr_server_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(info),
                                     ctypes.byref(lat)))
        if not done.value:
            return False, None, None
        return True, Dump(info.samples_accumulated, info.start_sample, info.n_dumps), lat.value

    def wait(self, ticket: int):
        info = DumpInfo()
        lat = ctypes.c_double(0)
        _check(lib.xcorr_server_wait(self._h, int(ticket), ctypes.byref(info), ctypes.byref(lat)))
        return Dump(info.samples_accumulated, info.start_sample, info.n_dumps), lat.value

    def set_deadline(self, sid: int, sample_period_s: float):
        """Windows of this stream are due n_time * sample_period_s after submission."""
        _check(lib.xcorr_server_set_deadline(self._h, int(sid), float(sample_period_s)))

    def close_stream(self, sid: int):
        _check(lib.xcorr_server_close(self._h, int(sid)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib.xcorr_server_query(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib.xcorr_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def corner_turn(packets: torch.Tensor, n_fengines: int, inputs_per_feng: int, n_channels: int,
                spectra_per_packet: int, valid: torch.Tensor | None = None, out_fmt: str = "ci4",
                out: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """X-stage input from captured F-engine packets (see xcorr_corner_turn)."""
    if packets.dtype != torch.uint8 or not packets.is_contiguous() or not packets.is_cuda:
        raise ValueError("packets must be a contiguous uint8 device tensor")
    per_block = n_fengines * spectra_per_packet * n_channels * inputs_per_feng
    if packets.numel() % per_block:
        raise ValueError("packet buffer size is not a whole number of blocks")
    n_blocks = packets.numel() // per_block
    n_in = n_fengines * inputs_per_feng
    shape = (n_channels, n_blocks * spectra_per_packet, n_in)
    if out_fmt == "ci8":
        shape = shape + (2,)
    dt = torch.uint8 if out_fmt == "ci4" else torch.int8
    if out is None:
        out = torch.empty(shape, dtype=dt, device=packets.device)
    elif tuple(out.shape) != shape or out.dtype != dt or not out.is_contiguous():
        raise ValueError("output must be a contiguous %s tensor %s" % (dt, shape))
    if valid is not None and (valid.dtype != torch.uint8 or valid.numel() != n_blocks * n_fengines
                              or not valid.is_contiguous() or valid.device != packets.device):
        raise ValueError("valid must be a contiguous uint8 device tensor [n_blocks][n_fengines]")
    lay = PacketLayout(n_blocks, n_fengines, inputs_per_feng, n_channels, spectra_per_packet)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.xcorr_corner_turn(ctypes.c_void_p(packets.data_ptr()),
                                 ctypes.c_void_p(valid.data_ptr() if valid is not None else 0),
                                 ctypes.byref(lay), FORMATS[out_fmt], ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(int(s.cuda_stream))))
    return out


def accumulate_gated(plans, x: torch.Tensor, gate) -> None:
    """Pulsar gating: sample t of x goes to plans[gate[t]] (255 = discarded)."""
    t = plans[0]._check_input(x)
    for p in plans[1:]:
        p._check_input(x)
    g = bytes(int(v) for v in gate)
    if len(g) != t:
        raise ValueError("one gate per sample")
    hs = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    buf = (ctypes.c_uint8 * max(1, len(g))).from_buffer_copy(g if g else b"\0")
    _check(lib.xcorr_accumulate_gated(hs, len(plans), ctypes.c_void_p(x.data_ptr() if t else 0), t,
                                      ctypes.cast(buf, ctypes.c_void_p)))


def fstage(adc: torch.Tensor, coeff: torch.Tensor, gain: torch.Tensor, chan_begin: int, n_chan: int,
           n_taps: int = 2, n_points: int = 8192, out_kind: str = "ci4", n_samples: int | None = None,
           out: torch.Tensor | None = None, work: torch.Tensor | None = None,
           stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """F-stage: int8 ADC samples [n_inputs][stride] -> X-stage input (see xcorr_fstage).

    Returns uint8 [n_chan][n_spectra][n_inputs] ("ci4") or float32
    [n_chan][n_spectra][n_inputs][2] ("f32").  `work` (uint8, device) is the
    scratch of the CI4 output; one of the needed size is made if absent."""
    if adc.dtype != torch.int8 or adc.dim() != 2 or adc.stride(1) != 1 or not adc.is_cuda:
        raise ValueError("adc must be an int8 device tensor [n_inputs][samples] with unit sample stride")
    n_in = adc.shape[0]
    n_samples = adc.shape[1] if n_samples is None else n_samples
    for name, t in (("coeff", coeff), ("gain", gain)):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != adc.device:
            raise ValueError("%s must be a contiguous float32 tensor on the ADC's device" % name)
    if coeff.numel() != n_taps * n_points or gain.numel() != n_in * n_chan:
        raise ValueError("coeff must hold n_taps * n_points values and gain n_inputs * n_chan")
    n_spec = max(0, n_samples // n_points - n_taps + 1)
    kind = {"ci4": FSTAGE_CI4, "f32": FSTAGE_F32}[out_kind]
    shape = (n_chan, n_spec, n_in) if kind == FSTAGE_CI4 else (n_chan, n_spec, n_in, 2)
    dt = torch.uint8 if kind == FSTAGE_CI4 else torch.float32
    if out is None:
        out = torch.empty(shape, dtype=dt, device=adc.device)
    elif tuple(out.shape) != shape or out.dtype != dt or not out.is_contiguous():
        raise ValueError("output must be a contiguous %s tensor %s" % (dt, shape))
    d = FstageDesc(n_in, n_points, n_taps, chan_begin, n_chan, kind)
    nb = ctypes.c_size_t(0)
    _check(lib.xcorr_fstage_work_bytes(ctypes.byref(d), n_samples, ctypes.byref(nb)))
    if work is None or work.numel() < nb.value:
        work = torch.empty(max(1, nb.value), dtype=torch.uint8, device=adc.device) if nb.value else None
    got = ctypes.c_int64(-1)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.xcorr_fstage(ctypes.byref(d), ctypes.c_void_p(adc.data_ptr()), adc.stride(0), n_samples,
                            ctypes.c_void_p(coeff.data_ptr()), ctypes.c_void_p(gain.data_ptr()),
                            ctypes.c_void_p(work.data_ptr() if work is not None else 0),
                            ctypes.c_void_p(out.data_ptr() if out.numel() else 0), ctypes.byref(got),
                            ctypes.c_void_p(int(s.cuda_stream))))
    if got.value != n_spec:
        raise RuntimeError("spectra count mismatch")
    return out


class ClockProbe:
    """Shader clock under load (measurement support): start() launches one
    wave on `stream` that waits `ms` of wall-clock time; mhz(), once the
    stream has passed it, is the shader clock that wave saw."""

    def __init__(self, device=None):
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.buf = torch.zeros(4, dtype=torch.int64, device=dev)
        khz = ctypes.c_int32(0)
        # a one-tick probe, only to read the wall-clock rate
        _check(lib.xcorr_clock_probe(ctypes.c_void_p(self.buf.data_ptr()), 1, ctypes.byref(khz),
                                     ctypes.c_void_p(int(torch.cuda.current_stream(dev).cuda_stream))))
        torch.cuda.synchronize(dev)
        self.wall_khz = khz.value

    def start(self, ms: float, stream: torch.cuda.Stream):
        ticks = max(1, int(ms * self.wall_khz))
        _check(lib.xcorr_clock_probe(ctypes.c_void_p(self.buf.data_ptr()), ticks, None,
                                     ctypes.c_void_p(int(stream.cuda_stream))))

    def mhz(self) -> float:
        r0, r1, c0, c1 = (int(v) for v in self.buf.cpu())
        if r1 <= r0 or self.wall_khz <= 0:
            raise RuntimeError("clock probe did not run")
        return (c1 - c0) / (r1 - r0) * self.wall_khz / 1e3
