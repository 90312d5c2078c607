"""String sample sort on one AMD Instinct MI355X (gfx950).

Thin ctypes binding of ``libss.so`` (C ABI in ``include/ss.h``).  Tensors
provide device memory and streams; every step of the sort runs in the HIP
kernels of the library.  The binding only marshals arguments: it never sorts
or computes LCPs itself, and it raises if the compiled library is missing.

    import torch, paper_1808_00963_amd as ss
    perm, lcp = ss.sort(chars_u8_cuda, offsets_i64_cuda)

Outputs are uint32 values stored in int32 tensors.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libss.so")

SS_OK, SS_INVALID_ARG, SS_OUT_OF_MEMORY, SS_HIP_ERROR, SS_LIMIT, SS_REJECTED, SS_TIMEOUT, SS_INTERNAL = range(8)
MODE_LEVELS, MODE_PERSISTENT, MODE_HOST_LEVELS = range(3)
MODES = {"levels": MODE_LEVELS, "persistent": MODE_PERSISTENT, "host_levels": MODE_HOST_LEVELS}
ALPHABET_AUTO, ALPHABET_BYTES, ALPHABET_COMPRESS = range(3)
ALPHABETS = {"auto": ALPHABET_AUTO, "bytes": ALPHABET_BYTES, "compress": ALPHABET_COMPRESS}

_lib = None


class SSError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


class Config(ctypes.Structure):
    _fields_ = [("max_log_splitters", ctypes.c_uint32), ("bucket_target", ctypes.c_uint32),
                ("base_max", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("alphabet", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("dist_segments", ctypes.c_uint32),
                ("dist_tiles", ctypes.c_uint32), ("base_segments", ctypes.c_uint32),
                ("pending_lcps", ctypes.c_uint32), ("max_depth", ctypes.c_uint32),
                ("base_rounds", ctypes.c_uint32), ("base_segments_by_class", ctypes.c_uint32 * 4),
                ("base_strings_by_class", ctypes.c_uint64 * 4), ("key_chars", ctypes.c_uint32),
                ("alphabet_size", ctypes.c_uint32), ("alphabet_retries", ctypes.c_uint32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("unit", ctypes.c_char_p), ("launches", ctypes.c_uint32),
                ("total_ms", ctypes.c_double), ("units", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("chars", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n", ctypes.c_uint32),
                ("perm_out", ctypes.c_void_p), ("lcp_out", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("strings_completed", ctypes.c_uint64), ("chars_completed", ctypes.c_uint64),
                ("inflight_max", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("footprint_max", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("iter_max_us", ctypes.c_double), ("iter_max_wait_us", ctypes.c_double),
                ("iter_max_stage_us", ctypes.c_double)]


def lib():
    """Loads libss.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1808_00963_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sig = {
            "ss_status_string": (ctypes.c_char_p, [i32]),
            "ss_version": (ctypes.c_char_p, []),
            "ss_ctx_create": (i32, [ctypes.POINTER(vp), i32, ctypes.c_size_t]),
            "ss_ctx_destroy": (None, [vp]),
            "ss_get_config": (i32, [vp, ctypes.POINTER(Config)]),
            "ss_set_config": (i32, [vp, ctypes.POINTER(Config)]),
            "ss_workspace_query": (i32, [vp, u32, ctypes.POINTER(ctypes.c_size_t)]),
            "ss_sort_ex": (i32, [vp, vp, vp, u32, vp, vp, vp]),
            "ss_sort": (i32, [vp, vp, u32, vp, vp, vp]),
            "ss_sort_noalloc": (i32, [vp, vp, u32, vp, vp, vp, vp]),
            "ss_sort_batch": (i32, [vp, vp, vp, u32, vp, u32, vp, vp, vp]),
            "ss_get_last_error": (i32, [vp]),
            "ss_clear_error": (None, [vp]),
            "ss_get_stats": (i32, [vp, ctypes.POINTER(Stats)]),
            "ss_graph_create_batch": (i32, [vp, vp, vp, u32, vp, u32, vp, vp, ctypes.POINTER(vp)]),
            "ss_graph_launch": (i32, [vp, vp]),
            "ss_graph_destroy": (None, [vp]),
            "ss_graph_levels": (u32, [vp]),
            "ss_ctx_sync": (i32, [vp, vp]),
            "ss_server_create": (i32, [ctypes.POINTER(vp), i32, ctypes.c_size_t, u32, u32, ctypes.POINTER(Config)]),
            "ss_server_submit": (i32, [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]),
            "ss_server_wait": (i32, [vp, u64, i32, ctypes.POINTER(ctypes.c_double)]),
            "ss_server_cancel": (i32, [vp, u64]),
            "ss_server_footprint": (ctypes.c_size_t, [vp, u32, u64]),
            "ss_server_get_stats": (i32, [vp, ctypes.POINTER(ServerStats)]),
            "ss_server_reset_stats": (None, [vp]),
            "ss_server_destroy": (None, [vp]),
            "ss_set_profiling": (i32, [vp, i32]),
            "ss_set_profiling_only": (i32, [vp, ctypes.c_char_p]),
            "ss_get_kernel_times": (i32, [vp, ctypes.POINTER(KernelTime), u32, ctypes.POINTER(u32)]),
            "ss_reset_kernel_times": (None, [vp]),
            "ss_hbm_copy": (i32, [vp, vp, ctypes.c_size_t, vp]),
            "ss_autotune": (i32, [vp, vp, vp, u32, vp, u32, vp, vp, vp, u32, i32, ctypes.POINTER(Config),
                                  ctypes.POINTER(ctypes.c_double)]),
            "ss_autotune_clear_cache": (None, []),
            "ss_merge_runs": (i32, [vp, vp, vp, u32, vp, vp, ctypes.POINTER(u64), u32, vp, vp, vp]),
            "ss_suffix_array": (i32, [vp, vp, u32, vp, vp, ctypes.POINTER(u32), vp]),
            "ss_host_key": (u64, [vp, u64, u64, ctypes.POINTER(u32)]),
            "ss_host_gather_key": (u64, [vp, u64, u32, u32]),
            "ss_host_gather_packed": (u64, [vp, u64, u32, u32, vp, vp, vp]),
            "ss_host_lcp_stream": (u32, [vp, u64, u32, u64, u32, u32, u32, u32]),
            "ss_host_key_lcp": (u32, [vp, u64, u32, u64, u32, u32]),
            "ss_host_level_index": (u32, [u32, u32]),
            "ss_host_inorder_index": (u32, [u32, u32]),
            "ss_host_classify": (i32, [vp, vp, u32, vp, vp, u32, vp]),
            "ss_host_select_splitters": (i32, [vp, vp, u32, u32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().ss_status_string(status).decode()


def version() -> str:
    return lib().ss_version().decode()


def _check(status: int, what: str):
    if status != SS_OK:
        raise SSError(status, what)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_inputs(chars: torch.Tensor, offsets: torch.Tensor):
    if not (chars.is_cuda and offsets.is_cuda):
        raise ValueError("chars and offsets must be device tensors")
    if chars.dtype != torch.uint8 or offsets.dtype not in (torch.int64, torch.uint64):
        raise TypeError("chars must be uint8 and offsets int64/uint64")
    if not (chars.is_contiguous() and offsets.is_contiguous()):
        raise ValueError("inputs must be contiguous")
    if offsets.numel() < 1:
        raise ValueError("offsets needs n+1 entries")


class Context:
    """An ss_ctx: owns the device workspace of one host thread's sorts."""

    def __init__(self, device: int | None = None, scratch_limit: int = 0):
        self._h = ctypes.c_void_p()
        dev = torch.cuda.current_device() if device is None else device
        _check(lib().ss_ctx_create(ctypes.byref(self._h), dev, scratch_limit), "ss_ctx_create")
        self.device = dev

    def close(self):
        if self._h:
            lib().ss_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def config(self) -> Config:
        c = Config()
        _check(lib().ss_get_config(self._h, ctypes.byref(c)), "ss_get_config")
        return c

    def set_config(self, max_log_splitters=None, bucket_target=None, base_max=None, mode=None, alphabet=None):
        """mode: "levels" (device-driven levels, default), "persistent" or
        "host_levels" (or the MODE_* constants); alphabet: "bytes"
        (default), "auto" or "compress" (or the ALPHABET_* constants)."""
        c = self.config
        if max_log_splitters is not None:
            c.max_log_splitters = max_log_splitters
        if bucket_target is not None:
            c.bucket_target = bucket_target
        if base_max is not None:
            c.base_max = base_max
        if mode is not None:
            c.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        if alphabet is not None:
            c.alphabet = ALPHABETS[alphabet] if isinstance(alphabet, str) else int(alphabet)
        _check(lib().ss_set_config(self._h, ctypes.byref(c)), "ss_set_config")

    def stats(self) -> dict:
        s = Stats()
        _check(lib().ss_get_stats(self._h, ctypes.byref(s)), "ss_get_stats")
        out = {}
        for f, _ in Stats._fields_:
            v = getattr(s, f)
            out[f] = list(v) if isinstance(v, ctypes.Array) else v
        return out

    def set_profiling(self, on: bool = True, only: str | None = None):
        """Per-kernel HIP-event timing; `only` limits it to one kernel."""
        if on and only:
            _check(lib().ss_set_profiling_only(self._h, only.encode()), "ss_set_profiling_only")
        else:
            _check(lib().ss_set_profiling(self._h, 1 if on else 0), "ss_set_profiling")

    def kernel_times(self) -> dict:
        """{kernel: {"launches", "total_ms", "units", "unit"}} accumulated while profiling."""
        arr = (KernelTime * 32)()
        cnt = ctypes.c_uint32()
        _check(lib().ss_get_kernel_times(self._h, arr, 32, ctypes.byref(cnt)), "ss_get_kernel_times")
        return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                       "units": arr[i].units, "unit": arr[i].unit.decode()}
                for i in range(min(cnt.value, 32))}

    def reset_kernel_times(self):
        lib().ss_reset_kernel_times(self._h)

    def workspace_bytes(self, n: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().ss_workspace_query(self._h, n, ctypes.byref(b)), "ss_workspace_query")
        return b.value

    def last_error(self) -> int:
        return lib().ss_get_last_error(self._h)

    def clear_error(self):
        lib().ss_clear_error(self._h)

    def sort(self, chars, offsets, perm=None, lcp=None, stream=None):
        """Enqueues the sort of one set on `stream` (current stream if None)
        and returns (perm, lcp) int32 tensors holding uint32, complete once
        the stream reaches this point.  Device-side errors are raised by
        sync()."""
        _check_inputs(chars, offsets)
        n = offsets.numel() - 1
        if perm is None:
            perm = torch.empty(n, dtype=torch.int32, device=chars.device)
        if lcp is None:
            lcp = torch.empty(n, dtype=torch.int32, device=chars.device)
        st = lib().ss_sort_ex(self._h, ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                              ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                              _stream_ptr(stream))
        _check(st, "ss_sort_ex")
        return perm, lcp

    def sync(self, stream=None):
        """Waits for the stream and the context's last sort; raises on a
        (sticky) device-side error of any sort since clear_error()."""
        _check(lib().ss_ctx_sync(self._h, _stream_ptr(stream)), "ss_ctx_sync")

    def graph_batch(self, chars, offsets, set_begin, perm, lcp) -> "Graph":
        """Captures the batched sort of these buffers as a hipGraph with one
        persistent kernel (see ss_graph_create_batch)."""
        _check_inputs(chars, offsets)
        n = offsets.numel() - 1
        g = ctypes.c_void_p()
        st = lib().ss_graph_create_batch(self._h, ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                         n, ctypes.c_void_p(set_begin.data_ptr()), set_begin.numel() - 1,
                                         ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                                         ctypes.byref(g))
        _check(st, "ss_graph_create_batch")
        return Graph(g, self, (chars, offsets, set_begin, perm, lcp))

    def sort_batch(self, chars, offsets, set_begin, perm=None, lcp=None, stream=None):
        """Sorts the sets delimited by set_begin (int32/uint32 device tensor,
        num_sets+1 entries); outputs hold set-local indices."""
        _check_inputs(chars, offsets)
        if not set_begin.is_cuda or set_begin.dtype not in (torch.int32, torch.uint32):
            raise TypeError("set_begin must be an int32/uint32 device tensor")
        n = offsets.numel() - 1
        num_sets = set_begin.numel() - 1
        if perm is None:
            perm = torch.empty(n, dtype=torch.int32, device=chars.device)
        if lcp is None:
            lcp = torch.empty(n, dtype=torch.int32, device=chars.device)
        st = lib().ss_sort_batch(self._h, ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                                 ctypes.c_void_p(set_begin.data_ptr()), num_sets,
                                 ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                                 _stream_ptr(stream))
        _check(st, "ss_sort_batch")
        return perm, lcp

    def merge_runs(self, chars, offsets, perm, lcp, run_begin, perm_out=None, lcp_out=None, stream=None):
        """LCP-aware merge of the sorted runs perm[run_begin[r]:run_begin[r+1]]
        (with their LCP arrays) into one sorted sequence (ss_merge_runs);
        run_begin is a host sequence of num_runs+1 ints.  Returns
        (perm_out, lcp_out) int32 tensors holding uint32."""
        _check_inputs(chars, offsets)
        for t in (perm, lcp):
            if not t.is_cuda or t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous():
                raise TypeError("perm and lcp must be contiguous int32/uint32 device tensors")
        rb = [int(x) for x in run_begin]
        if len(rb) < 2:
            raise ValueError("run_begin needs num_runs+1 entries")
        m = rb[-1]
        if perm.numel() < m or lcp.numel() < m:
            raise ValueError("perm/lcp shorter than run_begin[-1]")
        if perm_out is None:
            perm_out = torch.empty(m, dtype=torch.int32, device=chars.device)
        if lcp_out is None:
            lcp_out = torch.empty(m, dtype=torch.int32, device=chars.device)
        if perm_out.numel() < m or lcp_out.numel() < m:
            raise ValueError("outputs shorter than run_begin[-1]")
        arr = (ctypes.c_uint64 * len(rb))(*rb)
        st = lib().ss_merge_runs(self._h, ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                 offsets.numel() - 1, ctypes.c_void_p(perm.data_ptr()),
                                 ctypes.c_void_p(lcp.data_ptr()), arr, len(rb) - 1,
                                 ctypes.c_void_p(perm_out.data_ptr()), ctypes.c_void_p(lcp_out.data_ptr()),
                                 _stream_ptr(stream))
        _check(st, "ss_merge_runs")
        return perm_out, lcp_out

    def suffix_array(self, text, sa=None, isa=None, stream=None):
        """Suffix array of a uint8 device text by prefix doubling
        (ss_suffix_array); returns (sa, isa, rounds) with int32 tensors
        holding uint32."""
        if not text.is_cuda or text.dtype != torch.uint8 or not text.is_contiguous():
            raise TypeError("text must be a contiguous uint8 device tensor")
        n = text.numel()
        if sa is None:
            sa = torch.empty(n, dtype=torch.int32, device=text.device)
        if isa is None:
            isa = torch.empty(n, dtype=torch.int32, device=text.device)
        rounds = ctypes.c_uint32(0)
        st = lib().ss_suffix_array(self._h, ctypes.c_void_p(text.data_ptr()), n, ctypes.c_void_p(sa.data_ptr()),
                                   ctypes.c_void_p(isa.data_ptr()), ctypes.byref(rounds), _stream_ptr(stream))
        _check(st, "ss_suffix_array")
        return sa, isa, rounds.value

    def autotune(self, chars, offsets, set_begin=None, perm=None, lcp=None, reps=3, use_cache=True,
                 stream=None):
        """Times candidate configurations on this input (ss_autotune), keeps
        the fastest as this context's configuration and returns
        (config dict, median ms, perm, lcp); perm/lcp hold the result."""
        _check_inputs(chars, offsets)
        n = offsets.numel() - 1
        if set_begin is None:
            sb, num_sets = None, 1
        else:
            if not set_begin.is_cuda or set_begin.dtype not in (torch.int32, torch.uint32):
                raise TypeError("set_begin must be an int32/uint32 device tensor")
            sb, num_sets = ctypes.c_void_p(set_begin.data_ptr()), set_begin.numel() - 1
        if perm is None:
            perm = torch.empty(n, dtype=torch.int32, device=chars.device)
        if lcp is None:
            lcp = torch.empty(n, dtype=torch.int32, device=chars.device)
        best = Config()
        ms = ctypes.c_double(0.0)
        st = lib().ss_autotune(self._h, ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                               sb, num_sets, ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                               _stream_ptr(stream), reps, 1 if use_cache else 0, ctypes.byref(best),
                               ctypes.byref(ms))
        _check(st, "ss_autotune")
        cfg = {f: int(getattr(best, f)) for f, _ in Config._fields_}
        return cfg, ms.value, perm, lcp


def autotune_clear_cache():
    lib().ss_autotune_clear_cache()


class Graph:
    """A captured batched sort (ss_graph); keeps its buffers alive."""

    def __init__(self, handle, ctx, keep):
        self._h = handle
        self.ctx = ctx
        self._keep = keep

    def launch(self, stream=None):
        _check(lib().ss_graph_launch(self._h, _stream_ptr(stream)), "ss_graph_launch")

    @property
    def levels(self) -> int:
        """Level launches in the graph before its persistent tail."""
        return int(lib().ss_graph_levels(self._h))

    def close(self):
        if self._h:
            lib().ss_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching sort server (ss_server): host numpy requests in,
    host numpy results out.  See include/ss.h."""

    def __init__(self, hbm_budget: int, max_inflight: int = 1024, mean_len_hint: int = 0, device: int | None = None,
                 config: Config | None = None):
        self._h = ctypes.c_void_p()
        dev = torch.cuda.current_device() if device is None else device
        cfg = ctypes.byref(config) if config is not None else None
        _check(lib().ss_server_create(ctypes.byref(self._h), dev, hbm_budget, max_inflight, mean_len_hint, cfg),
               "ss_server_create")
        self._live = {}

    def footprint(self, n: int, n_chars: int) -> int:
        return int(lib().ss_server_footprint(self._h, n, n_chars))

    def submit(self, chars, offsets, perm_out=None, lcp_out=None) -> int:
        """Queues one request (numpy uint8 chars, uint64 offsets); returns a
        ticket.  perm_out / lcp_out: optional uint32 host arrays of at least
        n entries for the results (pinned memory makes the copies back
        asynchronous); new arrays otherwise."""
        import numpy as np
        chars = np.ascontiguousarray(chars, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = offsets.size - 1
        perm = np.empty(max(n, 1), dtype=np.uint32) if perm_out is None else perm_out
        lcp = np.empty(max(n, 1), dtype=np.uint32) if lcp_out is None else lcp_out
        for a in (perm, lcp):
            if a.dtype != np.uint32 or a.size < max(n, 1) or not a.flags.c_contiguous:
                raise ValueError("output arrays must be contiguous uint32 with at least n entries")
        req = Request(chars.ctypes.data if chars.size else None, offsets.ctypes.data, n,
                      perm.ctypes.data, lcp.ctypes.data)
        t = ctypes.c_uint64()
        _check(lib().ss_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "ss_server_submit")
        self._live[t.value] = (chars, offsets, perm, lcp, n)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """Returns (perm, lcp, latency_us) once the request is done."""
        lat = ctypes.c_double()
        st = lib().ss_server_wait(self._h, ticket, timeout_ms, ctypes.byref(lat))
        if st == SS_TIMEOUT:
            raise TimeoutError(f"request {ticket} not done after {timeout_ms} ms")
        keep = self._live.pop(ticket, None)
        _check(st, "ss_server_wait")
        _, _, perm, lcp, n = keep
        return perm[:n], lcp[:n], lat.value

    def cancel(self, ticket: int):
        _check(lib().ss_server_cancel(self._h, ticket), "ss_server_cancel")
        self._live.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ss_server_get_stats(self._h, ctypes.byref(st)), "ss_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_ if f != "pad"}

    def reset_stats(self):
        lib().ss_server_reset_stats(self._h)

    def close(self):
        if self._h:
            lib().ss_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sort(chars, offsets, stream=None):
    """ss_sort with the implicit per-device context."""
    _check_inputs(chars, offsets)
    n = offsets.numel() - 1
    perm = torch.empty(n, dtype=torch.int32, device=chars.device)
    lcp = torch.empty(n, dtype=torch.int32, device=chars.device)
    st = lib().ss_sort(ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                       ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()), _stream_ptr(stream))
    _check(st, "ss_sort")
    return perm, lcp


NOALLOC_MAX_STRINGS = 1 << 20


def sort_noalloc(chars, offsets, perm, lcp, err=None, stream=None):
    """ss_sort_noalloc: the sort with the library's fixed workspace (at most
    NOALLOC_MAX_STRINGS strings, no allocation); perm/lcp (and err, one
    int32 device word receiving the device-side error bits) are
    caller-provided device tensors."""
    _check_inputs(chars, offsets)
    n = offsets.numel() - 1
    if perm.numel() < n or lcp.numel() < n:
        raise ValueError("outputs shorter than n")
    st = lib().ss_sort_noalloc(ctypes.c_void_p(chars.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n,
                               ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                               ctypes.c_void_p(err.data_ptr()) if err is not None else None, _stream_ptr(stream))
    _check(st, "ss_sort_noalloc")
    return perm, lcp


def hbm_copy(dst, src, stream=None):
    """Streaming device copy (bandwidth calibration); tensors of equal byte size."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(lib().ss_hbm_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                             _stream_ptr(stream)), "ss_hbm_copy")


# ---- host-side test entry points (no GPU needed) ----

def host_key(s: bytes, h: int):
    buf = ctypes.create_string_buffer(s, len(s) + 16)
    r = ctypes.c_uint32()
    k = lib().ss_host_key(ctypes.cast(buf, ctypes.c_void_p), len(s), h, ctypes.byref(r))
    return int(k), int(r.value)


def host_level_index(j: int, d: int) -> int:
    return int(lib().ss_host_level_index(j, d))


def host_inorder_index(l: int, d: int) -> int:
    return int(lib().ss_host_inorder_index(l, d))


def host_classify(xk, xr, d, ck, cr):
    import numpy as np
    xk = np.ascontiguousarray(xk, np.uint64); xr = np.ascontiguousarray(xr, np.uint32)
    ck = np.ascontiguousarray(ck, np.uint64); cr = np.ascontiguousarray(cr, np.uint32)
    out = np.zeros(len(ck), np.uint32)
    _check(lib().ss_host_classify(xk.ctypes.data, xr.ctypes.data, d, ck.ctypes.data, cr.ctypes.data, len(ck),
                                  out.ctypes.data), "ss_host_classify")
    return out


def host_select_splitters(sk, sr, d):
    import numpy as np
    sk = np.ascontiguousarray(sk, np.uint64); sr = np.ascontiguousarray(sr, np.uint32)
    v = (1 << d) - 1
    xk = np.zeros(v, np.uint64); xr = np.zeros(v, np.uint32)
    _check(lib().ss_host_select_splitters(sk.ctypes.data, sr.ctypes.data, len(sk), d, xk.ctypes.data, xr.ctypes.data),
           "ss_host_select_splitters")
    return xk, xr
