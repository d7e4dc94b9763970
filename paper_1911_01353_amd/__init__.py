"""MI355X (gfx950) Fourier-domain jerk search matched filter: Python binding.

Thin wrapper over the C ABI in ``include/jerk.h`` (same names). It only
marshals arguments: every step of the search runs in the HIP kernels of
``libjerk.so``. PyTorch supplies device memory and streams; tensors are passed
to the library as raw device pointers.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (JERK_EAGAIN, JERK_ECANCELED, JERK_EHIP, JERK_EINVAL, JERK_ENOMEM, JERK_EPENDING, JERK_OK,
                   NOALLOC_MAX_ROWS, PATH_AUTO, PATH_FFT_FP32, PATH_GEMM_FP16, PATH_GEMM_SPLIT_BF16, PATH_NAMES,
                   JerkError)

__all__ = [
    "Plan", "Server", "peaks_reduce", "stream_check", "stats_workspace_bytes", "plane_stats", "find_candidates",
    "candidates_numpy", "CANDIDATE_DTYPE", "peaks_numpy", "PEAK_DTYPE", "spectrum_workspace_bytes", "prepare_spectrum", "JERK_EHIP", "JERK_ECANCELED", "JerkError", "load", "version", "PATH_FFT_FP32", "PATH_GEMM_SPLIT_BF16", "PATH_GEMM_FP16",
    "PATH_AUTO", "PATH_NAMES", "NOALLOC_MAX_ROWS", "JERK_OK", "JERK_EINVAL", "JERK_ENOMEM", "JERK_EAGAIN", "JERK_EPENDING",
]


def load():
    """Load the HIP library; raises ImportError if it is not built."""
    return _lib.load()


def version() -> str:
    return _lib.load().jerk_version().decode()


def stream_check(stream=None) -> int:
    """``jerk_stream_check``: JERK_OK when the stream's work has finished, JERK_EPENDING while it
    runs; raises JerkError on a device error."""
    st = _lib.load().jerk_stream_check(_stream_ptr(stream))
    if st == JERK_EPENDING:
        return st
    _lib.check(st)
    return st


def _stream_ptr(stream) -> C.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _dev_ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("tensor must be in device memory")
    return C.c_void_p(int(t.data_ptr()))


class Plan:
    """A search plan: lattice, half-widths, width groups and bank layout (host object).

    Mirrors ``jerk_plan_create``; ``path`` is one of ``"fft"``, ``"split_bf16"``,
    ``"fp16"``, ``"auto"`` or a ``PATH_*`` constant.
    """

    def __init__(self, nbins: int, zmax: float, wmax: float, dz: float = 2.0, dw: float = 20.0,
                 path="fft", margin: int = 16, seg_len: int = 0, templates_per_block: int = 0,
                 tap_quantum: int = 0, numbetween: int = 2):
        lib = _lib.load()
        if isinstance(path, str):
            path = PATH_NAMES[path]
        d = _lib.PlanDesc(nbins=nbins, zmax=zmax, wmax=wmax, dz=dz, dw=dw, numbetween=numbetween,
                          margin_bins=margin, path=path, seg_len=seg_len,
                          templates_per_block=templates_per_block, tap_quantum=tap_quantum, flags=0)
        h = C.c_void_p()
        _lib.check(lib.jerk_plan_create(C.byref(d), C.byref(h)))
        self._h = h
        self.desc = d

    # -- host queries ---------------------------------------------------------
    @property
    def handle(self) -> C.c_void_p:
        if self._h is None:
            raise ValueError("plan is closed")
        return self._h

    def info(self) -> dict:
        out = _lib.PlanInfo()
        _lib.check(_lib.load().jerk_plan_info(self.handle, C.byref(out)))
        return {f: getattr(out, f) for f, _ in out._fields_}

    def group(self, g: int) -> dict:
        out = _lib.GroupInfo()
        _lib.check(_lib.load().jerk_plan_group(self.handle, g, C.byref(out)))
        return {f: getattr(out, f) for f, _ in out._fields_}

    def groups(self) -> list:
        return [self.group(g) for g in range(self.info()["n_groups"])]

    def template(self, t: int) -> tuple:
        zb, w = C.c_double(), C.c_double()
        h, g, s = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(_lib.load().jerk_plan_template(self.handle, t, C.byref(zb), C.byref(w), C.byref(h),
                                                  C.byref(g), C.byref(s)))
        return zb.value, w.value, h.value, g.value, s.value

    def members(self) -> np.ndarray:
        n = self.info()["n_templates"]
        out = np.zeros(n, dtype=np.int32)
        _lib.check(_lib.load().jerk_plan_members(self.handle, out.ctypes.data_as(C.POINTER(C.c_int32)), n))
        return out

    def set_group(self, g: int, seg_len: int, templates_per_block: int, path, ept: int = 0) -> None:
        if isinstance(path, str):
            path = PATH_NAMES[path]
        _lib.check(_lib.load().jerk_plan_set_group(self.handle, g, seg_len, templates_per_block, path, ept))

    # -- device work ------------------------------------------------------------
    def new_bank(self, device="cuda"):
        import torch
        return torch.empty(self.info()["bank_bytes"], dtype=torch.uint8, device=device)

    def build_templates(self, bank, stream=None) -> None:
        _lib.check(_lib.load().jerk_templates_build(self.handle, _dev_ptr(bank), bank.numel() * bank.element_size(),
                                                    _stream_ptr(stream)))

    def search(self, bank, spec, plane, t_begin: int = 0, t_end: int | None = None, ws=None,
               stream=None) -> None:
        """Enqueue ``jerk_search``: rows [t_begin, t_end) of ``spec``'s plane into ``plane``.

        ``spec``: complex64 device tensor (n,). ``plane``: float32 device tensor
        (rows, >= 2n) whose row stride is the plane's ``ld``.
        """
        import torch
        if spec.dtype != torch.complex64 or spec.dim() != 1 or not spec.is_contiguous():
            raise ValueError("spec must be a contiguous 1-D complex64 tensor")
        if plane.dtype != torch.float32 or plane.dim() != 2 or plane.stride(1) != 1:
            raise ValueError("plane must be a 2-D float32 tensor with unit column stride")
        n = spec.shape[0]
        if t_end is None:
            t_end = self.info()["n_templates"]
        if plane.shape[0] < t_end - t_begin or plane.shape[1] < 2 * n:
            raise ValueError("plane too small for the requested rows")
        ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
        _lib.check(_lib.load().jerk_search(self.handle, _dev_ptr(bank), _dev_ptr(spec), n, _dev_ptr(plane),
                                           plane.stride(0), t_begin, t_end, _dev_ptr(ws), ws_bytes,
                                           _stream_ptr(stream)))

    def search_group(self, bank, spec, plane, g: int, t_begin: int = 0, t_end: int | None = None,
                     stream=None) -> None:
        """Enqueue ``jerk_search_group``: like ``search`` for width group ``g`` only."""
        n = spec.shape[0]
        if t_end is None:
            t_end = self.info()["n_templates"]
        if plane.shape[0] < t_end - t_begin or plane.shape[1] < 2 * n or plane.stride(1) != 1:
            raise ValueError("plane too small for the requested rows")
        _lib.check(_lib.load().jerk_search_group(self.handle, _dev_ptr(bank), _dev_ptr(spec), n, _dev_ptr(plane),
                                                 plane.stride(0), t_begin, t_end, g, _stream_ptr(stream)))

    def autotune(self, spec, uniform: bool = False, stream=None) -> None:
        """Run ``jerk_plan_autotune`` on a device spectrum (synchronous); scratch from torch."""
        import torch
        n = spec.shape[0]
        nbytes = int(_lib.load().jerk_autotune_scratch_bytes(self.handle, n))
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=spec.device)
        _lib.check(_lib.load().jerk_plan_autotune(self.handle, _dev_ptr(spec), n, _dev_ptr(scratch), nbytes,
                                                  _lib.TUNE_UNIFORM if uniform else 0, _stream_ptr(stream)))
        del scratch

    def search_members(self, bank, spec, plane, g: int, m_begin: int, m_end: int, stream=None) -> None:
        """Enqueue ``jerk_search_members``: members [m_begin, m_end) of group g, row = member - m_begin."""
        n = spec.shape[0]
        if plane.shape[0] < m_end - m_begin or plane.shape[1] < 2 * n or plane.stride(1) != 1:
            raise ValueError("plane too small for the requested rows")
        _lib.check(_lib.load().jerk_search_members(self.handle, _dev_ptr(bank), _dev_ptr(spec), n, _dev_ptr(plane),
                                                   plane.stride(0), g, m_begin, m_end, _stream_ptr(stream)))

    # -- batched search -----------------------------------------------------------
    def batch_workspace_bytes(self, count: int) -> int:
        return int(_lib.load().jerk_batch_workspace_bytes(self.handle, count))

    def keys_per_row(self, nbins: int) -> int:
        return int(_lib.load().jerk_batch_keys_per_row(self.handle, nbins))

    def batch_search(self, bank, items, ws, t_begin: int = 0, t_end: int | None = None, graph: bool = False,
                     flat: bool = True, stream=None) -> None:
        """Enqueue ``jerk_batch_search`` over ``items``: (spec, plane or None, peak keys or None).

        ``plane``: float32 (rows, >= 2n); ``keys``: uint64-sized (rows, >= keys_per_row(n))
        tensor (torch.int64 storage; every key of a row is written, so no clearing is needed).
        ``flat``: one flat launch (the default); ``flat=False``: the persistent kernel
        (JERK_BATCH_PERSISTENT).
        """
        if t_end is None:
            t_end = self.info()["n_templates"]
        arr = (_lib.BatchItem * max(1, len(items)))()
        for i, (spec, plane, keys) in enumerate(items):
            n = spec.shape[0]
            arr[i].spec = _dev_ptr(spec).value
            arr[i].nbins = n
            arr[i].plane = _dev_ptr(plane).value if plane is not None else None
            arr[i].ld = plane.stride(0) if plane is not None else 0
            arr[i].peaks = _dev_ptr(keys).value if keys is not None else None
            arr[i].keys_ld = keys.stride(0) if keys is not None else 0
        _lib.check(_lib.load().jerk_batch_search(self.handle, _dev_ptr(bank), arr, len(items), t_begin, t_end,
                                                 _dev_ptr(ws), ws.numel() * ws.element_size(),
                                                 (_lib.BATCH_GRAPH if graph else 0) | (_lib.BATCH_FLAT if flat else _lib.BATCH_PERSISTENT),
                                                 _stream_ptr(stream)))

    def harmonic_shape(self, n_r: int, n_harm: int) -> tuple:
        """(n_zf, n_wf, n_pf) of the harmonic sum of n_harm harmonics (``jerk_harmonic_shape``)."""
        zf, wf, pf = C.c_int32(), C.c_int32(), C.c_int64()
        _lib.check(_lib.load().jerk_harmonic_shape(self.handle, n_r, n_harm, C.byref(zf), C.byref(wf), C.byref(pf)))
        return zf.value, wf.value, pf.value

    def search_peaks(self, bank, spec, t_begin: int = 0, t_end: int | None = None, out=None, ws=None,
                     stream=None):
        """Enqueue ``jerk_search_peaks``: per-row peaks of rows [t_begin, t_end) without a plane.
        Returns ``out``, a (rows, 2) int32 device tensor of jerk_peak records (float32 power bits,
        uint32 p); ``peaks_numpy`` turns it into a structured array."""
        import torch
        if spec.dtype != torch.complex64 or spec.dim() != 1 or not spec.is_contiguous():
            raise ValueError("spec must be a contiguous 1-D complex64 tensor")
        if t_end is None:
            t_end = self.info()["n_templates"]
        rows = t_end - t_begin
        if out is None:
            out = torch.empty((max(rows, 1), 2), dtype=torch.int32, device=spec.device)
        if out.shape[0] < rows or out.shape[1] != 2 or not out.is_contiguous():
            raise ValueError("out must be a contiguous (rows, 2) tensor")
        need = int(_lib.load().jerk_search_peaks_workspace_bytes(self.handle, t_begin, t_end))
        if ws is None:
            ws = torch.empty(max(need, 8), dtype=torch.uint8, device=spec.device)
        _lib.check(_lib.load().jerk_search_peaks(self.handle, _dev_ptr(bank), _dev_ptr(spec), spec.shape[0], t_begin,
                                                 t_end, _dev_ptr(out), _dev_ptr(ws), ws.numel() * ws.element_size(),
                                                 _stream_ptr(stream)))
        return out

    def search_peaks_noalloc(self, bank, spec, out, t_begin: int = 0, t_end: int | None = None, stream=None):
        """Enqueue ``jerk_search_peaks_noalloc``: ``search_peaks`` with the library's fixed device
        workspace (at most ``NOALLOC_MAX_ROWS`` rows per call); allocates nothing, so ``out`` (a
        contiguous (rows, 2) int32 device tensor) is required. Calls on one GPU must not overlap."""
        import torch
        if spec.dtype != torch.complex64 or spec.dim() != 1 or not spec.is_contiguous():
            raise ValueError("spec must be a contiguous 1-D complex64 tensor")
        if t_end is None:
            t_end = self.info()["n_templates"]
        if out.shape[0] < t_end - t_begin or out.shape[1] != 2 or not out.is_contiguous():
            raise ValueError("out must be a contiguous (rows, 2) tensor")
        _lib.check(_lib.load().jerk_search_peaks_noalloc(self.handle, _dev_ptr(bank), _dev_ptr(spec), spec.shape[0],
                                                         t_begin, t_end, _dev_ptr(out), _stream_ptr(stream)))
        return out

    def batch_search_candidates(self, bank, items, k_sigma: float, pre_level: float | None = None,
                                t_begin: int = 0, t_end: int | None = None, staged: int = 0, ws=None, stream=None):
        """Enqueue ``jerk_batch_search_candidates`` over ``items``: (spec, out, count, stats or None)
        per spectrum, as for ``search_candidates``. Returns the workspace (allocated when omitted)."""
        import torch
        if pre_level is None:
            pre_level = 0.9 * (1.0 + float(k_sigma))
        if t_end is None:
            t_end = self.info()["n_templates"]
        arr = (_lib.BatchCandItem * max(1, len(items)))()
        for i, (spec, out, count, stats) in enumerate(items):
            if spec.dtype != torch.complex64 or spec.dim() != 1 or not spec.is_contiguous():
                raise ValueError("spec must be a contiguous 1-D complex64 tensor")
            if out.dim() != 2 or out.shape[1] != 4 or not out.is_contiguous():
                raise ValueError("out must be a contiguous (capacity, 4) tensor")
            arr[i].spec = _dev_ptr(spec).value
            arr[i].nbins = spec.shape[0]
            arr[i].out = _dev_ptr(out).value
            arr[i].capacity = out.shape[0]
            arr[i].count = _dev_ptr(count).value
            arr[i].stats = _dev_ptr(stats).value if stats is not None else None
        lib = _lib.load()
        if ws is None:
            need = int(lib.jerk_batch_search_candidates_workspace_bytes(self.handle, arr, len(items), t_begin, t_end,
                                                                        float(pre_level), staged))
            dev = items[0][0].device if items else "cuda"
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        _lib.check(lib.jerk_batch_search_candidates(self.handle, _dev_ptr(bank), arr, len(items), t_begin, t_end,
                                                    float(k_sigma), float(pre_level), staged, _dev_ptr(ws),
                                                    ws.numel() * ws.element_size(), _stream_ptr(stream)))
        return ws

    def search_candidates_workspace_bytes(self, nbins: int, pre_level: float, t_begin: int = 0,
                                          t_end: int | None = None, staged: int = 0) -> int:
        if t_end is None:
            t_end = self.info()["n_templates"]
        return int(_lib.load().jerk_search_candidates_workspace_bytes(self.handle, nbins, t_begin, t_end,
                                                                      float(pre_level), staged))

    def search_candidates(self, bank, spec, k_sigma: float, pre_level: float | None, out, count, t_begin: int = 0,
                          t_end: int | None = None, staged: int = 0, stats=None, ws=None, stream=None):
        """Enqueue ``jerk_search_candidates``: the search of rows [t_begin, t_end) with candidate
        selection and no plane. ``pre_level``: the speculative level (None: 0.9 (1 + k_sigma), for a
        spectrum of unit mean power); ``out``: (capacity, 4) int32 device tensor of jerk_candidate
        records; ``count``: one-element int64 device tensor the caller zeroes first; ``staged``:
        staging slots per tile (0 = automatic); ``stats``: optional (rows, 2) float64 device tensor
        of row (mean, sigma). ``ws`` is allocated here when omitted; returns it so that the caller
        can keep it alive with the stream."""
        import torch
        if pre_level is None:
            pre_level = 0.9 * (1.0 + float(k_sigma))
        if spec.dtype != torch.complex64 or spec.dim() != 1 or not spec.is_contiguous():
            raise ValueError("spec must be a contiguous 1-D complex64 tensor")
        if out.dim() != 2 or out.shape[1] != 4 or not out.is_contiguous():
            raise ValueError("out must be a contiguous (capacity, 4) tensor")
        n = spec.shape[0]
        if t_end is None:
            t_end = self.info()["n_templates"]
        if stats is not None and (not stats.is_contiguous() or stats.shape[0] < t_end - t_begin):
            raise ValueError("stats must be a contiguous (rows, 2) float64 tensor")
        need = self.search_candidates_workspace_bytes(n, pre_level, t_begin, t_end, staged)
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=spec.device)
        _lib.check(_lib.load().jerk_search_candidates(
            self.handle, _dev_ptr(bank), _dev_ptr(spec), n, t_begin, t_end, float(k_sigma), float(pre_level),
            int(staged), _dev_ptr(stats) if stats is not None else None, _dev_ptr(out), out.shape[0],
            _dev_ptr(count), _dev_ptr(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)))
        return ws

    def harmonic_sum(self, plane, n_harm: int, out=None, n_r: int | None = None, stream=None):
        """Enqueue ``jerk_harmonic_sum`` over a full (T, >= n_r) float32 plane; returns ``out``
        ((n_zf * n_wf, >= n_pf) float32, allocated here when omitted)."""
        import torch
        n_r = plane.shape[1] if n_r is None else n_r
        zf, wf, pf = self.harmonic_shape(n_r, n_harm)
        if plane.shape[0] != self.info()["n_templates"] or plane.stride(1) != 1:
            raise ValueError("plane must hold every template, rows contiguous")
        if out is None:
            out = torch.empty((zf * wf, pf), dtype=torch.float32, device=plane.device)
        if out.shape[0] < zf * wf or out.shape[1] < pf or out.stride(1) != 1:
            raise ValueError("out too small")
        _lib.check(_lib.load().jerk_harmonic_sum(self.handle, _dev_ptr(plane), plane.stride(0), n_r, n_harm,
                                                 _dev_ptr(out), out.stride(0), _stream_ptr(stream)))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.load().jerk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def peaks_reduce(keys, keys_per_row: int, out, stream=None) -> None:
    """Enqueue ``jerk_peaks_reduce``: keys (rows, ld) int64 tensor -> out (rows, 2) int32-sized tensor of
    (power bits, p) pairs (view it as float32 / uint32)."""
    rows = keys.shape[0]
    _lib.check(_lib.load().jerk_peaks_reduce(_dev_ptr(keys), rows, keys_per_row, keys.stride(0), _dev_ptr(out),
                                             _stream_ptr(stream)))


def spectrum_workspace_bytes(n_samples: int) -> int:
    return int(_lib.load().jerk_spectrum_workspace_bytes(n_samples))


def prepare_spectrum(series, out=None, ws=None, stream=None):
    """Enqueue ``jerk_spectrum_prepare``: float32 device series of N samples -> complex64 device
    spectrum of N/2 bins (``out``, allocated here when omitted). Returns ``(out, ws)``; keep the
    workspace alive until the stream has run."""
    import torch
    n = series.shape[0]
    if series.dtype != torch.float32 or not series.is_contiguous():
        raise ValueError("series must be a contiguous float32 tensor")
    if out is None:
        out = torch.empty(n // 2, dtype=torch.complex64, device=series.device)
    if out.dtype != torch.complex64 or out.numel() < n // 2 or not out.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor of n/2 bins")
    if ws is None:
        ws = torch.empty(max(spectrum_workspace_bytes(n), 1), dtype=torch.uint8, device=series.device)
    _lib.check(_lib.load().jerk_spectrum_prepare(_dev_ptr(series), n, _dev_ptr(out), _dev_ptr(ws), ws.numel(),
                                                 _stream_ptr(stream)))
    return out, ws


CANDIDATE_DTYPE = np.dtype([("t", np.uint32), ("p", np.uint32), ("power", np.float32), ("sigma", np.float32)])


def stats_workspace_bytes(rows: int, n_r: int) -> int:
    return int(_lib.load().jerk_stats_workspace_bytes(rows, n_r))


def plane_stats(plane, stats, n_r: int | None = None, ws=None, stream=None):
    """Enqueue ``jerk_plane_stats`` on a (rows, >= n_r) float32 slab into stats (rows, 2) float64.

    ``ws`` is a device uint8 tensor of at least ``stats_workspace_bytes`` bytes (allocated here
    when omitted). Returns the workspace so that the caller can keep it alive with the stream.
    """
    import torch
    rows = plane.shape[0]
    n_r = plane.shape[1] if n_r is None else n_r
    if plane.stride(1) != 1 or stats.shape[0] < rows or not stats.is_contiguous():
        raise ValueError("plane rows must be contiguous and stats (rows, 2) contiguous")
    need = stats_workspace_bytes(rows, n_r)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=plane.device)
    _lib.check(_lib.load().jerk_plane_stats(_dev_ptr(plane), plane.stride(0), rows, n_r, _dev_ptr(stats),
                                            _dev_ptr(ws), ws.numel(), _stream_ptr(stream)))
    return ws


def find_candidates(plane, stats, k_sigma: float, out, count, n_r: int | None = None, row_template=None,
                    t_base: int = 0, stream=None) -> None:
    """Enqueue ``jerk_find_candidates``: candidates of a (rows, >= n_r) slab appended to ``out``
    (a (capacity, 4) int32 device tensor holding jerk_candidate records) and counted in ``count``
    (a one-element int64 device tensor the caller zeroes first)."""
    rows = plane.shape[0]
    n_r = plane.shape[1] if n_r is None else n_r
    if plane.stride(1) != 1 or out.dim() != 2 or out.shape[1] != 4 or not out.is_contiguous():
        raise ValueError("plane rows must be contiguous and out a contiguous (capacity, 4) tensor")
    rt = _dev_ptr(row_template) if row_template is not None else None
    _lib.check(_lib.load().jerk_find_candidates(_dev_ptr(plane), plane.stride(0), rows, n_r, _dev_ptr(stats),
                                                float(k_sigma), rt, t_base, _dev_ptr(out), out.shape[0],
                                                _dev_ptr(count), _stream_ptr(stream)))


PEAK_DTYPE = np.dtype([("power", np.float32), ("p", np.uint32)])


def peaks_numpy(out, rows: int | None = None) -> np.ndarray:
    """Host copy of (rows, 2) jerk_peak records as a structured array (fields power, p)."""
    n = out.shape[0] if rows is None else rows
    return out[:n].cpu().numpy().view(PEAK_DTYPE).reshape(n)


def candidates_numpy(out, count) -> np.ndarray:
    """Host copy of the stored candidates as a structured array sorted by (t, p)."""
    n = min(int(count.item()), out.shape[0])
    a = out[:n].cpu().numpy().view(CANDIDATE_DTYPE).reshape(n)
    return np.sort(a, order=["t", "p"])


class Server:
    """``jerk_serve_*``: continuous-batching request server on the current device.

    ``arena``: a 256-byte-aligned device buffer (e.g. a torch uint8 tensor) the server
    sub-allocates, or an integer address with ``dry_run=True`` (host-only scheduler test).
    """

    def __init__(self, arena, arena_bytes: int | None = None, max_active: int = 4, queue_capacity: int = 64,
                 tiles_per_launch: int = 0, seg_len: int = 0, slots: int = 0, dry_run: bool = False):
        lib = _lib.load()
        if isinstance(arena, int):
            ptr, nbytes = C.c_void_p(arena), arena_bytes
        else:
            ptr, nbytes = _dev_ptr(arena), arena.numel() * arena.element_size()
        self._arena = arena  # keep the buffer alive
        d = _lib.ServeDesc(max_active=max_active, queue_capacity=queue_capacity, tiles_per_launch=tiles_per_launch,
                           seg_len=seg_len, slots=slots, flags=_lib.SERVE_DRYRUN if dry_run else 0)
        h = C.c_void_p()
        _lib.check(lib.jerk_serve_create(C.byref(d), ptr, nbytes, C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, spec, zmax: float, wmax: float, dz: float = 2.0, dw: float = 20.0, path="fft", plane=None,
               n_templates: int | None = None, nbins: int | None = None, top_k: int = 0) -> int:
        """Queue a request; returns its ticket. ``spec``: device complex64 tensor (or an address with ``nbins``).
        ``n_templates``: also return every row's peak; ``top_k``: also return the k strongest row peaks."""
        if isinstance(path, str):
            path = PATH_NAMES[path]
        if isinstance(spec, int):
            sp, n = spec, nbins
        else:
            sp, n = _dev_ptr(spec).value, spec.shape[0]
        peaks = None
        if n_templates:
            peaks = (_lib.Peak * n_templates)()
        top = (_lib.Top * top_k)() if top_k > 0 else None
        r = _lib.Request(spec=sp, nbins=n, zmax=zmax, wmax=wmax, dz=dz, dw=dw, path=path,
                         peaks_capacity=n_templates or 0,
                         plane=_dev_ptr(plane).value if plane is not None else None,
                         ld=plane.stride(0) if plane is not None else 0,
                         peaks=C.cast(peaks, C.c_void_p) if peaks is not None else None,
                         top=C.cast(top, C.c_void_p) if top is not None else None, top_capacity=top_k)
        t = C.c_uint64()
        _lib.check(_lib.load().jerk_serve_submit(self._h, C.byref(r), C.byref(t)))
        self._keep[t.value] = (spec, plane, peaks, top)
        return t.value

    def _result(self, res, ticket):
        out = {f: getattr(res, f) for f, _ in res._fields_}
        spec, plane, peaks, top = self._keep.get(ticket, (None, None, None, None))
        if peaks is not None:
            arr = np.frombuffer(peaks, dtype=np.dtype([("power", np.float32), ("p", np.uint32)])).copy()
            out["peaks_power"] = arr["power"]
            out["peaks_p"] = arr["p"]
        if top is not None:
            arr = np.frombuffer(top, dtype=np.dtype([("t", np.int32), ("p", np.uint32), ("power", np.float32),
                                                     ("reserved", np.int32)]))[:res.top_count].copy()
            out["top"] = arr[["t", "p", "power"]]
        return out

    def poll(self, ticket: int):
        res = _lib.Result()
        st = _lib.load().jerk_serve_poll(self._h, ticket, C.byref(res))
        if st == JERK_EPENDING:
            return None
        _lib.check(st)
        return self._result(res, ticket)

    def wait(self, ticket: int, timeout_s: float = -1.0):
        res = _lib.Result()
        st = _lib.load().jerk_serve_wait(self._h, ticket, C.byref(res), timeout_s)
        if st == JERK_EPENDING:
            return None
        _lib.check(st)
        return self._result(res, ticket)

    def stats(self) -> dict:
        out = _lib.ServeStats()
        _lib.check(_lib.load().jerk_serve_stats_get(self._h, C.byref(out)))
        return {f: getattr(out, f) for f, _ in out._fields_}

    def inject_failure(self, op: int, n: int) -> None:
        _lib.check(_lib.load().jerk_serve_inject_failure(self._h, op, n))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.load().jerk_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
