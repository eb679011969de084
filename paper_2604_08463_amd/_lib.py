"""ctypes binding of ``libcs.so``: argument marshalling only, every step runs in the HIP library.

The functions keep the C names (``cs_likelihood``, ``cs_likelihood_grad``, ``cs_optimize_batch``,
...).  :class:`Problem` owns the device workspace (a torch uint8 tensor) and forwards torch
tensors as raw device pointers on torch's current HIP stream.  There is no CPU fallback: a
missing library or a non-GPU tensor raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcs.so")

CS_OK, CS_E_INVALID, CS_E_LABEL, CS_E_WORKSPACE, CS_E_HIP, CS_E_UNSUPPORTED, CS_E_STATE = range(7)
PRECISION = {"fp64": 0, "fp32_bulk": 1, "fp32_store": 2}
NOT_PD, NONFINITE, LS_FAIL, MAXITER, CONVERGED, RUNNING = 1, 2, 4, 8, 16, 32


class CsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Desc(C.Structure):
    _fields_ = [
        ("nfreq", C.c_int32), ("npix", C.c_int32), ("nitems", C.c_int32),
        ("freqs_ghz", C.POINTER(C.c_double)),
        ("nu0_dust_ghz", C.c_double), ("nu0_sync_ghz", C.c_double), ("tcmb_k", C.c_double),
        ("precision", C.c_int), ("d_dtype", C.c_int),
        ("d", C.c_void_p), ("d_item_stride", C.c_int64),
        ("ninv_mode", C.c_int),
        ("ninv_band", C.POINTER(C.c_double)),
        ("ninv_pixel", C.c_void_p), ("ninv_item_stride", C.c_int64),
        ("labels", C.c_void_p), ("labels_item_stride", C.c_int64),
        ("nclusters", C.POINTER(C.c_int32)),
    ]


class OptimOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("gtol_rel", C.c_double), ("max_iter", C.c_int32), ("iters_per_graph", C.c_int32),
                ("max_backtracks", C.c_int32), ("c1", C.c_double), ("fp64_polish", C.c_int32),
                ("solver", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("topk", C.c_double), ("switch_rel", C.c_double)]


SOLVER_LBFGS, SOLVER_ADATOPK = 0, 1


class Schedule(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32), ("xcd_remap", C.c_int32),
                ("shared_segments", C.c_int32)]


_lib = None

EXPORTS = [
    "cs_problem_create", "cs_problem_param_offsets", "cs_problem_workspace_bytes", "cs_problem_prepare",
    "cs_problem_item_info", "cs_problem_segments", "cs_likelihood", "cs_likelihood_grad", "cs_component_maps",
    "cs_component_maps_sorted", "cs_problem_pixel_order",
    "cs_kmeans_workspace_bytes", "cs_kmeans_batch", "cs_kmeans_batch_static", "cs_optim_default_opts",
    "cs_optimizer_workspace_bytes", "cs_optimize_batch", "cs_optimize_batch_run", "cs_item_range",
    "cs_problem_desc_slice", "cs_problem_get_schedule", "cs_problem_set_schedule",
    "cs_problem_autotune", "cs_problem_set_timing", "cs_problem_kernel_time", "cs_problem_destroy", "cs_status_str",
    "cs_last_error",
]


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2604_08463_amd.build.build()")
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    P = C.POINTER
    L.cs_problem_create.argtypes = [P(Desc), P(vp)]
    L.cs_problem_param_offsets.argtypes = [vp, P(i64)]
    L.cs_problem_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.cs_problem_prepare.argtypes = [vp, vp, C.c_size_t, vp]
    L.cs_problem_item_info.argtypes = [vp, i32, P(i64), P(i64)]
    L.cs_problem_segments.argtypes = [vp, i32, i32, vp, vp, vp]
    L.cs_likelihood.argtypes = [vp, vp, vp, vp, vp]
    L.cs_likelihood_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.cs_component_maps.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.cs_component_maps_sorted.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.cs_problem_pixel_order.argtypes = [vp, i32, vp, vp]
    L.cs_kmeans_workspace_bytes.argtypes = [i64, i32, P(i32), P(C.c_size_t)]
    L.cs_kmeans_batch.argtypes = [vp, i64, i32, vp, i64, P(i32), vp, i64, i32, vp, i64, vp, vp, C.c_size_t, vp]
    L.cs_kmeans_batch_static.argtypes = [vp, i64, i32, vp, i64, P(i32), vp, i64, i32, vp, i64, vp, vp]
    L.cs_optim_default_opts.argtypes = [P(OptimOpts)]
    L.cs_optimizer_workspace_bytes.argtypes = [vp, i32, P(C.c_size_t)]
    L.cs_optimize_batch.argtypes = [vp, P(OptimOpts), vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
    L.cs_optimize_batch_run.argtypes = [vp, P(OptimOpts), vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, i32, i32, P(i32),
                                        vp]
    L.cs_item_range.argtypes = [i32, i32, i32, P(i32), P(i32)]
    L.cs_problem_desc_slice.argtypes = [P(Desc), i32, i32, P(Desc)]
    L.cs_problem_get_schedule.argtypes = [vp, P(Schedule)]
    L.cs_problem_set_schedule.argtypes = [vp, P(Schedule)]
    L.cs_problem_autotune.argtypes = [vp, vp, vp, vp, i32, P(Schedule), vp]
    L.cs_problem_set_timing.argtypes = [vp, i32]
    L.cs_problem_kernel_time.argtypes = [vp, P(C.c_double), P(i64)]
    L.cs_problem_destroy.argtypes = [vp]
    L.cs_problem_destroy.restype = None
    L.cs_status_str.argtypes = [C.c_int]
    L.cs_status_str.restype = C.c_char_p
    L.cs_last_error.argtypes = []
    L.cs_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("cs_problem_destroy", "cs_status_str", "cs_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != CS_OK:
        L = load()
        raise CsError(rc, where, f"{L.cs_status_str(rc).decode()}: {L.cs_last_error().decode()}")


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("the HIP library takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def default_opts(**kw) -> OptimOpts:
    o = OptimOpts()
    _check(load().cs_optim_default_opts(C.byref(o)), "cs_optim_default_opts")
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def item_range(rank: int, nranks: int, nitems: int) -> tuple[int, int]:
    """Items ``[begin, end)`` of worker ``rank`` of ``nranks`` (contiguous chunking)."""
    b, e = C.c_int32(), C.c_int32()
    _check(load().cs_item_range(rank, nranks, nitems, C.byref(b), C.byref(e)), "cs_item_range")
    return b.value, e.value


class OptState:
    """The optimiser workspace of one problem: the complete, resumable state of a batched run
    (256-byte aligned view of a device buffer).  ``to_host()`` copies it out (a checkpoint);
    ``from_host()`` puts a checkpoint into a fresh workspace."""

    def __init__(self, nbytes: int, device):
        self.nbytes = nbytes
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._off = (-self._buf.data_ptr()) % 256
        self.view = self._buf[self._off:self._off + nbytes]

    @property
    def ptr(self):
        return C.c_void_p(self.view.data_ptr())

    def to_host(self) -> np.ndarray:
        return self.view.cpu().numpy().copy()

    @classmethod
    def from_host(cls, data: np.ndarray, device) -> "OptState":
        st = cls(int(data.size), device)
        st.view.copy_(torch.from_numpy(np.ascontiguousarray(data, dtype=np.uint8)))
        return st


def kmeans_batch(vecs: torch.Tensor, k, init: torch.Tensor, keep: torch.Tensor | None = None, iters: int = 20,
                 stream=None):
    """Spherical K-means patching of T tasks over the unit vectors ``vecs[n][3]`` (device FP64).

    ``k``: T cluster counts; ``init[T][>= max k]`` (device int32): per task, indices into the task's
    kept vectors (ascending pixel order) of the starting centroids; ``keep[T][n]`` (device uint8,
    optional): which vectors a task clusters.  Returns ``(labels[T][n] int32, keff[T] int32)``;
    ``keff[t] = -1`` flags a task whose ``init`` row is out of range.
    """
    L = load()
    vecs = vecs.to(torch.float64).contiguous()
    n = vecs.shape[0]
    kk = np.ascontiguousarray(np.asarray(k, dtype=np.int32).reshape(-1))
    T = kk.size
    init = init.to(torch.int32).contiguous()
    if init.dim() != 2 or init.shape[0] != T:
        raise ValueError("init must be [T][>= max k]")
    if keep is not None:
        keep = keep.to(torch.uint8).contiguous()
        if keep.shape != (T, n):
            raise ValueError("keep must be [T][n]")
    kp = kk.ctypes.data_as(C.POINTER(C.c_int32))
    nb = C.c_size_t()
    _check(L.cs_kmeans_workspace_bytes(n, T, kp, C.byref(nb)), "cs_kmeans_workspace_bytes")
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=vecs.device)
    wp = C.c_void_p((ws.data_ptr() + 255) & ~255)
    labels = torch.empty((T, n), dtype=torch.int32, device=vecs.device)
    keff = torch.empty(T, dtype=torch.int32, device=vecs.device)
    _check(L.cs_kmeans_batch(_ptr(vecs), n, T, _ptr(keep), 0, kp, _ptr(init), init.shape[1], iters, _ptr(labels), 0,
                             _ptr(keff), wp, nb.value, _stream(stream)), "cs_kmeans_batch")
    if stream is not None:
        ws.record_stream(stream)  # the workspace is released in that stream's order
    return labels, keff


def kmeans_batch_static(vecs: torch.Tensor, k, init: torch.Tensor, keep: torch.Tensor | None = None,
                        iters: int = 20, stream=None):
    """As :func:`kmeans_batch`, on the library's own per-GPU scratch array (no workspace is
    allocated); raises when the tasks need more than CS_KMEANS_STATIC_BYTES."""
    L = load()
    vecs = vecs.to(torch.float64).contiguous()
    n = vecs.shape[0]
    kk = np.ascontiguousarray(np.asarray(k, dtype=np.int32).reshape(-1))
    T = kk.size
    init = init.to(torch.int32).contiguous()
    if init.dim() != 2 or init.shape[0] != T:
        raise ValueError("init must be [T][>= max k]")
    if keep is not None:
        keep = keep.to(torch.uint8).contiguous()
        if keep.shape != (T, n):
            raise ValueError("keep must be [T][n]")
    labels = torch.empty((T, n), dtype=torch.int32, device=vecs.device)
    keff = torch.empty(T, dtype=torch.int32, device=vecs.device)
    _check(L.cs_kmeans_batch_static(_ptr(vecs), n, T, _ptr(keep), 0, kk.ctypes.data_as(C.POINTER(C.c_int32)),
                                    _ptr(init), init.shape[1], iters, _ptr(labels), 0, _ptr(keff), _stream(stream)),
           "cs_kmeans_batch_static")
    return labels, keff


class Problem:
    """A batch of items prepared on the device (segments, packed data) and ready to evaluate.

    ``d``: device tensor ``[B or 1][2][F][P]`` (float64 or float32; one shared sky when its
    first dimension is 1), ``labels``: device int32 ``[B or 1][3][P]``, ``ninv``: host ``[2][F]``
    array (band weights) or device tensor ``[B or 1][2][F][P]`` (per-pixel weights).
    """

    def __init__(self, freqs, d: torch.Tensor, ninv, labels: torch.Tensor, nclusters, *, nitems: int | None = None,
                 precision: str = "fp64", nu0_dust: float = 353.0, nu0_sync: float = 23.0, tcmb: float = 2.7255,
                 stream=None):
        L = load()
        self.freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        F = self.freqs.size
        P = int(labels.shape[-1])
        ncl = np.ascontiguousarray(np.atleast_2d(nclusters), dtype=np.int32)
        B = int(nitems if nitems is not None else ncl.shape[0])
        if ncl.shape[0] == 1 and B > 1:
            ncl = np.ascontiguousarray(np.tile(ncl, (B, 1)))
        if ncl.shape != (B, 3):
            raise ValueError("nclusters must be [B][3]")
        if d.dim() != 4 or tuple(d.shape[1:]) != (2, F, P) or d.shape[0] not in (1, B):
            raise ValueError(f"d must be [B or 1][2][{F}][{P}], got {tuple(d.shape)}")
        if labels.dtype != torch.int32 or labels.dim() != 3 or tuple(labels.shape[1:]) != (3, P) or labels.shape[0] not in (1, B):
            raise ValueError("labels must be int32 [B or 1][3][P]")
        if d.dtype not in (torch.float64, torch.float32):
            raise ValueError("d must be float64 or float32")
        self._keep = [d, labels]
        desc = Desc()
        desc.nfreq, desc.npix, desc.nitems = F, P, B
        desc.freqs_ghz = self.freqs.ctypes.data_as(C.POINTER(C.c_double))
        desc.nu0_dust_ghz, desc.nu0_sync_ghz, desc.tcmb_k = nu0_dust, nu0_sync, tcmb
        desc.precision = PRECISION[precision]
        desc.d_dtype = 0 if d.dtype == torch.float64 else 1
        desc.d = _ptr(d)
        desc.d_item_stride = 0 if d.shape[0] == 1 else 2 * F * P
        if isinstance(ninv, torch.Tensor):
            if ninv.dtype != d.dtype or ninv.dim() != 4 or tuple(ninv.shape[1:]) != (2, F, P):
                raise ValueError("per-pixel ninv must match d's dtype and be [B or 1][2][F][P]")
            desc.ninv_mode = 1
            desc.ninv_pixel = _ptr(ninv)
            desc.ninv_item_stride = 0 if ninv.shape[0] == 1 else 2 * F * P
            self._keep.append(ninv)
        else:
            self._ninv = np.ascontiguousarray(ninv, dtype=np.float64).reshape(2, F)
            desc.ninv_mode = 0
            desc.ninv_band = self._ninv.ctypes.data_as(C.POINTER(C.c_double))
        desc.labels = _ptr(labels)
        desc.labels_item_stride = 0 if labels.shape[0] == 1 else 3 * P
        self._ncl = ncl
        desc.nclusters = ncl.ctypes.data_as(C.POINTER(C.c_int32))
        self._setup(desc, d.device, precision, stream)

    def _setup(self, desc, dev, precision, stream):
        """Creates and prepares the library problem of a filled descriptor."""
        L = load()
        self._desc = desc
        B, F, P = desc.nitems, desc.nfreq, desc.npix
        ncl = np.ctypeslib.as_array(desc.nclusters, shape=(B, 3)).copy()
        h = C.c_void_p()
        _check(L.cs_problem_create(C.byref(desc), C.byref(h)), "cs_problem_create")
        self._h = h
        self.nitems, self.nfreq, self.npix, self.precision = B, F, P, precision
        self.nclusters = ncl
        off = np.zeros(B + 1, dtype=np.int64)
        _check(L.cs_problem_param_offsets(h, off.ctypes.data_as(C.POINTER(C.c_int64))), "cs_problem_param_offsets")
        self.param_offsets = off
        nb = C.c_size_t()
        _check(L.cs_problem_workspace_bytes(h, C.byref(nb)), "cs_problem_workspace_bytes")
        self.workspace_bytes = nb.value
        self.device = dev
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        base = self._ws.data_ptr()
        self._ws_ptr = C.c_void_p((base + 255) & ~255)
        self._stream = stream
        _check(L.cs_problem_prepare(h, self._ws_ptr, nb.value, _stream(stream)), "cs_problem_prepare")
        self.param_item = torch.as_tensor(np.repeat(np.arange(B), np.diff(off)), device=dev)

    def chunk(self, rank: int, nranks: int, stream=None) -> "Problem":
        """A problem over this batch's items of worker ``rank`` of ``nranks`` (contiguous chunking,
        the same device arrays, no copy): ``cs_item_range`` then ``cs_problem_desc_slice``."""
        b, e = item_range(rank, nranks, self.nitems)
        out = Desc()
        _check(load().cs_problem_desc_slice(C.byref(self._desc), b, e, C.byref(out)), "cs_problem_desc_slice")
        sub = Problem.__new__(Problem)
        # the arrays the sliced descriptor points into
        sub._keep = list(self._keep)
        sub.freqs, sub._ncl, sub._ninv = self.freqs, self._ncl, getattr(self, "_ninv", None)
        sub._setup(out, self.device, self.precision, stream)
        sub.item_begin = b
        return sub

    @classmethod
    def from_sky(cls, sky, precision: str = "fp64", device="cuda", d_dtype=torch.float64, **kw):
        d = sky.d.to(device=device, dtype=d_dtype).contiguous()
        labels = sky.labels.to(device=device, dtype=torch.int32).contiguous()
        return cls(sky.freqs, d, sky.ninv, labels, sky.nclusters, nitems=sky.nitems, precision=precision,
                   nu0_dust=sky.nu0_dust, nu0_sync=sky.nu0_sync, tcmb=sky.tcmb, **kw)

    def close(self):
        if getattr(self, "_h", None):
            load().cs_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------------------------------
    @property
    def nparams(self) -> int:
        return int(self.param_offsets[-1])

    def _x(self, x):
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        if x.numel() != self.nparams:
            raise ValueError(f"x must hold {self.nparams} packed parameters")
        return x

    def item_info(self, item: int):
        n, s = C.c_int64(), C.c_int64()
        _check(load().cs_problem_item_info(self._h, item, C.byref(n), C.byref(s)), "cs_problem_item_info")
        return n.value, s.value

    def segments(self, item: int, labeling: int):
        n, _ = self.item_info(item)
        k = int(self.nclusters[item, labeling])
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        off = torch.empty(k + 1, dtype=torch.int32, device=self.device)
        _check(load().cs_problem_segments(self._h, item, labeling, _ptr(perm), _ptr(off), _stream(self._stream)),
               "cs_problem_segments")
        return perm[:n], off

    def cs_likelihood(self, x):
        x = self._x(x)
        f = torch.empty(self.nitems, dtype=torch.float64, device=self.device)
        st = torch.empty(self.nitems, dtype=torch.int32, device=self.device)
        _check(load().cs_likelihood(self._h, _ptr(x), _ptr(f), _ptr(st), _stream(self._stream)), "cs_likelihood")
        return f, st

    def cs_likelihood_grad(self, x, cluster: bool = False, out=None):
        x = self._x(x)
        if out is None:
            f = torch.empty(self.nitems, dtype=torch.float64, device=self.device)
            g = torch.empty(self.nparams, dtype=torch.float64, device=self.device)
            st = torch.empty(self.nitems, dtype=torch.int32, device=self.device)
        else:
            f, g, st = out
        cf = torch.empty(self.nparams, dtype=torch.float64, device=self.device) if cluster else None
        _check(load().cs_likelihood_grad(self._h, _ptr(x), _ptr(f), _ptr(g), _ptr(cf), _ptr(st), _stream(self._stream)),
               "cs_likelihood_grad")
        return f, g, cf, st

    def cs_component_maps(self, x, maps: bool = True, sorted_order: bool = False):
        """Returns ``(maps [B][2][3][P] or None, cmb_var [B], status [B])`` (device tensors); with
        ``sorted_order`` the maps are in processing order (see :meth:`pixel_order`)."""
        x = self._x(x)
        B = self.nitems
        m = torch.empty((B, 2, 3, self.npix), dtype=torch.float64, device=self.device) if maps else None
        v = torch.empty(B, dtype=torch.float64, device=self.device)
        st = torch.empty(B, dtype=torch.int32, device=self.device)
        fn = load().cs_component_maps_sorted if sorted_order else load().cs_component_maps
        _check(fn(self._h, _ptr(x), _ptr(m), 0, _ptr(v), _ptr(st), _stream(self._stream)), "cs_component_maps")
        return m, v, st

    def pixel_order(self, item: int):
        """Caller's pixel index of each processing slot of an item (device int32 [n_included])."""
        n, _ = self.item_info(item)
        out = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        _check(load().cs_problem_pixel_order(self._h, item, _ptr(out), _stream(self._stream)),
               "cs_problem_pixel_order")
        return out[:n]

    def optimizer_state(self, m: int = 10) -> OptState:
        nb = C.c_size_t()
        _check(load().cs_optimizer_workspace_bytes(self._h, m, C.byref(nb)), "cs_optimizer_workspace_bytes")
        return OptState(nb.value, self.device)

    def cs_optimize_batch(self, lower, upper, x0, opts: OptimOpts | None = None, *, state: OptState | None = None,
                          resume: bool = False, max_replays: int = 0):
        """Batched bounded minimisation.  Without ``state`` a fresh workspace is used; with it
        the run keeps its state there, ``resume=True`` continues a run held in it, and
        ``max_replays > 0`` pauses after that many graph replays (items still running carry
        ``RUNNING``).  Returns ``dict(x, f, iters, status, nevals, running, state)``."""
        L = load()
        o = opts if opts is not None else default_opts()
        lo, hi = self._x(lower), self._x(upper)
        x = self._x(x0).clone() if x0 is not None else torch.empty(self.nparams, dtype=torch.float64,
                                                                   device=self.device)
        B = self.nitems
        f = torch.empty(B, dtype=torch.float64, device=self.device)
        it = torch.empty(B, dtype=torch.int32, device=self.device)
        st = torch.empty(B, dtype=torch.int32, device=self.device)
        ne = torch.empty(B, dtype=torch.int64, device=self.device)
        ws = state if state is not None else self.optimizer_state(o.m)
        running = C.c_int32(0)
        _check(L.cs_optimize_batch_run(self._h, C.byref(o), _ptr(lo), _ptr(hi), _ptr(x), _ptr(f), _ptr(it), _ptr(st),
                                       _ptr(ne), ws.ptr, ws.nbytes, int(resume), int(max_replays),
                                       C.byref(running), _stream(self._stream)), "cs_optimize_batch_run")
        return dict(x=x, f=f, iters=it, status=st, nevals=ne, running=running.value, state=ws)

    def get_schedule(self) -> Schedule:
        s = Schedule()
        _check(load().cs_problem_get_schedule(self._h, C.byref(s)), "cs_problem_get_schedule")
        return s

    def set_schedule(self, waves_per_block=2, blocks_per_cu=0, xcd_remap=1, shared_segments=2):
        s = Schedule(waves_per_block, blocks_per_cu, xcd_remap, shared_segments)
        _check(load().cs_problem_set_schedule(self._h, C.byref(s)), "cs_problem_set_schedule")

    def autotune(self, x, reps: int = 3) -> Schedule:
        x = self._x(x)
        f = torch.empty(self.nitems, dtype=torch.float64, device=self.device)
        g = torch.empty(self.nparams, dtype=torch.float64, device=self.device)
        s = Schedule()
        _check(load().cs_problem_autotune(self._h, _ptr(x), _ptr(f), _ptr(g), reps, C.byref(s), _stream(self._stream)),
               "cs_problem_autotune")
        return s

    def set_timing(self, enable: bool):
        _check(load().cs_problem_set_timing(self._h, int(enable)), "cs_problem_set_timing")

    def kernel_time(self):
        ms, n = C.c_double(), C.c_int64()
        _check(load().cs_problem_kernel_time(self._h, C.byref(ms), C.byref(n)), "cs_problem_kernel_time")
        return ms.value, n.value
