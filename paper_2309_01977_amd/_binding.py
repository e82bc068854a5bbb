"""ctypes binding of the HIP C ABI (include/spect.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the projector and of the OSEM update runs
in the library's kernels.  There is no CPU fallback: without the built
library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libspect_hip.so")

SPECT_OK = 0
SPECT_EINVAL = -1
SPECT_ENOMEM = -2
SPECT_EHIP = -3
SPECT_EUNSUPPORTED = -4
OP_FWD, OP_BACK, OP_SENS, OP_OSEM, OP_RECON, OP_BSREM_STEP, OP_BSREM = 0, 1, 2, 3, 4, 5, 6
OP_STEP, OP_STEP_VJP = 7, 8
ATT_TABLE = 2   # with_mu code of the attenuation-table calls

EXPORTS = ("spect_plan_create", "spect_plan_destroy", "spect_workspace_size", "spect_fwd", "spect_fwd_static",
           "spect_back", "spect_sensitivity", "spect_table_size", "spect_sensitivity_table",
           "spect_fwd_table", "spect_back_table", "osem_subset_step", "osem_list_step", "osem_list_step_vjp",
           "osem_reconstruct", "osem_reconstruct_ones",
           "spect_rdp_gradient", "bsrem_subset_step", "bsrem_reconstruct", "spect_batch_create",
           "spect_batch_destroy", "spect_batch_workspace_size", "osem_batch_reconstruct", "osem_batch_autotune",
           "spect_batch_schedule", "spect_batch_set_schedule", "spect_server_create", "spect_server_destroy",
           "spect_server_submit", "spect_server_progress", "spect_server_status", "spect_server_wait",
           "spect_server_forget", "spect_server_stats", "spect_profile_enable",
           "spect_profile_reset", "spect_profile_query", "spect_last_error")
KERNELS = ("tau_prepass", "fwd_main", "fwd_reduce", "back_rot", "back_gather", "fill_zero", "rdp_grad",
           "vol_sum", "fwd_batch", "reduce_batch", "back_batch", "gather_batch", "sens_line", "pad_columns")


class SpectError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"spect error {code}: {msg}")
        self.code = code


class Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nz", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("voxel_cm", ctypes.c_double),
                ("angles_deg", ctypes.POINTER(ctypes.c_double)),
                ("radius_cm", ctypes.POINTER(ctypes.c_double)),
                ("psf_a", ctypes.c_double), ("psf_b", ctypes.c_double),
                ("psf_nsigma", ctypes.c_double)]


_lib = None


def load_library(path: Optional[str] = None):
    """Load the built library (no fallback: raises if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} (run python -m paper_2309_01977_amd.build)")
    lib = ctypes.CDLL(p)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.spect_plan_create.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(vp)]
    lib.spect_plan_destroy.argtypes = [vp]
    lib.spect_workspace_size.argtypes = [vp, ctypes.c_int, i32, ctypes.c_int, ctypes.POINTER(sz)]
    lib.spect_fwd.argtypes = [vp, vp, vp, vp, i32p, i32, vp, sz, vp]
    lib.spect_fwd_static.argtypes = [vp, vp, vp, vp, i32p, i32, vp]
    lib.spect_back.argtypes = [vp, vp, vp, vp, i32p, i32, ctypes.c_int, vp, sz, vp]
    lib.spect_sensitivity.argtypes = [vp, vp, vp, i32p, i32, vp, sz, vp]
    lib.spect_table_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    lib.spect_sensitivity_table.argtypes = [vp, vp, vp, vp, i32p, i32, vp, sz, vp]
    lib.spect_fwd_table.argtypes = [vp, vp, vp, vp, i32p, i32, vp, sz, vp]
    lib.spect_back_table.argtypes = [vp, vp, vp, vp, i32p, i32, ctypes.c_int, vp, sz, vp]
    lib.osem_subset_step.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, vp, sz, vp]
    lib.osem_reconstruct.argtypes = [vp, vp, vp, vp, vp, i32, i32, vp, sz, vp]
    lib.osem_reconstruct_ones.argtypes = [vp, vp, vp, vp, vp, i32, i32, vp, sz, vp]
    lib.osem_list_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32p, i32, vp, sz, vp]
    lib.osem_list_step_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32p, i32, vp, vp, vp, sz, vp]
    f32 = ctypes.c_float
    lib.spect_rdp_gradient.argtypes = [vp, vp, vp, f32, vp]
    lib.bsrem_subset_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, i32, f32, f32, f32, vp, sz, vp]
    lib.bsrem_reconstruct.argtypes = [vp, vp, vp, vp, vp, i32, i32, f32, f32, ctypes.POINTER(f32), vp, sz, vp]
    vpp = ctypes.POINTER(vp)
    lib.spect_batch_create.argtypes = [vpp, i32, i32, ctypes.c_int, vpp]
    lib.spect_batch_destroy.argtypes = [vp]
    lib.spect_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.osem_batch_reconstruct.argtypes = [vp, vpp, vpp, vpp, vpp, i32, i32, vp, sz, vp]
    lib.osem_batch_autotune.argtypes = [vp, vpp, vpp, vpp, vpp, vp, sz, vp]
    lib.spect_batch_schedule.argtypes = [vp, i32p, ctypes.POINTER(ctypes.c_double)]
    lib.spect_batch_set_schedule.argtypes = [vp, i32]
    i64 = ctypes.c_int64
    lib.spect_server_create.argtypes = [i32, sz, vpp]
    lib.spect_server_destroy.argtypes = [vp]
    lib.spect_server_submit.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, vp, ctypes.POINTER(i64)]
    lib.spect_server_progress.argtypes = [vp, i32p, i32p]
    lib.spect_server_status.argtypes = [vp, i64, i32p]
    lib.spect_server_wait.argtypes = [vp, i64]
    lib.spect_server_forget.argtypes = [vp, i64]
    lib.spect_server_stats.argtypes = [vp, i32p, i32p, i32p, ctypes.POINTER(sz)]
    lib.spect_profile_enable.argtypes = [ctypes.c_int]
    lib.spect_profile_reset.argtypes = []
    lib.spect_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.spect_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(code: int):
    if code != SPECT_OK:
        raise SpectError(code, load_library().spect_last_error().decode())


def _ptr(t: Optional[torch.Tensor], shape: Tuple[int, ...], name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float32 tensor of shape {shape}, "
                         f"got {tuple(t.shape)} {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Immutable projector plan for one acquisition geometry (spect_plan)."""

    def __init__(self, n: int, nz: int, n_angles: int, voxel_cm: float, psf_a: float = 0.0,
                 psf_b: float = 0.0, psf_nsigma: float = 4.0,
                 angles_deg: Optional[Sequence[float]] = None,
                 radius_cm: Optional[Sequence[float]] = None):
        lib = load_library()
        self.n, self.nz, self.n_angles = int(n), int(nz), int(n_angles)
        self.voxel_cm = float(voxel_cm)
        self._ang = None if angles_deg is None else (ctypes.c_double * n_angles)(*angles_deg)
        self._rad = None if radius_cm is None else (ctypes.c_double * n_angles)(*radius_cm)
        g = Geometry(self.n, self.nz, self.n_angles, 0, self.voxel_cm,
                     ctypes.cast(self._ang, ctypes.POINTER(ctypes.c_double)) if self._ang else None,
                     ctypes.cast(self._rad, ctypes.POINTER(ctypes.c_double)) if self._rad else None,
                     float(psf_a), float(psf_b), float(psf_nsigma))
        h = ctypes.c_void_p()
        _check(lib.spect_plan_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h
        self._ws: Dict[Tuple[int, int, int, int], torch.Tensor] = {}

    @classmethod
    def for_workload(cls, w) -> "Plan":
        return cls(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)

    @property
    def object_shape(self):
        return (self.n, self.n, self.nz)

    @property
    def proj_shape(self):
        return (self.n_angles, self.n, self.nz)

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize()
            load_library().spect_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load_library().spect_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass

    @staticmethod
    def _mu_code(with_mu) -> int:
        if isinstance(with_mu, bool) or with_mu is None:
            return int(bool(with_mu))
        return int(with_mu)

    def workspace_size(self, op: int, n_idx: int, with_mu) -> int:
        """with_mu: False / True, or ATT_TABLE for the table calls."""
        b = ctypes.c_size_t()
        _check(load_library().spect_workspace_size(self._h, op, int(n_idx), self._mu_code(with_mu),
                                                   ctypes.byref(b)))
        return b.value

    def workspace(self, op: int, n_idx: int, with_mu) -> torch.Tensor:
        """The scratch of one call, kept for reuse per (op, size, attenuation
        mode, stream): calls on one stream run in order, calls on different
        streams get different scratch (two calls in flight at once must not
        share it)."""
        key = (op, int(n_idx), self._mu_code(with_mu), torch.cuda.current_stream().cuda_stream)
        ws = self._ws.get(key)
        if ws is None:
            nbytes = max(self.workspace_size(op, n_idx, with_mu), 256)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self._ws[key] = ws
        return ws

    def _idx(self, idx):
        if idx is None:
            return None, self.n_angles
        arr = (ctypes.c_int32 * len(idx))(*[int(i) for i in idx])
        return arr, len(idx)

    def forward(self, f: torch.Tensor, mu: Optional[torch.Tensor] = None, idx=None,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Rows idx of H f (spect_fwd); other rows of ``out`` are untouched."""
        if out is None:
            out = torch.zeros(self.proj_shape, dtype=torch.float32, device=f.device)
        arr, n = self._idx(idx)
        ws = self.workspace(OP_FWD, max(n, 1), mu is not None)
        _check(load_library().spect_fwd(self._h, _ptr(f, self.object_shape, "f"),
                                         _ptr(mu, self.object_shape, "mu"),
                                         _ptr(out, self.proj_shape, "proj"), arr, n,
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
        return out

    def forward_static(self, f: torch.Tensor, mu: Optional[torch.Tensor] = None, idx=None,
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Rows idx of H f through spect_fwd_static: no workspace, the
        library's fixed scratch array (calls on one device must not overlap)."""
        if out is None:
            out = torch.zeros(self.proj_shape, dtype=torch.float32, device=f.device)
        arr, n = self._idx(idx)
        _check(load_library().spect_fwd_static(self._h, _ptr(f, self.object_shape, "f"),
                                                _ptr(mu, self.object_shape, "mu"),
                                                _ptr(out, self.proj_shape, "proj"), arr, n, _stream()))
        return out

    def back(self, proj: torch.Tensor, mu: Optional[torch.Tensor] = None, idx=None,
             out: Optional[torch.Tensor] = None, accumulate: bool = False) -> torch.Tensor:
        """sum over n in idx of H_n^T proj[n] (spect_back)."""
        if out is None:
            out = torch.empty(self.object_shape, dtype=torch.float32, device=proj.device)
            accumulate = False
        arr, n = self._idx(idx)
        ws = self.workspace(OP_BACK, max(n, 1), mu is not None)
        _check(load_library().spect_back(self._h, _ptr(proj, self.proj_shape, "proj"),
                                          _ptr(mu, self.object_shape, "mu"),
                                          _ptr(out, self.object_shape, "f_out"), arr, n,
                                          int(bool(accumulate)), ctypes.c_void_p(ws.data_ptr()),
                                          ws.numel(), _stream()))
        return out

    def sensitivity(self, mu: Optional[torch.Tensor] = None, idx=None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """H_idx^T 1 (spect_sensitivity)."""
        if out is None:
            out = torch.empty(self.object_shape, dtype=torch.float32, device="cuda")
        arr, n = self._idx(idx)
        ws = self.workspace(OP_SENS, max(n, 1), mu is not None)
        _check(load_library().spect_sensitivity(self._h, _ptr(mu, self.object_shape, "mu"),
                                                 _ptr(out, self.object_shape, "sens"), arr, n,
                                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                                 _stream()))
        return out

    # ------------------------------------------------ attenuation tables --

    def table_size(self, n_idx: int) -> int:
        b = ctypes.c_size_t()
        _check(load_library().spect_table_size(self._h, int(n_idx), ctypes.byref(b)))
        return b.value

    def _table(self, table: torch.Tensor, n: int) -> ctypes.c_void_p:
        if not isinstance(table, torch.Tensor) or table.device.type != "cuda" or table.dtype != torch.float32:
            raise TypeError("table must be a float32 CUDA tensor")
        if not table.is_contiguous() or table.numel() * 4 < self.table_size(n):
            raise ValueError(f"table must be contiguous with at least {self.table_size(n)} bytes")
        return ctypes.c_void_p(table.data_ptr())

    def new_table(self, n_idx: int) -> torch.Tensor:
        return torch.empty(self.table_size(n_idx) // 4, dtype=torch.float32, device="cuda")

    def sensitivity_table(self, mu: torch.Tensor, idx=None, out: Optional[torch.Tensor] = None,
                          table: Optional[torch.Tensor] = None):
        """(H_idx^T 1, attenuation-factor table of the listed angles) (spect_sensitivity_table)."""
        arr, n = self._idx(idx)
        if out is None:
            out = torch.empty(self.object_shape, dtype=torch.float32, device="cuda")
        if table is None:
            table = self.new_table(n)
        ws = self.workspace(OP_SENS, max(n, 1), ATT_TABLE)
        _check(load_library().spect_sensitivity_table(
            self._h, _ptr(mu, self.object_shape, "mu"), _ptr(out, self.object_shape, "sens"),
            self._table(table, n), arr, n, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
        return out, table

    def forward_table(self, f: torch.Tensor, table: torch.Tensor, idx=None,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Rows idx of H f with the factors of ``table`` (spect_fwd_table)."""
        if out is None:
            out = torch.zeros(self.proj_shape, dtype=torch.float32, device=f.device)
        arr, n = self._idx(idx)
        ws = self.workspace(OP_FWD, max(n, 1), ATT_TABLE)
        _check(load_library().spect_fwd_table(self._h, _ptr(f, self.object_shape, "f"), self._table(table, n),
                                               _ptr(out, self.proj_shape, "proj"), arr, n,
                                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
        return out

    def back_table(self, proj: torch.Tensor, table: torch.Tensor, idx=None,
                   out: Optional[torch.Tensor] = None, accumulate: bool = False) -> torch.Tensor:
        """sum over n in idx of H_n^T proj[n] with the factors of ``table`` (spect_back_table)."""
        if out is None:
            out = torch.empty(self.object_shape, dtype=torch.float32, device=proj.device)
            accumulate = False
        arr, n = self._idx(idx)
        ws = self.workspace(OP_BACK, max(n, 1), ATT_TABLE)
        _check(load_library().spect_back_table(self._h, _ptr(proj, self.proj_shape, "proj"),
                                                self._table(table, n), _ptr(out, self.object_shape, "f_out"),
                                                arr, n, int(bool(accumulate)), ctypes.c_void_p(ws.data_ptr()),
                                                ws.numel(), _stream()))
        return out

    def osem_subset_step(self, f: torch.Tensor, g: torch.Tensor, sens_m: torch.Tensor, m: int,
                         n_subsets: int, mu: Optional[torch.Tensor] = None,
                         s_add: Optional[torch.Tensor] = None) -> torch.Tensor:
        """One OSEM subiteration on subset m, f updated in place."""
        ws = self.workspace(OP_OSEM, n_subsets, mu is not None)
        _check(load_library().osem_subset_step(
            self._h, _ptr(f, self.object_shape, "f"), _ptr(mu, self.object_shape, "mu"),
            _ptr(g, self.proj_shape, "g"), _ptr(s_add, self.proj_shape, "s_add"),
            _ptr(sens_m, self.object_shape, "sens_m"), int(m), int(n_subsets),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
        return f


def _step_att(mu, table):
    """with_mu code of the subiteration calls: a table, a map or neither."""
    if mu is not None and table is not None:
        raise ValueError("pass an attenuation map or a table, not both")
    return ATT_TABLE if table is not None else int(mu is not None)


def _osem_list_step(self, f: torch.Tensor, g: torch.Tensor, sens: torch.Tensor, idx,
                    mu: Optional[torch.Tensor] = None, table: Optional[torch.Tensor] = None,
                    s_add: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One OSEM subiteration over the angle list idx (osem_list_step): returns
    out = f * H^T(g / (H f + s)) / sens (f where sens = 0); out may be f."""
    if out is None:
        out = torch.empty(self.object_shape, dtype=torch.float32, device=f.device)
    arr, n = self._idx(idx)
    code = _step_att(mu, table)
    ws = self.workspace(OP_STEP, max(n, 1), code)
    _check(load_library().osem_list_step(
        self._h, _ptr(f, self.object_shape, "f"), _ptr(out, self.object_shape, "f_out"),
        _ptr(mu, self.object_shape, "mu"), None if table is None else self._table(table, n),
        _ptr(g, self.proj_shape, "g"), _ptr(s_add, self.proj_shape, "s_add"),
        _ptr(sens, self.object_shape, "sens"), arr, n, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


def _osem_list_step_vjp(self, f: torch.Tensor, g: torch.Tensor, sens: torch.Tensor, idx,
                        grad_out: torch.Tensor, mu: Optional[torch.Tensor] = None,
                        table: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """(d osem_list_step / d f)^T grad_out (osem_list_step_vjp); out may be grad_out."""
    if out is None:
        out = torch.empty(self.object_shape, dtype=torch.float32, device=f.device)
    arr, n = self._idx(idx)
    code = _step_att(mu, table)
    ws = self.workspace(OP_STEP_VJP, max(n, 1), code)
    _check(load_library().osem_list_step_vjp(
        self._h, _ptr(f, self.object_shape, "f"), _ptr(mu, self.object_shape, "mu"),
        None if table is None else self._table(table, n), _ptr(g, self.proj_shape, "g"),
        _ptr(s_add, self.proj_shape, "s_add"), _ptr(sens, self.object_shape, "sens"), arr, n,
        _ptr(grad_out, self.object_shape, "grad_out"), _ptr(out, self.object_shape, "grad_f"),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


Plan.osem_list_step = _osem_list_step
Plan.osem_list_step_vjp = _osem_list_step_vjp


class KernelTimer:
    """Per-kernel HIP-event timing of the library's launches (spect_profile_*).

    with KernelTimer() as kt:
        ...library calls...
    kt.stats()  -> {kernel: (launches, total_ms)}
    """

    def __enter__(self):
        lib = load_library()
        _check(lib.spect_profile_reset())
        _check(lib.spect_profile_enable(1))
        return self

    def __exit__(self, *exc):
        _check(load_library().spect_profile_enable(0))
        return False

    def stats(self):
        lib = load_library()
        out = {}
        for k in KERNELS:
            n, ms = ctypes.c_int32(), ctypes.c_double()
            _check(lib.spect_profile_query(k.encode(), ctypes.byref(n), ctypes.byref(ms)))
            if n.value:
                out[k] = (n.value, ms.value)
        _check(lib.spect_profile_reset())
        return out


def _recon_method(self, g: torch.Tensor, n_iters: int, n_subsets: int,
                  mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                  f: Optional[torch.Tensor] = None, from_ones: bool = False) -> torch.Tensor:
    """Whole OSEM reconstruction: f holds the initial image and receives the
    result (osem_reconstruct); with from_ones, or when f is None, the start
    image is 1 everywhere and f is only written (osem_reconstruct_ones)."""
    if f is None:
        f = torch.empty(self.object_shape, dtype=torch.float32, device=g.device)
        from_ones = True
    ws = self.workspace(OP_RECON, n_subsets, mu is not None)
    lib = load_library()
    fn = lib.osem_reconstruct_ones if from_ones else lib.osem_reconstruct
    _check(fn(
        self._h, _ptr(f, self.object_shape, "f"), _ptr(mu, self.object_shape, "mu"),
        _ptr(g, self.proj_shape, "g"), _ptr(s_add, self.proj_shape, "s_add"), int(n_iters),
        int(n_subsets), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return f


Plan.reconstruct = _recon_method


def subset_angles(n_angles: int, n_subsets: int, m: int):
    """Interleaved subset m = {n : n mod M = m}."""
    return list(range(m, n_angles, n_subsets))


def _rdp_gradient(self, f: torch.Tensor, gamma: float = 2.0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gradient of the relative difference prior at f (spect_rdp_gradient)."""
    if out is None:
        out = torch.empty(self.object_shape, dtype=torch.float32, device=f.device)
    _check(load_library().spect_rdp_gradient(self._h, _ptr(f, self.object_shape, "f"),
                                             _ptr(out, self.object_shape, "grad"), float(gamma), _stream()))
    return out


def _bsrem_step(self, f: torch.Tensor, g: torch.Tensor, sens_m: torch.Tensor, sens_all: torch.Tensor, m: int,
                n_subsets: int, alpha: float, beta: float = 0.3, gamma: float = 2.0,
                mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One BSREM-RDP subiteration on subset m, f updated in place (bsrem_subset_step)."""
    ws = self.workspace(OP_BSREM_STEP, n_subsets, mu is not None)
    _check(load_library().bsrem_subset_step(
        self._h, _ptr(f, self.object_shape, "f"), _ptr(mu, self.object_shape, "mu"),
        _ptr(g, self.proj_shape, "g"), _ptr(s_add, self.proj_shape, "s_add"),
        _ptr(sens_m, self.object_shape, "sens_m"), _ptr(sens_all, self.object_shape, "sens_all"), int(m),
        int(n_subsets), float(alpha), float(beta), float(gamma), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        _stream()))
    return f


def _bsrem_method(self, g: torch.Tensor, n_iters: int, n_subsets: int, mu: Optional[torch.Tensor] = None,
                  s_add: Optional[torch.Tensor] = None, f: Optional[torch.Tensor] = None, beta: float = 0.3,
                  gamma: float = 2.0, relaxation: Optional[Sequence[float]] = None) -> torch.Tensor:
    """Whole BSREM-RDP reconstruction (bsrem_reconstruct); f holds the initial
    image (1 everywhere if None) and receives the result."""
    if f is None:
        f = torch.ones(self.object_shape, dtype=torch.float32, device=g.device)
    rel = None
    if relaxation is not None:
        if len(relaxation) < n_iters:
            raise ValueError("relaxation needs one value per iteration")
        rel = (ctypes.c_float * len(relaxation))(*[float(a) for a in relaxation])
    ws = self.workspace(OP_BSREM, n_subsets, mu is not None)
    _check(load_library().bsrem_reconstruct(
        self._h, _ptr(f, self.object_shape, "f"), _ptr(mu, self.object_shape, "mu"),
        _ptr(g, self.proj_shape, "g"), _ptr(s_add, self.proj_shape, "s_add"), int(n_iters), int(n_subsets),
        float(beta), float(gamma), rel, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return f


Plan.rdp_gradient = _rdp_gradient
Plan.bsrem_subset_step = _bsrem_step
Plan.bsrem = _bsrem_method


BATCH_EAGER = 1


class Batch:
    """Batched OSEM over several geometries (spect_batch_*).

    batch = Batch([plan_a, plan_b, ...], n_subsets=8, with_mu=True)
    batch.autotune(fs, mus, gs)               # optional: pick the fastest schedule
    batch.reconstruct(fs, mus, gs, n_iters)   # fs updated in place
    """

    def __init__(self, plans: Sequence[Plan], n_subsets: int, with_mu: bool):
        lib = load_library()
        self.plans = list(plans)
        self.n_subsets = int(n_subsets)
        self.with_mu = bool(with_mu)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.spect_batch_create(arr, len(self.plans), self.n_subsets, int(self.with_mu), ctypes.byref(h)))
        self._h = h
        b = ctypes.c_size_t()
        _check(lib.spect_batch_workspace_size(self._h, ctypes.byref(b)))
        self.workspace_bytes = b.value
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            load_library().spect_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _arrays(self, fs, mus, gs, ss):
        R = len(self.plans)
        if len(fs) != R or len(gs) != R:
            raise ValueError(f"need {R} images and {R} data sets")
        fa = (ctypes.c_void_p * R)(*[_ptr(f, p.object_shape, "f").value for f, p in zip(fs, self.plans)])
        ga = (ctypes.c_void_p * R)(*[_ptr(g, p.proj_shape, "g").value for g, p in zip(gs, self.plans)])
        ma = None if mus is None else (ctypes.c_void_p * R)(
            *[_ptr(m, p.object_shape, "mu").value for m, p in zip(mus, self.plans)])
        sa = None if ss is None else (ctypes.c_void_p * R)(
            *[None if s is None else _ptr(s, p.proj_shape, "s_add").value for s, p in zip(ss, self.plans)])
        if self._ws is None:
            self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
        return fa, ma, ga, sa

    def reconstruct(self, fs, mus, gs, n_iters: int, s_adds=None, eager: bool = False):
        fa, ma, ga, sa = self._arrays(fs, mus, gs, s_adds)
        _check(load_library().osem_batch_reconstruct(self._h, fa, ma, ga, sa, int(n_iters),
                                                      BATCH_EAGER if eager else 0,
                                                      ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                                      _stream()))
        return fs

    def autotune(self, fs, mus, gs, s_adds=None):
        fa, ma, ga, sa = self._arrays(fs, mus, gs, s_adds)
        _check(load_library().osem_batch_autotune(self._h, fa, ma, ga, sa, ctypes.c_void_p(self._ws.data_ptr()),
                                                   self._ws.numel(), _stream()))
        return self.schedule()

    def schedule(self):
        """(schedule, [ms per iteration of each candidate, -1 if not timed])."""
        s = ctypes.c_int32()
        ms = (ctypes.c_double * 8)()
        _check(load_library().spect_batch_schedule(self._h, ctypes.byref(s), ms))
        return s.value, list(ms)

    def set_schedule(self, schedule: int):
        _check(load_library().spect_batch_set_schedule(self._h, int(schedule)))


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class Server:
    """Reconstruction server (spect_server_*): whole OSEM reconstructions
    admitted as slots and pool memory free up, overlapping on the device."""

    def __init__(self, n_slots: int, pool_bytes: int):
        h = ctypes.c_void_p()
        _check(load_library().spect_server_create(int(n_slots), int(pool_bytes), ctypes.byref(h)))
        self._h = h
        self._keep = {}   # request id -> tensors that must stay alive until it finishes

    def close(self):
        if getattr(self, "_h", None):
            load_library().spect_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, plan: Plan, f: torch.Tensor, g: torch.Tensor, n_iters: int, n_subsets: int,
               mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None) -> int:
        rid = ctypes.c_int64()
        _check(load_library().spect_server_submit(
            self._h, plan._h, _ptr(f, plan.object_shape, "f"), _ptr(mu, plan.object_shape, "mu"),
            _ptr(g, plan.proj_shape, "g"), _ptr(s_add, plan.proj_shape, "s_add"), int(n_iters), int(n_subsets),
            _stream(), ctypes.byref(rid)))
        self._keep[rid.value] = (plan, f, g, mu, s_add)
        return rid.value

    def progress(self):
        """(running, queued) after retiring finished requests and admitting."""
        nr, nq = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().spect_server_progress(self._h, ctypes.byref(nr), ctypes.byref(nq)))
        return nr.value, nq.value

    def status(self, rid: int) -> int:
        st = ctypes.c_int32()
        _check(load_library().spect_server_status(self._h, int(rid), ctypes.byref(st)))
        if st.value == REQ_DONE:
            self._keep.pop(rid, None)
        return st.value

    def wait(self, rid: int):
        _check(load_library().spect_server_wait(self._h, int(rid)))
        self._keep.pop(rid, None)

    def forget(self, rid: int):
        _check(load_library().spect_server_forget(self._h, int(rid)))

    def stats(self):
        """(running, queued, peak running, pool bytes in use)."""
        nr, nq, pk = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        used = ctypes.c_size_t()
        _check(load_library().spect_server_stats(self._h, ctypes.byref(nr), ctypes.byref(nq), ctypes.byref(pk),
                                                  ctypes.byref(used)))
        return nr.value, nq.value, pk.value, used.value
