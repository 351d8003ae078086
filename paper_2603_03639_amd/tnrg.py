"""ctypes binding of libtnrg (include/tnrg.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch supplies device memory and the stream.  Importing this
module fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtnrg.so")

(OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENONFINITE, EOVERFLOW, EUNSUPPORTED,
 ESTALE) = 0, -1, -2, -3, -4, -5, -6, -7, -8
FLAG_OVERFLOW, FLAG_NOCONV, FLAG_NONFINITE, FLAG_STALE = 1, 2, 4, 8
PHASES = ("load", "theta", "lq", "jacobi", "finish", "env_left", "env_right", "total")
CLOCK_HZ = 100e6  # constant-rate counter behind the phase ticks


class TnrgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tnrg error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
    return ctypes.CDLL(LIB_PATH)


_lib = _load()


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class _Model(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("dt", ctypes.c_double),
                ("chi", ctypes.c_int32), ("trunc_eps", ctypes.c_double),
                ("renormalize", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("profile", ctypes.c_int32),
                ("zz_mask", ctypes.POINTER(ctypes.c_uint8)),
                ("xt_mask", ctypes.POINTER(ctypes.c_uint8)),
                ("split_order", ctypes.c_int32),
                ("xt_model", ctypes.c_int32)]


class _Batch(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("dcap", ctypes.c_int32), ("bond_dim", ctypes.c_void_p),
                ("data", ctypes.c_void_p)]


class _Request(ctypes.Structure):
    _fields_ = [("md", ctypes.POINTER(_Model)), ("ux", ctypes.c_void_p),
                ("uy", ctypes.c_void_p), ("uzz", ctypes.c_void_p), ("K", ctypes.c_int32),
                ("J", ctypes.c_void_p), ("R", ctypes.c_int32),
                ("inputs", ctypes.POINTER(_Batch)), ("targets", ctypes.POINTER(_Batch)),
                ("dcap", ctypes.c_int32), ("F", ctypes.c_void_p), ("g_ux", ctypes.c_void_p),
                ("g_uy", ctypes.c_void_p), ("g_uzz", ctypes.c_void_p),
                ("overlaps", ctypes.c_void_p)]


class _Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32),
                ("dcap", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("running", ctypes.c_int32),
                ("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("regrown", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("arena_bytes", ctypes.c_size_t),
                ("arena_free", ctypes.c_size_t), ("arena_largest_free", ctypes.c_size_t)]


_vp, _i32, _i64, _sz, _dp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_size_t, ctypes.c_void_p)
_MP = ctypes.POINTER(_Model)
_BP = ctypes.POINTER(_Batch)
_SP = ctypes.c_void_p  # tnrg_server*

_SIGS = {
    "tnrg_bond_cap": (_i32, [_i32, _i32, _i32]),
    "tnrg_mps_site_offset": (_i64, [_i32, _i32, _i32]),
    "tnrg_mps_traj_elems": (_i64, [_i32, _i32]),
    "mps_evolve_workspace_bytes": (_sz, [_MP, _i32, _i32]),
    "mps_evolve": (ctypes.c_int, [_MP, _dp, _dp, _dp, _dp, _i32, _i32, _i32, _BP, _vp, _sz, _vp]),
    "mps_overlap_workspace_bytes": (_sz, [_i32, _i32, _i32]),
    "mps_overlap": (ctypes.c_int, [_BP, _BP, _vp, _vp, _sz, _vp]),
    "grape_workspace_bytes": (_sz, [_MP, _i32, _i32, _i32, _i32]),
    "grape_fidelity_grad": (ctypes.c_int, [_MP, _dp, _dp, _dp, _i32, _dp, _i32, _BP, _BP,
                                           _i32, _i32, _dp, _dp, _dp, _dp, _vp, _vp, _vp,
                                           _sz, _vp]),
    "grape_forward": (ctypes.c_int, [_MP, _dp, _dp, _dp, _i32, _dp, _i32, _BP, _BP, _i32, _i32,
                                     _dp, _vp, _vp, _sz, _vp]),
    "grape_backward": (ctypes.c_int, [_MP, _dp, _dp, _dp, _i32, _dp, _i32, _BP, _BP, _i32,
                                      _i32, _dp, _dp, _dp, _vp, _vp, _sz, _vp]),
    "tnrg_status": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int64), _vp]),
    "tnrg_server_create": (ctypes.c_int, [_vp, _sz, _i32, _i32, _i32, ctypes.POINTER(_SP)]),
    "tnrg_server_submit": (ctypes.c_int, [_SP, ctypes.POINTER(_Request),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "tnrg_server_progress": (ctypes.c_int, [_SP, ctypes.POINTER(_Completion), _i32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "tnrg_server_cancel_queued": (ctypes.c_int, [_SP, ctypes.POINTER(ctypes.c_int64), _i32,
                                                 ctypes.POINTER(ctypes.c_int32)]),
    "tnrg_server_info_get": (ctypes.c_int, [_SP, ctypes.POINTER(_ServerInfo)]),
    "tnrg_server_destroy": (ctypes.c_int, [_SP]),
    "tnrg_plan_set_threads": (ctypes.c_int, [_i32, _i32]),
    "tnrg_plan_set_jacobi_lds": (ctypes.c_int, [_i32]),
    "tnrg_plan_threads": (_i32, [_i32]),
    "tnrg_last_error": (ctypes.c_char_p, []),
    "tnrg_version": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = tuple(_SIGS)


def version() -> str:
    return _lib.tnrg_version().decode()


def _check(rc: int):
    if rc != OK:
        raise TnrgError(rc, _lib.tnrg_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------
@dataclass
class Model:
    """Problem statement of the C ABI (tnrg_model)."""
    N: int
    M: int
    dt: float
    chi: int
    eps: float = 1e-12
    renormalize: bool = True
    max_sweeps: int = 0
    profile: bool = False
    zz_mask: Optional[np.ndarray] = None
    xt_mask: Optional[np.ndarray] = None
    order: int = 2  # Trotter split: 2 (R Z R) or 1 (the first-order X Y Z)
    xt_model: int = 0  # crosstalk: 0 = J ZZ, 1 = J^x XX + J^y YY + J^z ZZ (Sec. III Eq. 9)

    def check_J(self, J, rows: int) -> None:
        """J must be [rows][N-1] (xt_model 0) or [rows][N-1][3] (xt_model 1)."""
        want = (rows, self.N - 1) + ((3,) if self.xt_model == 1 else ())
        if tuple(J.shape) != want:
            raise ValueError(f"J has shape {tuple(J.shape)}, the model needs {want}")

    def c(self) -> _Model:
        zz = np.ascontiguousarray(self.zz_mask if self.zz_mask is not None
                                  else np.zeros(self.N - 1), np.uint8)
        xt = np.ascontiguousarray(self.xt_mask if self.xt_mask is not None
                                  else np.zeros(self.N - 1), np.uint8)
        m = _Model(self.N, self.M, float(self.dt), self.chi, float(self.eps),
                   1 if self.renormalize else 0, int(self.max_sweeps),
                   1 if self.profile else 0,
                   zz.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                   xt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(self.order),
                   int(self.xt_model))
        m._keep = (zz, xt)
        return m

    @classmethod
    def from_problem(cls, p, **kw) -> "Model":
        return cls(N=p.N, M=p.M, dt=p.dt, chi=p.chi, eps=p.eps,
                   renormalize=p.renormalize, zz_mask=p.zz_mask,
                   xt_mask=p.xt_mask, order=getattr(p, "order", 2),
                   xt_model=1 if getattr(p, "xt_model", "zz") == "heisenberg" else 0, **kw)


def bond_cap(N: int, dcap: int, b: int) -> int:
    return int(_lib.tnrg_bond_cap(N, dcap, b))


def traj_elems(N: int, dcap: int) -> int:
    return int(_lib.tnrg_mps_traj_elems(N, dcap))


def site_offset(N: int, dcap: int, j: int) -> int:
    return int(_lib.tnrg_mps_site_offset(N, dcap, j))


class MPSBatch:
    """Device batch of MPS in the fixed-capacity layout of tnrg_mps_batch."""

    def __init__(self, N: int, n_traj: int, dcap: int, device="cuda",
                 data: Optional[torch.Tensor] = None,
                 dims: Optional[torch.Tensor] = None):
        self.N, self.n_traj, self.dcap = N, n_traj, dcap
        self.elems = traj_elems(N, dcap)
        self.data = data if data is not None else torch.zeros(
            (n_traj, self.elems), dtype=torch.complex128, device=device)
        self.dims = dims if dims is not None else torch.ones(
            (n_traj, N + 1), dtype=torch.int32, device=device)
        self._max_dim = None if dims is not None else 1

    @property
    def max_dim(self) -> int:
        """Largest bond dimension in the batch (read from the device once
        unless the batch was built from host tensors)."""
        if self._max_dim is None:
            self._max_dim = int(self.dims.max())
        return self._max_dim

    def c(self) -> _Batch:
        return _Batch(self.n_traj, self.N, self.dcap, self.dims.data_ptr(),
                      self.data.data_ptr())

    @classmethod
    def from_mps(cls, states: Sequence[List[np.ndarray]], dcap: Optional[int] = None,
                 device="cuda") -> "MPSBatch":
        """Pack host MPS (lists of (Dl, 2, Dr) arrays) into the device layout."""
        N = len(states[0])
        if dcap is None:
            dcap = max(max(a.shape[0] for a in s) for s in states)
            dcap = max(dcap, max(max(a.shape[2] for a in s) for s in states))
        elems = traj_elems(N, dcap)
        host = np.zeros((len(states), elems), np.complex128)
        dims = np.ones((len(states), N + 1), np.int32)
        for t, s in enumerate(states):
            for j, A in enumerate(s):
                Dl, _, Dr = A.shape
                cr = bond_cap(N, dcap, j + 1)
                if Dl > bond_cap(N, dcap, j) or Dr > cr:
                    raise ValueError(f"site {j} dims {A.shape} exceed capacity {dcap}")
                o = site_offset(N, dcap, j)
                blk = np.zeros((Dl * 2, cr), np.complex128)
                blk[:, :Dr] = A.reshape(Dl * 2, Dr)
                host[t, o:o + Dl * 2 * cr] = blk.reshape(-1)
                dims[t, j] = Dl
                dims[t, j + 1] = Dr
        out = cls(N, len(states), dcap, device,
                  torch.from_numpy(host).to(device), torch.from_numpy(dims).to(device))
        out._max_dim = int(dims.max())
        return out

    @classmethod
    def from_product(cls, vecs, device="cuda") -> "MPSBatch":
        """Bond-1 batch of product states: vecs[t][j] is the 2-vector of qubit j."""
        vecs = np.asarray(vecs, np.complex128)
        n_traj, N, _ = vecs.shape
        return cls.from_mps([[vecs[t, j].reshape(1, 2, 1) for j in range(N)]
                             for t in range(n_traj)], dcap=1, device=device)

    def to_mps(self) -> List[List[np.ndarray]]:
        host = self.data.cpu().numpy()
        dims = self.dims.cpu().numpy()
        out = []
        for t in range(self.n_traj):
            s = []
            for j in range(self.N):
                Dl, Dr = int(dims[t, j]), int(dims[t, j + 1])
                cr = bond_cap(self.N, self.dcap, j + 1)
                o = site_offset(self.N, self.dcap, j)
                blk = host[t, o:o + Dl * 2 * cr].reshape(Dl * 2, cr)[:, :Dr]
                s.append(blk.reshape(Dl, 2, Dr).copy())
            out.append(s)
        return out


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def status(ws: torch.Tensor, n_traj: int, stream=None, raise_on_error=True):
    flags = np.zeros(n_traj, np.int32)
    stats = np.zeros(18, np.int64)
    rc = _lib.tnrg_status(_ptr(ws), n_traj,
                          flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          stats.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          _stream(stream))
    info = dict(rc=rc, flags=flags, max_dim=int(stats[0]), max_sweeps=int(stats[1]),
                total_sweeps=int(stats[2]), n_svd=int(stats[3]),
                jacobi_flops=int(stats[4]), contraction_flops=int(stats[5]),
                phase_ticks=dict(zip(PHASES, (int(x) for x in stats[6:14]))),
                jacobi_rounds=int(stats[14]), lq_steps=int(stats[15]),
                jacobi_round_ticks=int(stats[16]), jacobi_sweep_end_ticks=int(stats[17]))
    if raise_on_error and rc != OK:
        raise TnrgError(rc, _lib.tnrg_last_error().decode())
    return info


def _f64(x, device):
    return torch.as_tensor(np.ascontiguousarray(x, np.float64) if isinstance(x, np.ndarray) else x,
                           dtype=torch.float64, device=device).contiguous()


# ----------------------------------------------------------------------------
def mps_evolve(model: Model, ux, uy, uzz, J, psi: MPSBatch, l_begin=0, l_end=None,
               adjoint=False, stream=None, check=True):
    """In-place evolution of a batch (J: [n_traj][N-1], or [n_traj][N-1][3]
    with Heisenberg crosstalk)."""
    dev = psi.data.device
    l_end = model.M if l_end is None else l_end
    ux, uy, uzz, J = (_f64(a, dev) for a in (ux, uy, uzz, J))
    model.check_J(J, psi.n_traj)
    cm = model.c()
    nbytes = _lib.mps_evolve_workspace_bytes(ctypes.byref(cm), psi.n_traj, psi.dcap)
    ws = _workspace(nbytes, dev)
    bc = psi.c()
    _check(_lib.mps_evolve(ctypes.byref(cm), _ptr(ux), _ptr(uy), _ptr(uzz), _ptr(J),
                           l_begin, l_end, 1 if adjoint else 0, ctypes.byref(bc),
                           _ptr(ws), ws.numel(), _stream(stream)))
    if check:
        return status(ws, psi.n_traj, stream)
    return ws


def mps_overlap(bra: MPSBatch, ket: MPSBatch, stream=None) -> torch.Tensor:
    dev = ket.data.device
    out = torch.empty(ket.n_traj, dtype=torch.complex128, device=dev)
    ws = _workspace(_lib.mps_overlap_workspace_bytes(ket.n_traj, ket.N,
                                                     max(ket.dcap, bra.dcap)), dev)
    b, k = bra.c(), ket.c()
    _check(_lib.mps_overlap(ctypes.byref(b), ctypes.byref(k), _ptr(out), _ptr(ws),
                            ws.numel(), _stream(stream)))
    return out


# Capacity buckets tried in order when a bond outgrows the current one; the
# last working bucket per problem shape is remembered (the chi-bucket plan).
# Buckets up to 32 keep the working buffers in LDS, 64 and 128 in global
# scratch.
BUCKETS = (4, 8, 16, 32, 64, 128)
_plan_cache = {}


def _bucket_sequence(model: Model, start: Optional[int], floor: int = 1):
    """Capacities to try: the buckets up to min(chi, 2^(N/2)), none below
    ``floor`` (the largest bond of the inputs and targets, which the states
    must hold before their first truncation to chi)."""
    cap_max = max(min(model.chi, 2 ** min(model.N // 2, 30)), floor)
    seq = [b for b in BUCKETS if floor <= b < cap_max] + [cap_max]
    if start is not None:
        seq = [b for b in seq if b >= start] or [cap_max]
    return seq


def grape_workspace_bytes(model: Model, K: int, R: int, dcap: int, ckpt_stride: int = 0) -> int:
    cm = model.c()
    return int(_lib.grape_workspace_bytes(ctypes.byref(cm), K, R, dcap, ckpt_stride))


class GrapeCall:
    """One prepared fidelity+gradient evaluation with its device buffers.

    The workspace and outputs are allocated once; ``run()`` launches the
    persistent kernel (asynchronously) and ``check()`` reads the device flags.
    """

    def __init__(self, model: Model, K: int, R: int, inputs: MPSBatch,
                 targets: MPSBatch, dcap: int, ckpt_stride: int = 0,
                 want_traj_dO: bool = False, device="cuda"):
        self.model, self.K, self.R = model, K, R
        self.inputs, self.targets = inputs, targets
        self.dcap, self.ckpt_stride = dcap, ckpt_stride
        self.cm = model.c()
        N, M = model.N, model.M
        self.nctrl = 2 * M * N + M * (N - 1)
        self.ws = _workspace(grape_workspace_bytes(model, K, R, dcap, ckpt_stride), device)
        self.F = torch.zeros(1, dtype=torch.float64, device=device)
        self.g_ux = torch.zeros((M, N), dtype=torch.float64, device=device)
        self.g_uy = torch.zeros((M, N), dtype=torch.float64, device=device)
        self.g_uzz = torch.zeros((M, N - 1), dtype=torch.float64, device=device)
        self.overlaps = torch.zeros(K * R, dtype=torch.complex128, device=device)
        self.traj_dO = (torch.zeros((K * R, self.nctrl), dtype=torch.complex128, device=device)
                        if want_traj_dO else None)
        self._bin, self._btg = inputs.c(), targets.c()

    def run(self, ux, uy, uzz, J, stream=None):
        _check(_lib.grape_fidelity_grad(
            ctypes.byref(self.cm), _ptr(ux), _ptr(uy), _ptr(uzz), self.K, _ptr(J), self.R,
            ctypes.byref(self._bin), ctypes.byref(self._btg), self.dcap, self.ckpt_stride,
            _ptr(self.F), _ptr(self.g_ux), _ptr(self.g_uy), _ptr(self.g_uzz),
            _ptr(self.overlaps), _ptr(self.traj_dO), _ptr(self.ws), self.ws.numel(),
            _stream(stream)))

    def forward(self, ux, uy, uzz, J, stream=None):
        """Forward propagation only: F and the overlaps; the checkpoints stay
        in this call's workspace for ``backward()``."""
        _check(_lib.grape_forward(
            ctypes.byref(self.cm), _ptr(ux), _ptr(uy), _ptr(uzz), self.K, _ptr(J), self.R,
            ctypes.byref(self._bin), ctypes.byref(self._btg), self.dcap, self.ckpt_stride,
            _ptr(self.F), _ptr(self.overlaps), _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def backward(self, ux, uy, uzz, J, stream=None):
        """Adjoint sweep from the checkpoints of the last ``forward()`` with
        the same buffers: the gradient (and traj_dO when requested)."""
        _check(_lib.grape_backward(
            ctypes.byref(self.cm), _ptr(ux), _ptr(uy), _ptr(uzz), self.K, _ptr(J), self.R,
            ctypes.byref(self._bin), ctypes.byref(self._btg), self.dcap, self.ckpt_stride,
            _ptr(self.g_ux), _ptr(self.g_uy), _ptr(self.g_uzz), _ptr(self.traj_dO),
            _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def check(self, stream=None, raise_on_error=True):
        return status(self.ws, self.K * self.R, stream, raise_on_error)


def prepare(model: Model, ux, uy, uzz, J, inputs: MPSBatch, targets: MPSBatch,
            dcap: Optional[int] = None, ckpt_stride: int = 0, want_traj_dO: bool = False,
            stream=None):
    """Run the forward propagation in the smallest capacity bucket that
    holds every bond (searching upward on overflow) and return the prepared
    GrapeCall, its F and overlaps computed and its checkpoints ready for
    ``backward()``."""
    dev = inputs.data.device
    K = int(J.shape[0])
    R = inputs.n_traj
    model.check_J(J, K)
    key = (model.N, model.M, model.chi, model.xt_model, K, R)
    start = dcap if dcap is not None else _plan_cache.get(key)
    floor = max(inputs.max_dim, targets.max_dim)
    seq = [dcap] if dcap is not None else _bucket_sequence(model, start, floor)
    last = None
    for cap in seq:
        call = GrapeCall(model, K, R, inputs, targets, cap, ckpt_stride, want_traj_dO, dev)
        call.forward(ux, uy, uzz, J, stream)
        info = call.check(stream, raise_on_error=False)
        if info["rc"] == EOVERFLOW and dcap is None:
            last = info
            # hand the overflowed bucket's workspace back before the next,
            # larger one is allocated
            call = None
            torch.cuda.empty_cache()
            continue
        if info["rc"] != OK:
            raise TnrgError(info["rc"], _lib.tnrg_last_error().decode())
        _plan_cache[key] = cap
        return call
    raise TnrgError(EOVERFLOW, f"bond dimension exceeded every bucket up to chi ({last})")


def fidelity(model: Model, ux, uy, uzz, J, inputs: MPSBatch, targets: MPSBatch,
             dcap: Optional[int] = None, stream=None):
    """Ensemble fidelity without the gradient (forward propagation only).
    Returns (F, overlaps[K][R]) as device tensors."""
    dev = inputs.data.device
    ux, uy, uzz, J = (_f64(a, dev) for a in (ux, uy, uzz, J))
    call = prepare(model, ux, uy, uzz, J, inputs, targets, dcap, stream=stream)
    return call.F[0], call.overlaps.view(call.K, call.R)


def grape_fidelity_grad(model: Model, ux, uy, uzz, J, inputs: MPSBatch, targets: MPSBatch,
                        dcap: Optional[int] = None, ckpt_stride: int = 0,
                        want_traj_dO: bool = False, stream=None):
    """Ensemble fidelity and gradient; grows the capacity bucket on overflow."""
    dev = inputs.data.device
    K = int(J.shape[0])
    R = inputs.n_traj
    ux, uy, uzz, J = (_f64(a, dev) for a in (ux, uy, uzz, J))
    model.check_J(J, K)
    key = (model.N, model.M, model.chi, model.xt_model, K, R)
    start = dcap if dcap is not None else _plan_cache.get(key)
    floor = max(inputs.max_dim, targets.max_dim)
    seq = [dcap] if dcap is not None else _bucket_sequence(model, start, floor)
    last = None
    for cap in seq:
        call = GrapeCall(model, K, R, inputs, targets, cap, ckpt_stride, want_traj_dO, dev)
        call.run(ux, uy, uzz, J, stream)
        info = call.check(stream, raise_on_error=False)
        if info["rc"] == EOVERFLOW and dcap is None:
            last = info
            # hand the overflowed bucket's workspace back before the next,
            # larger one is allocated
            call = None
            torch.cuda.empty_cache()
            continue
        if info["rc"] != OK:
            raise TnrgError(info["rc"], _lib.tnrg_last_error().decode())
        _plan_cache[key] = cap
        out = dict(F=call.F, g_ux=call.g_ux, g_uy=call.g_uy, g_uzz=call.g_uzz,
                   overlaps=call.overlaps.view(K, R), dcap=cap, info=info)
        if want_traj_dO:
            out["traj_dO"] = call.traj_dO
        return out
    raise TnrgError(EOVERFLOW, f"bond dimension exceeded every bucket up to chi ({last})")
