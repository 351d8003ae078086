"""Python face of the native serving runtime (tnrg_server_* in tnrg.h).

The server runs fidelity+gradient requests of concurrent optimisations on
one GPU with continuous batching: every request is one persistent launch on
one of the server's HIP streams, admitted in arrival order as soon as a
stream slot and a block of the device arena large enough for its workspace
are free.  This module only marshals arguments and keeps each request's
device tensors alive until its completion has been returned.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import torch

from . import tnrg


@dataclass
class Request:
    """A device-resident fidelity+gradient request and its output buffers."""
    model: tnrg.Model
    ux: torch.Tensor
    uy: torch.Tensor
    uzz: torch.Tensor
    J: torch.Tensor
    inputs: tnrg.MPSBatch
    targets: tnrg.MPSBatch
    dcap: int = 0
    F: torch.Tensor = field(default=None)
    g_ux: torch.Tensor = field(default=None)
    g_uy: torch.Tensor = field(default=None)
    g_uzz: torch.Tensor = field(default=None)
    overlaps: torch.Tensor = field(default=None)

    def __post_init__(self):
        dev = self.inputs.data.device
        M, N = self.model.M, self.model.N
        z = lambda *shape: torch.zeros(shape, dtype=torch.float64, device=dev)
        self.F = z(1) if self.F is None else self.F
        self.g_ux = z(M, N) if self.g_ux is None else self.g_ux
        self.g_uy = z(M, N) if self.g_uy is None else self.g_uy
        self.g_uzz = z(M, N - 1) if self.g_uzz is None else self.g_uzz
        self.model.check_J(self.J, int(self.J.shape[0]))
        if self.overlaps is None:
            self.overlaps = torch.zeros(int(self.J.shape[0]) * self.inputs.n_traj,
                                        dtype=torch.complex128, device=dev)

    @property
    def K(self) -> int:
        return int(self.J.shape[0])

    @property
    def R(self) -> int:
        return self.inputs.n_traj

    def workspace_bytes(self, dcap: int) -> int:
        return tnrg.grape_workspace_bytes(self.model, self.K, self.R, dcap)


class Server:
    def __init__(self, arena_bytes: int, n_streams: int = 4, max_bypass: int = 8,
                 max_dcap: int = 0, device="cuda"):
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = tnrg._SP()
        tnrg._check(tnrg._lib.tnrg_server_create(tnrg._ptr(self.arena), self.arena.numel(),
                                                 n_streams, max_bypass, max_dcap,
                                                 ctypes.byref(h)))
        self._h = h
        self._live: Dict[int, tuple] = {}

    def submit(self, req: Request) -> int:
        cm = req.model.c()
        bi, bt = req.inputs.c(), req.targets.c()
        q = tnrg._Request(ctypes.pointer(cm), req.ux.data_ptr(), req.uy.data_ptr(),
                          req.uzz.data_ptr(), req.K, req.J.data_ptr(), req.R,
                          ctypes.pointer(bi), ctypes.pointer(bt), int(req.dcap),
                          req.F.data_ptr(), req.g_ux.data_ptr(), req.g_uy.data_ptr(),
                          req.g_uzz.data_ptr(), req.overlaps.data_ptr())
        t = ctypes.c_int64()
        tnrg._check(tnrg._lib.tnrg_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        self._live[t.value] = (req,)
        return t.value

    def progress(self, max_done: int = 64) -> List[dict]:
        buf = (tnrg._Completion * max_done)()
        n = ctypes.c_int32()
        tnrg._check(tnrg._lib.tnrg_server_progress(self._h, buf, max_done, ctypes.byref(n)))
        out = []
        for c in buf[:n.value]:
            req = self._live.pop(c.ticket)[0]
            out.append(dict(ticket=c.ticket, status=c.status, dcap=c.dcap, launches=c.launches,
                            queue_ms=c.queue_ms, total_ms=c.total_ms, request=req))
        return out

    def cancel_queued(self) -> List[int]:
        info = self.info()
        cap = max(info["queued"], 1)
        buf = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        tnrg._check(tnrg._lib.tnrg_server_cancel_queued(self._h, buf, cap, ctypes.byref(n)))
        out = list(buf[:n.value])
        for t in out:
            self._live.pop(t, None)
        return out

    def info(self) -> dict:
        i = tnrg._ServerInfo()
        tnrg._check(tnrg._lib.tnrg_server_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in tnrg._ServerInfo._fields_}

    def drain(self, poll_s: float = 0.0005) -> List[dict]:
        """Run the loop until nothing is queued or running."""
        import time
        out = []
        while True:
            out += self.progress()
            i = self.info()
            if i["queued"] == 0 and i["running"] == 0:
                return out + self.progress()
            time.sleep(poll_s)

    def close(self):
        if self._h:
            rc = tnrg._lib.tnrg_server_destroy(self._h)
            self._h = None
            self._live.clear()
            tnrg._check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
