"""Batched solves of many independent problems through iugkp_batch_*."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .solver import _Marshal, _defaults, _stream_handle


class BatchSolver:
    """Solve a list of problems together; outputs per instance as Solver.solve()."""

    def __init__(self, workloads, device="cuda", per_instance=None, **kw):
        """per_instance: optional list of option dicts, one per workload, each
        overriding the shared keyword options for its instance."""
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the IUGKP library needs a ROCm GPU (torch.cuda) device")
        self.ws = list(workloads)
        if per_instance is not None and len(per_instance) != len(self.ws):
            raise ValueError("per_instance needs one option dict per workload")
        self._m = []
        for i, w in enumerate(self.ws):
            o = dict(kw)
            if per_instance is not None:
                o.update(per_instance[i])
            opts = _defaults(w, o)
            if o:
                raise TypeError(f"unknown options {sorted(o)}")
            self._m.append(_Marshal(w, self.device, **opts))
        n = len(self.ws)
        probs = (C.c_void_p * n)(*[C.addressof(m.problem) for m in self._m])
        opts = (C.c_void_p * n)(*[C.addressof(m.options) for m in self._m])
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().iugkp_batch_create(probs, opts, n,
                                               C.c_void_p(_stream_handle(self.device)),
                                               C.byref(h)), "iugkp_batch_create")
        self.h = h
        L.register(self)

    def close(self):
        if getattr(self, "h", None):
            L.lib().iugkp_batch_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=L.finalizing):
        # (module globals may already be gone when the collector runs at shutdown)
        try:
            if _finalizing():
                return
            self.close()
        except Exception:
            pass

    def solve(self):
        n = len(self.ws)
        Ts, qxs, qys = [], [], []
        for w in self.ws:
            nfx = w.ny * (w.nx + 1)
            nfy = (w.ny + 1) * w.nx if w.dim == 2 else 0
            Ts.append(torch.empty(w.nx * w.ny, dtype=torch.float64, device=self.device))
            qxs.append(torch.empty(nfx, dtype=torch.float64, device=self.device))
            qys.append(torch.empty(max(nfy, 1), dtype=torch.float64, device=self.device))
        pT = (C.c_void_p * n)(*[t.data_ptr() for t in Ts])
        px = (C.c_void_p * n)(*[t.data_ptr() for t in qxs])
        py = (C.c_void_p * n)(*[t.data_ptr() for t in qys])
        st = (L.Stats * n)()
        with torch.cuda.device(self.device):
            rc = L.lib().iugkp_batch_solve(self.h, pT, px, py, st)
        # per-instance failures are reported in each instance's stats["status"];
        # only argument and memory errors concern the whole batch
        if rc in (L.E_INVALID_ARG, L.E_NOMEM):
            L.check(rc, "iugkp_batch_solve")
        out = []
        for i, w in enumerate(self.ws):
            nfy = (w.ny + 1) * w.nx if w.dim == 2 else 0
            out.append((Ts[i], qxs[i], qys[i][:nfy], st[i].as_dict()))
        return rc, out

    def tuning(self):
        """The multigrid pool's autotuner: (per-iteration us, per-cell us, group
        size of each instance in the last replay)."""
        import numpy as np
        a = C.c_double(0.0)
        c = C.c_double(0.0)
        g = np.zeros(len(self.ws), dtype=np.int32)
        L.check(L.lib().iugkp_batch_tuning(self.h, C.addressof(a), C.addressof(c),
                                           g.ctypes.data), "iugkp_batch_tuning")
        return a.value, c.value, g

    def tile_edges(self):
        """The tile march's autotuned tile edge (8 or 16 cells) of each instance."""
        import numpy as np
        e = np.zeros(len(self.ws), dtype=np.int32)
        L.check(L.lib().iugkp_batch_tiles(self.h, e.ctypes.data), "iugkp_batch_tiles")
        return e
