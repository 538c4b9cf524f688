"""ctypes binding of the C-ABI in ``include/mrlbm.h`` (argument marshalling only).

Every step of the method runs in the HIP library ``libmrlbm.so``; PyTorch only
provides device memory (the workspace, input and output buffers) and the HIP
stream. There is no fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .workloads import SCHEME_DIMS

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmrlbm.so")

SCHEME_IDS = {"D1Q2": 1, "D1Q3": 2, "D2Q9": 3, "D2Q4E": 4, "D3Q6": 5}
METRIC_IDS = {"linf": 0, "l2": 1}  # sibling metric of the details: max norm, or its l2 form
STATUS = {0: "ok", -1: "invalid argument", -2: "buffer too small", -3: "non-finite leaf value",
          -4: "HIP runtime error", -5: "call out of order", -6: "device-side wait gave up"}
FIELDS = {"leaf_table": 1, "populations": 2, "moments": 3, "finest": 4}
EXPORTS = ["mrlbm_workspace_size", "mrlbm_create", "mrlbm_init_equilibrium", "mrlbm_adapt",
           "mrlbm_transport_collide", "mrlbm_step", "mrlbm_get_state", "mrlbm_set_state", "mrlbm_sizes",
           "mrlbm_stats", "mrlbm_leaves", "mrlbm_destroy", "mrlbm_status_string", "mrlbm_transport_tables",
           "mrlbm_profile", "mrlbm_read_counters", "mrlbm_adjoint_workspace_size", "mrlbm_forward_record",
           "mrlbm_adjoint", "mrlbm_copy", "mrlbm_autotune", "mrlbm_set_tuning", "mrlbm_get_tuning",
           "mrlbm_fields", "mrlbm_get_mesh", "mrlbm_step_frozen", "mrlbm_debug_pair_wait", "mrlbm_create_static",
           "mrlbm_transport_tables_general"]


class MrlbmError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(status, "unknown"), status))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("jmin", ctypes.c_int), ("jmax", ctypes.c_int),
                ("precision", ctypes.c_int), ("lam", ctypes.c_double), ("eq_param", ctypes.c_double),
                ("eps", ctypes.c_double), ("mu_bar", ctypes.c_double), ("s", ctypes.c_double * 16),
                ("bc", ctypes.c_int * 4), ("gamma", ctypes.c_int), ("metric", ctypes.c_int),
                ("velocity", ctypes.c_double * 3)]

    @classmethod
    def from_cfg(cls, cfg: dict, precision: int = 8) -> "Params":
        s = list(cfg["s"]) + [0.0] * (16 - len(cfg["s"]))
        if int(cfg.get("bc_eval", 0)) != 0:
            raise ValueError("the library evaluates wall values on the leaf (bc_eval = 0) only")
        bc = [int(v) for v in cfg.get("bc", (0, 0, 0, 0))]
        return cls(SCHEME_IDS[cfg["scheme"]], int(cfg["jmin"]), int(cfg["jmax"]), int(precision),
                   float(cfg.get("lam", 1.0)), float(cfg.get("eq_param", 0.0)), float(cfg["eps"]),
                   float(cfg.get("mu_bar", 0.0)), (ctypes.c_double * 16)(*s), (ctypes.c_int * 4)(*bc),
                   int(cfg.get("gamma", 1)), METRIC_IDS[cfg.get("metric", "linf")],
                   (ctypes.c_double * 3)(*[float(v) for v in cfg.get("velocity", (0.0, 0.0, 0.0))]))


class Counters(ctypes.Structure):
    _fields_ = [("leaf_updates", ctypes.c_uint64), ("transport_launches", ctypes.c_uint64),
                ("transport_ms", ctypes.c_double), ("reconstruct_ms", ctypes.c_double),
                ("adapt_ms", ctypes.c_double), ("timed_launches", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("transport_variant", ctypes.c_int), ("list_grid_all", ctypes.c_int),
                ("list_grid_level", ctypes.c_int), ("graph", ctypes.c_int), ("pair_links", ctypes.c_int),
                ("from_cache", ctypes.c_int), ("ms_per_step", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libmrlbm.so`` (built in-tree by ``build.build()``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run paper_2103_02903_amd.build.build() "
                               "(or __graft_entry__.build()) first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER(Params)
        ci = ctypes.c_int
        sig = {
            "mrlbm_workspace_size": [P, ci, ctypes.POINTER(ctypes.c_size_t)],
            "mrlbm_create": [P, ci, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
            "mrlbm_create_static": [P, ci, vp, ctypes.POINTER(vp)],
            "mrlbm_init_equilibrium": [vp, ci, vp], "mrlbm_adapt": [vp], "mrlbm_transport_collide": [vp],
            "mrlbm_step": [vp, ci], "mrlbm_get_state": [vp, ci, vp, vp], "mrlbm_set_state": [vp, ci, vp, vp],
            "mrlbm_sizes": [vp, ci, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)],
            "mrlbm_stats": [vp, ci, ctypes.POINTER(ctypes.c_double), vp, vp, vp],
            "mrlbm_leaves": [vp, ci, vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
            "mrlbm_destroy": [vp], "mrlbm_transport_tables": [ctypes.c_int, ctypes.c_int, vp, vp],
            "mrlbm_transport_tables_general": [ci, ci, ci, ci, ci, vp, vp, vp],
            "mrlbm_profile": [vp, ctypes.c_int], "mrlbm_read_counters": [vp, ctypes.POINTER(Counters)],
            "mrlbm_adjoint_workspace_size": [vp, ci, ci, ctypes.POINTER(ctypes.c_size_t)],
            "mrlbm_forward_record": [vp, vp, ctypes.c_size_t, ci, ci],
            "mrlbm_adjoint": [vp, vp, vp, ctypes.POINTER(ctypes.c_double)],
            "mrlbm_copy": [vp, vp, ctypes.c_size_t, vp],
            "mrlbm_autotune": [vp, ci, ctypes.POINTER(Tuning)],
            "mrlbm_set_tuning": [vp, ctypes.POINTER(Tuning)],
            "mrlbm_get_tuning": [vp, ctypes.POINTER(Tuning)],
            "mrlbm_fields": [vp, ci, ci, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64)],
            "mrlbm_get_mesh": [vp, ci, vp], "mrlbm_step_frozen": [vp, vp],
            "mrlbm_debug_pair_wait": [vp, ctypes.c_uint32, ctypes.c_int32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.mrlbm_status_string.argtypes = [ctypes.c_int]
        L.mrlbm_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != 0:
        raise MrlbmError(fn, rc)


def copy(dst, src, nbytes: int, stream):
    """Device copy with the library's plain copy kernel (bandwidth reference)."""
    _check("mrlbm_copy", lib().mrlbm_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                          int(nbytes), ctypes.c_void_p(stream.cuda_stream)))


def transport_tables(scheme: str, n: int):
    """Host-side flattened transport weights W[q][25] and detail weights C[q][36]."""
    q = SCHEME_DIMS[scheme][1]
    W = np.zeros((q, 25), np.float64)
    C = np.zeros((q, 36), np.float64)
    _check("mrlbm_transport_tables",
           lib().mrlbm_transport_tables(SCHEME_IDS[scheme], int(n), W.ctypes.data, C.ctypes.data))
    return W, C


def transport_tables_general(scheme: str, n: int, gamma: int = 1, wall_x: int = 0, wall_y: int = 0):
    """Tables of the general transport path: W[q][(4 gamma + 1)^d],
    C[q][(4 gamma + 2)^d] and the counts N[q][2] of finest cells beyond the walls."""
    dim, q, _ = SCHEME_DIMS[scheme]
    W = np.zeros((q, (4 * gamma + 1) ** dim), np.float64)
    C = np.zeros((q, (4 * gamma + 2) ** dim), np.float64)
    N = np.zeros((q, 2), np.float64)
    _check("mrlbm_transport_tables_general",
           lib().mrlbm_transport_tables_general(SCHEME_IDS[scheme], int(n), int(gamma), int(wall_x), int(wall_y),
                                                W.ctypes.data, C.ctypes.data, N.ctypes.data))
    return W, C, N


class Batch:
    """A batch of independent MR-LBM instances advanced together on one GPU.
    ``cfgs`` are parameter dictionaries of ``workloads`` sharing the scheme and
    jmin; ``precision`` is 8 (FP64) or 4 (FP32)."""

    def __init__(self, cfgs, precision: int = 8, device: str = "cuda:0", static: bool = False):
        import torch

        self.torch = torch
        self.cfgs = [dict(c) for c in cfgs]
        self.B = len(self.cfgs)
        self.precision = int(precision)
        self.dim, self.q, self.nc = SCHEME_DIMS[self.cfgs[0]["scheme"]]
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == 8 else torch.float32
        self.np_dtype = np.float64 if precision == 8 else np.float32
        L = lib()
        self._p = (Params * self.B)(*[Params.from_cfg(c, precision) for c in self.cfgs])
        nbytes = ctypes.c_size_t(0)
        _check("mrlbm_workspace_size", L.mrlbm_workspace_size(self._p, self.B, ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        ctx = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            if static:  # the library's own per-device workspace (mrlbm_create_static)
                self.workspace = None
                _check("mrlbm_create_static", L.mrlbm_create_static(
                    self._p, self.B, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
            else:
                self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
                _check("mrlbm_create", L.mrlbm_create(self._p, self.B, ctypes.c_void_p(self.workspace.data_ptr()),
                                                      self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                                      ctypes.byref(ctx)))
        self._ctx = ctx
        self.total_cells = []
        for i in range(self.B):
            tot = ctypes.c_int64(0)
            q = ctypes.c_int(0)
            _check("mrlbm_sizes", L.mrlbm_sizes(ctx, i, ctypes.byref(tot), ctypes.byref(q)))
            self.total_cells.append(int(tot.value))
        self._keep = []

    def close(self):
        if getattr(self, "_ctx", None):
            lib().mrlbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- time stepping
    def init_equilibrium(self, i: int, m0):
        t = self.torch
        if isinstance(m0, t.Tensor):
            m = m0.detach().to(device=self.device, dtype=self.dtype).contiguous()
        else:
            m = t.as_tensor(np.ascontiguousarray(m0), dtype=self.dtype).to(self.device).contiguous()
        assert m.numel() == self.nc * (1 << (self.dim * int(self.cfgs[i]["jmax"])))
        self._keep.append(m)  # kept alive until the asynchronous kernel has read it
        _check("mrlbm_init_equilibrium", lib().mrlbm_init_equilibrium(self._ctx, int(i), ctypes.c_void_p(m.data_ptr())))

    def step(self, n: int = 1):
        _check("mrlbm_step", lib().mrlbm_step(self._ctx, int(n)))

    def adapt(self):
        _check("mrlbm_adapt", lib().mrlbm_adapt(self._ctx))

    def transport_collide(self):
        _check("mrlbm_transport_collide", lib().mrlbm_transport_collide(self._ctx))

    def synchronize(self):
        self.stream.synchronize()
        self._keep.clear()

    # ---- measurement
    def profile(self, enable=True):
        """Reset the counters; timing off (False / 0), every 8th transport launch
        of graph steps event-timed (True / 1) or every one (2)."""
        _check("mrlbm_profile", lib().mrlbm_profile(self._ctx, int(enable)))

    def counters(self) -> dict:
        c = Counters()
        _check("mrlbm_read_counters", lib().mrlbm_read_counters(self._ctx, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in Counters._fields_}

    # ---- state exchange (host arrays in the layouts of include/mrlbm.h)
    def get_state(self, i: int):
        tree = np.zeros(self.total_cells[i], np.uint8)
        values = np.zeros(self.q * self.total_cells[i], self.np_dtype)
        _check("mrlbm_get_state", lib().mrlbm_get_state(self._ctx, int(i), tree.ctypes.data, values.ctypes.data))
        return tree, values

    def set_state(self, i: int, tree, values):
        tree = np.ascontiguousarray(tree, dtype=np.uint8)
        values = np.ascontiguousarray(values, dtype=self.np_dtype)
        assert tree.size == self.total_cells[i] and values.size == self.q * self.total_cells[i]
        _check("mrlbm_set_state", lib().mrlbm_set_state(self._ctx, int(i), tree.ctypes.data, values.ctypes.data))

    def stats(self, i: int):
        mass = ctypes.c_double(0.0)
        n = int(self.cfgs[i]["jmax"]) + 1
        leaves, internal, ghosts = (np.zeros(n, np.int64) for _ in range(3))
        _check("mrlbm_stats", lib().mrlbm_stats(self._ctx, int(i), ctypes.byref(mass), leaves.ctypes.data,
                                                internal.ctypes.data, ghosts.ctypes.data))
        return dict(mass=float(mass.value), leaves=leaves, internal=internal, ghosts=ghosts)

    def fields(self, i: int, what: str):
        """One of the C-ABI's field outputs as a device tensor: "leaf_table"
        (int32 (level << 26) | cell per leaf), "populations" / "moments" ([n][q]
        per leaf, order (level, cell)), "finest" ([q][N_J^d] double-hat
        reconstruction on the finest level)."""
        t = self.torch
        code = FIELDS[what]
        n = ctypes.c_int64(0)
        rc = lib().mrlbm_fields(self._ctx, int(i), code, None, 0, ctypes.byref(n))
        if rc not in (0, -2):
            _check("mrlbm_fields", rc)
        count = int(n.value)
        dtype = t.int32 if what == "leaf_table" else self.dtype
        out = t.empty(max(count, 1), dtype=dtype, device=self.device)
        _check("mrlbm_fields", lib().mrlbm_fields(self._ctx, int(i), code, ctypes.c_void_p(out.data_ptr()),
                                                  out.element_size() * out.numel(), ctypes.byref(n)))
        out = out[:count]
        if what in ("populations", "moments"):
            return out.view(-1, self.q)
        if what == "finest":
            return out.view(self.q, -1)
        return out

    def get_mesh(self, i: int):
        tree = np.zeros(self.total_cells[i], np.uint8)
        _check("mrlbm_get_mesh", lib().mrlbm_get_mesh(self._ctx, int(i), tree.ctypes.data))
        return tree

    def step_frozen(self, trees):
        """One step on given new meshes: ``trees`` is one membership array per
        instance (or one array for a batch of one)."""
        if isinstance(trees, np.ndarray):
            trees = [trees]
        assert len(trees) == self.B
        flat = np.ascontiguousarray(np.concatenate([np.asarray(t, np.uint8).ravel() for t in trees]))
        assert flat.size == sum(self.total_cells)
        _check("mrlbm_step_frozen", lib().mrlbm_step_frozen(self._ctx, flat.ctypes.data))

    def debug_pair_wait(self, budget: int, count: int):
        """Test hook of the paired launches' bounded wait (see include/mrlbm.h)."""
        _check("mrlbm_debug_pair_wait", lib().mrlbm_debug_pair_wait(self._ctx, int(budget), int(count)))

    def leaves(self, i: int):
        """(cells int32 tensor of (level << 26) | cell, values [n][q] tensor) on the device."""
        t = self.torch
        count = ctypes.c_int64(0)
        rc = lib().mrlbm_leaves(self._ctx, int(i), None, None, 0, ctypes.byref(count))
        if rc not in (0, -2):
            _check("mrlbm_leaves", rc)
        n = int(count.value)
        cells = t.empty(max(n, 1), dtype=t.int32, device=self.device)
        vals = t.empty((max(n, 1), self.q), dtype=self.dtype, device=self.device)
        _check("mrlbm_leaves", lib().mrlbm_leaves(self._ctx, int(i), ctypes.c_void_p(cells.data_ptr()),
                                                  ctypes.c_void_p(vals.data_ptr()), n, ctypes.byref(count)))
        return cells[:n], vals[:n]


    # ---- launch schedule
    def autotune(self, reps: int = 5) -> dict:
        """Time the candidate launch schedules on the current state (unchanged)
        and adopt the fastest; returns the chosen schedule."""
        t = Tuning()
        _check("mrlbm_autotune", lib().mrlbm_autotune(self._ctx, int(reps), ctypes.byref(t)))
        return t.as_dict()

    def tuning(self) -> dict:
        t = Tuning()
        _check("mrlbm_get_tuning", lib().mrlbm_get_tuning(self._ctx, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, transport_variant: int, list_grid_all: int, list_grid_level: int, graph: int = 1,
                   pair_links: int = 0):
        t = Tuning(int(transport_variant), int(list_grid_all), int(list_grid_level), int(graph), int(pair_links), 0,
                   0.0)
        _check("mrlbm_set_tuning", lib().mrlbm_set_tuning(self._ctx, ctypes.byref(t)))

    # ---- adjoint on frozen meshes (batch of one)
    def forward_record(self, nsteps: int, ckpt_every: int):
        """Run ``nsteps`` steps, keeping a checkpoint every ``ckpt_every`` steps in
        a device workspace held by this object until :meth:`adjoint`."""
        nbytes = ctypes.c_size_t(0)
        _check("mrlbm_adjoint_workspace_size",
               lib().mrlbm_adjoint_workspace_size(self._ctx, int(nsteps), int(ckpt_every), ctypes.byref(nbytes)))
        self.adj_workspace = self.torch.empty(int(nbytes.value), dtype=self.torch.uint8, device=self.device)
        _check("mrlbm_forward_record",
               lib().mrlbm_forward_record(self._ctx, ctypes.c_void_p(self.adj_workspace.data_ptr()),
                                          int(nbytes.value), int(nsteps), int(ckpt_every)))

    def adjoint(self, abar_final):
        """Backward sweep of the recorded run. ``abar_final``: dJ/d(final leaf
        values), a device tensor in the values layout. Returns (dJ/dm0 device
        tensor [nc][N_J^d], dJ/ds numpy [q])."""
        t = self.torch
        a = abar_final.to(device=self.device, dtype=self.dtype).contiguous()
        assert a.numel() == self.q * self.total_cells[0]
        mbar = t.empty((self.nc, 1 << (self.dim * int(self.cfgs[0]["jmax"]))), dtype=self.dtype, device=self.device)
        sbar = (ctypes.c_double * 9)()
        _check("mrlbm_adjoint", lib().mrlbm_adjoint(self._ctx, ctypes.c_void_p(a.data_ptr()),
                                                    ctypes.c_void_p(mbar.data_ptr()), sbar))
        return mbar, np.array(sbar[:self.q])

    def state_tensor(self, i: int = 0):
        """(tree uint8, values) of instance i as device tensors (values layout)."""
        tree, values = Batch.get_state(self, i)
        return (self.torch.from_numpy(tree).to(self.device), self.torch.from_numpy(values).to(self.device))


class Sim(Batch):
    """A single MR-LBM instance (a batch of one)."""

    def __init__(self, cfg: dict, precision: int = 8, device: str = "cuda:0", static: bool = False):
        super().__init__([cfg], precision, device, static)
        self.cfg = self.cfgs[0]
        self.jmin, self.jmax = int(cfg["jmin"]), int(cfg["jmax"])

    def init_equilibrium(self, m0):
        super().init_equilibrium(0, m0)

    def get_state(self):
        return super().get_state(0)

    def set_state(self, tree, values):
        super().set_state(0, tree, values)

    def stats(self):
        return super().stats(0)

    def leaves(self):
        return super().leaves(0)

    def fields(self, what: str):
        return super().fields(0, what)

    def get_mesh(self):
        return super().get_mesh(0)
