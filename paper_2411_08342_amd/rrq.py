"""Thin Python binding of the C ABI in include/rrq.h (ctypes; argument marshalling only).

Device memory and streams come from PyTorch: every array argument is a CUDA (HIP) tensor
whose data pointer is handed to the library, and calls run on torch's current stream.  Every
step of the computation runs in the HIP library; there is no host fallback: a missing library
raises at import of the first call.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librrq.so")

RRQ_K_S, RRQ_K_D, RRQ_K_SP, RRQ_K_DP, RRQ_K_ALL = 1, 2, 4, 8, 15
RRQ_F_CORRECTION, RRQ_F_ONSURF_PV, RRQ_F_PLAIN, RRQ_F_LEARNED = 1, 2, 8, 16
KERNELS = ("S", "D", "Sp", "Dp")

EXPORTED = ("rrq_plan_create", "rrq_plan_refit", "rrq_plan_destroy", "rrq_workspace_size",
            "rrq_pair_offsets", "rrq_assemble", "rrq_apply", "rrq_autotune", "rrq_graph_create",
            "rrq_graph_launch", "rrq_graph_destroy", "rrq_collect_roots", "rrq_mlp_train",
            "rrq_mlp_loss_grad", "rrq_mlp_predict", "rrq_plan_set_mlp", "rrq_potentials",
            "rrq_smooth_potentials", "rrq_plan_fit_condition", "rrq_assemble_noalloc",
            "rrq_plan_patch_flags", "rrq_weights_size", "rrq_status_string")
RRQ_ERR_ARG, RRQ_ERR_DEVICE, RRQ_ERR_OOM, RRQ_ERR_ILLCONDITIONED = -1, -2, -3, -4
RRQ_ERR_UNSUPPORTED, RRQ_ERR_BUFFER, RRQ_ERR_NONFINITE = -5, -6, -7
MLP_PARAMS = 4866


class RRQError(RuntimeError):
    """A non-zero rrq_status; `code` is the status, `stats` the statistics of the call when it
    took any."""

    def __init__(self, msg, code=0, stats=None):
        super().__init__(msg)
        self.code = code
        self.stats = stats


class Surface(ctypes.Structure):
    _fields_ = [("npatch", ctypes.c_int32), ("order_host", ctypes.c_void_p),
                ("order", ctypes.c_void_p), ("node_off", ctypes.c_void_p),
                ("node_xyz", ctypes.c_void_p), ("node_nrm", ctypes.c_void_p),
                ("node_wt", ctypes.c_void_p), ("edge_off", ctypes.c_void_p),
                ("edge_xyz", ctypes.c_void_p), ("nnode", ctypes.c_int64),
                ("nedge", ctypes.c_int64)]


class Targets(ctypes.Structure):
    _fields_ = [("ntarget", ctypes.c_int64), ("nnz", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("nrm", ctypes.c_void_p), ("self_patch", ctypes.c_void_p),
                ("self_node", ctypes.c_void_p), ("near_ptr", ctypes.c_void_p),
                ("near_patch", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("rho_far", ctypes.c_double), ("newton_tol", ctypes.c_double),
                ("newton_maxit", ctypes.c_int32), ("tile_targets", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("ls_unweighted", ctypes.c_int32),
                ("ptilde_factor", ctypes.c_int32), ("u_rule", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("near_edges", ctypes.c_int64),
                ("newton_iters", ctypes.c_int64), ("newton_fail", ctypes.c_int64),
                ("learned_accept", ctypes.c_int64), ("newton_max", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("newton_wave_iters", ctypes.c_int64),
                ("panel_overflow", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
                ("flagged_pairs", ctypes.c_int64), ("invalid", ctypes.c_uint32),
                ("order_kernel_ms", ctypes.c_double * 5),
                ("newton_slots", ctypes.c_int64), ("newton_over", ctypes.c_int64 * 5)]
    NEWTON_OVER = (2, 4, 6, 8, 12)

    def as_dict(self):
        return _struct_dict(self)


ORDERS = (4, 5, 6, 8, 10)   # index of the per-order arrays of Stats and TuneResult


def _struct_dict(st):
    d = {}
    for k, t in st._fields_:
        v = getattr(st, k)
        if hasattr(v, "__len__"):
            d[k] = [float(x) if isinstance(x, float) else int(x) for x in v]
        else:
            d[k] = float(v) if isinstance(v, float) else int(v)
    return d


class MlpCfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_targets", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("from_cache", ctypes.c_int32),
                ("order_tile", ctypes.c_int32 * 5), ("order_grid", ctypes.c_int32 * 5),
                ("order_ms", ctypes.c_double * 5)]


_lib = None


def lib():
    """Load librrq.so (built in-tree by paper_2411_08342_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RRQError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
        L.rrq_plan_create.argtypes = [ctypes.POINTER(Surface), ctypes.POINTER(Options), vp,
                                      ctypes.POINTER(vp)]
        L.rrq_plan_refit.argtypes = [vp, ctypes.POINTER(Surface), vp]
        L.rrq_plan_destroy.argtypes = [vp]
        L.rrq_plan_fit_condition.argtypes = [vp, vp, vp]
        L.rrq_plan_patch_flags.argtypes = [vp, ctypes.c_double, vp, vp]
        L.rrq_weights_size.argtypes = [vp, ctypes.POINTER(Targets), ctypes.POINTER(i64), vp]
        L.rrq_workspace_size.argtypes = [vp, ctypes.POINTER(Targets), ctypes.POINTER(ctypes.c_size_t)]
        L.rrq_pair_offsets.argtypes = [vp, ctypes.POINTER(Targets), vp, vp, ctypes.c_size_t,
                                       ctypes.POINTER(i64), vp]
        L.rrq_assemble.argtypes = [vp, ctypes.POINTER(Targets), u32, u32, vp, vp, vp, vp, i64,
                                   vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(Stats)]
        L.rrq_assemble_noalloc.argtypes = [vp, ctypes.POINTER(Targets), u32, u32, vp, vp, vp,
                                           vp, i64, vp, vp, vp]
        L.rrq_apply.argtypes = [vp, ctypes.POINTER(Targets), u32, vp, vp, vp, vp, vp, vp, vp, vp,
                                vp, vp, vp]
        L.rrq_potentials.argtypes = [vp, ctypes.POINTER(Targets), u32, u32, vp, vp, vp, vp, vp,
                                     vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(Stats)]
        L.rrq_smooth_potentials.argtypes = [vp, ctypes.POINTER(Targets), u32, vp, vp, vp, vp, vp,
                                            vp]
        L.rrq_autotune.argtypes = [vp, ctypes.POINTER(Targets), u32, u32, vp, vp, vp, vp, i64,
                                   vp, vp, ctypes.c_size_t, ctypes.c_char_p, vp,
                                   ctypes.POINTER(TuneResult)]
        L.rrq_graph_create.argtypes = [vp, ctypes.POINTER(Surface), ctypes.POINTER(Targets), u32,
                                       u32, vp, vp, vp, vp, i64, vp, vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(vp)]
        L.rrq_graph_launch.argtypes = [vp, vp]
        L.rrq_graph_destroy.argtypes = [vp]
        L.rrq_collect_roots.argtypes = [vp, ctypes.POINTER(Targets), i64, vp, vp, vp,
                                        ctypes.POINTER(i64), vp]
        L.rrq_mlp_train.argtypes = [vp, vp, i64, ctypes.POINTER(MlpCfg), vp, vp, vp]
        L.rrq_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.rrq_mlp_predict.argtypes = [vp, vp, i64, vp, vp]
        L.rrq_plan_set_mlp.argtypes = [vp, vp, vp]
        L.rrq_status_string.argtypes = [i32]
        L.rrq_status_string.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name != "rrq_status_string":
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(rc, stats=None):
    if rc != 0:
        raise RRQError(f"rrq call failed: {rc} ({lib().rrq_status_string(rc).decode()})", rc,
                       stats.as_dict() if stats is not None else None)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


class DeviceSurface:
    """Surface arrays resident on the device (torch tensors) plus the host order list."""

    def __init__(self, surf):
        import torch
        self.order_host = np.ascontiguousarray(surf["order"], dtype=np.int32)
        self.order = _dev(self.order_host, torch.int32)
        self.node_off = _dev(surf["node_off"], torch.int64)
        self.node_xyz = _dev(surf["node_xyz"], torch.float64)
        self.node_nrm = _dev(surf["node_nrm"], torch.float64)
        self.node_wt = _dev(surf["node_wt"], torch.float64)
        self.edge_off = _dev(surf["edge_off"], torch.int64)
        self.edge_xyz = _dev(surf["edge_xyz"], torch.float64)
        self.npatch = int(len(self.order_host))

    def cstruct(self):
        return Surface(self.npatch, self.order_host.ctypes.data, self.order.data_ptr(),
                       self.node_off.data_ptr(), self.node_xyz.data_ptr(),
                       self.node_nrm.data_ptr(), self.node_wt.data_ptr(),
                       self.edge_off.data_ptr(), self.edge_xyz.data_ptr(),
                       int(self.node_xyz.shape[1]), int(self.edge_xyz.shape[1]))


class DeviceTargets:
    def __init__(self, tg):
        import torch
        self.xyz = _dev(tg["xyz"], torch.float64)
        self.nrm = _dev(tg["nrm"], torch.float64)
        self.self_patch = _dev(tg["self_patch"], torch.int32)
        self.self_node = _dev(tg["self_node"], torch.int32)
        self.near_ptr = _dev(tg["near_ptr"], torch.int64)
        self.near_patch = _dev(tg["near_patch"], torch.int32)
        self.ntarget = int(self.xyz.shape[1])
        self.nnz = int(self.near_patch.shape[0])

    def cstruct(self):
        return Targets(self.ntarget, self.nnz, self.xyz.data_ptr(), self.nrm.data_ptr(),
                       self.self_patch.data_ptr(), self.self_node.data_ptr(),
                       self.near_ptr.data_ptr(), self.near_patch.data_ptr() if self.nnz else 0)


class Plan:
    """rrq_plan: per-patch frames, coefficient maps and edge tables on the device."""

    def __init__(self, dsurf, rho_far=0.0, newton_tol=0.0, newton_maxit=0, tile_targets=0,
                 grid=0, ls_unweighted=0, ptilde_factor=0, u_rule=0):
        self.dsurf = dsurf
        self._s = dsurf.cstruct()
        self._o = Options(rho_far, newton_tol, newton_maxit, tile_targets, grid, ls_unweighted,
                          ptilde_factor, u_rule)
        h = ctypes.c_void_p()
        _check(lib().rrq_plan_create(ctypes.byref(self._s), ctypes.byref(self._o), _stream(),
                                     ctypes.byref(h)))
        self.handle = h

    def set_mlp(self, params):
        """Install a trained network (float32 CUDA tensor of MLP_PARAMS) or remove it (None)."""
        _check(lib().rrq_plan_set_mlp(self.handle, params.data_ptr() if params is not None else None,
                                      _stream()))

    def fit_condition(self):
        """(P, 2) host array: Frobenius-norm condition numbers ||A_w||_F ||A_w^+||_F of the
        weighted DLP and SLP systems of every patch."""
        out = np.zeros((self.dsurf.npatch, 2))
        _check(lib().rrq_plan_fit_condition(self.handle, out.ctypes.data, _stream()))
        return out

    def patch_flags(self, max_cond=0.0):
        """rrq_plan_patch_flags: (status, int32 host array [P]) with bit 1 / 2 = DLP / SLP fit
        condition estimate above max_cond, bit 4 = non-finite source data."""
        out = np.zeros(self.dsurf.npatch, dtype=np.int32)
        rc = lib().rrq_plan_patch_flags(self.handle, max_cond, out.ctypes.data, _stream())
        if rc not in (0, RRQ_ERR_ILLCONDITIONED):
            _check(rc)
        return rc, out

    def refit(self, dsurf=None):
        if dsurf is not None:
            self.dsurf = dsurf
            self._s = dsurf.cstruct()
        _check(lib().rrq_plan_refit(self.handle, ctypes.byref(self._s), _stream()))

    def close(self):
        if self.handle:
            _check(lib().rrq_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Assembler:
    """Pair offsets, workspace, output buffers and per-pair flags for one near list."""

    def __init__(self, plan, dtg, kmask=RRQ_K_ALL):
        import torch
        self.plan, self.dtg, self.kmask = plan, dtg, kmask
        self._t = dtg.cstruct()
        nw = ctypes.c_int64()
        _check(lib().rrq_weights_size(plan.handle, ctypes.byref(self._t), ctypes.byref(nw),
                                      _stream()))
        self.nweights = int(nw.value)
        self.pair_off = torch.empty(dtg.nnz + 1, dtype=torch.int64, device="cuda")
        self.pair_flags = torch.zeros(max(dtg.nnz, 1), dtype=torch.int32, device="cuda")
        sz = ctypes.c_size_t()
        _check(lib().rrq_workspace_size(plan.handle, ctypes.byref(self._t), ctypes.byref(sz)))
        self.workspace = torch.empty(int(sz.value), dtype=torch.uint8, device="cuda")
        nw2 = ctypes.c_int64()
        _check(lib().rrq_pair_offsets(plan.handle, ctypes.byref(self._t), self.pair_off.data_ptr(),
                                      self.workspace.data_ptr(), self.workspace.numel(),
                                      ctypes.byref(nw2), _stream()))
        assert int(nw2.value) == self.nweights
        self.out = {k: (torch.empty(self.nweights, dtype=torch.float64, device="cuda")
                        if kmask & (1 << i) else None) for i, k in enumerate(KERNELS)}

    def pair_offsets(self):
        _check(lib().rrq_pair_offsets(self.plan.handle, ctypes.byref(self._t),
                                      self.pair_off.data_ptr(), self.workspace.data_ptr(),
                                      self.workspace.numel(), None, _stream()))

    def assemble(self, flags=RRQ_F_CORRECTION | RRQ_F_ONSURF_PV, stats=False):
        """rrq_assemble into self.out (and the per-pair flags into self.pair_flags); with
        stats, synchronises and returns the statistics (a failed device check or NaN/Inf
        outputs raise RRQError carrying them)."""
        st = Stats() if stats else None
        ptr = [self.out[k].data_ptr() if self.out[k] is not None else None for k in KERNELS]
        _check(lib().rrq_assemble(self.plan.handle, ctypes.byref(self._t), self.kmask, flags,
                                  ptr[0], ptr[1], ptr[2], ptr[3], self.nweights,
                                  self.pair_off.data_ptr(), self.pair_flags.data_ptr(),
                                  self.workspace.data_ptr(), self.workspace.numel(), _stream(),
                                  ctypes.byref(st) if st is not None else None), st)
        return st.as_dict() if st is not None else None

    def assemble_noalloc(self, flags=RRQ_F_CORRECTION | RRQ_F_ONSURF_PV):
        """rrq_assemble_noalloc: the same assembly with the library's own device scratch
        instead of this object's workspace (no statistics)."""
        ptr = [self.out[k].data_ptr() if self.out[k] is not None else None for k in KERNELS]
        _check(lib().rrq_assemble_noalloc(self.plan.handle, ctypes.byref(self._t), self.kmask,
                                          flags, ptr[0], ptr[1], ptr[2], ptr[3], self.nweights,
                                          self.pair_off.data_ptr(), self.pair_flags.data_ptr(),
                                          _stream()))

    def apply(self, density):
        import torch
        dens = torch.as_tensor(density, dtype=torch.float64, device="cuda")
        pots = {k: (torch.empty(self.dtg.ntarget, dtype=torch.float64, device="cuda")
                    if self.out[k] is not None else None) for k in KERNELS}
        ptr = lambda d, k: d[k].data_ptr() if d[k] is not None else None
        _check(lib().rrq_apply(self.plan.handle, ctypes.byref(self._t), self.kmask,
                               ptr(self.out, "S"), ptr(self.out, "D"), ptr(self.out, "Sp"),
                               ptr(self.out, "Dp"), self.pair_off.data_ptr(), dens.data_ptr(),
                               ptr(pots, "S"), ptr(pots, "D"), ptr(pots, "Sp"), ptr(pots, "Dp"),
                               _stream()))
        return pots


class Evaluator:
    """Potentials mode: the correction (rrq_potentials) and the direct smooth rule
    (rrq_smooth_potentials) applied to a density without storing weights."""

    def __init__(self, plan, dtg, kmask=RRQ_K_ALL):
        import torch
        self.plan, self.dtg, self.kmask = plan, dtg, kmask
        self._t = dtg.cstruct()
        sz = ctypes.c_size_t()
        _check(lib().rrq_workspace_size(plan.handle, ctypes.byref(self._t), ctypes.byref(sz)))
        self.workspace = torch.empty(int(sz.value), dtype=torch.uint8, device="cuda")

    def _pots(self):
        import torch
        return {k: (torch.empty(self.dtg.ntarget, dtype=torch.float64, device="cuda")
                    if self.kmask & (1 << i) else None) for i, k in enumerate(KERNELS)}

    def potentials(self, density, flags=RRQ_F_CORRECTION | RRQ_F_ONSURF_PV, stats=False):
        import torch
        dens = torch.as_tensor(density, dtype=torch.float64, device="cuda").contiguous()
        pots = self._pots()
        ptr = [pots[k].data_ptr() if pots[k] is not None else None for k in KERNELS]
        st = Stats() if stats else None
        _check(lib().rrq_potentials(self.plan.handle, ctypes.byref(self._t), self.kmask, flags,
                                    dens.data_ptr(), ptr[0], ptr[1], ptr[2], ptr[3], None,
                                    self.workspace.data_ptr(), self.workspace.numel(), _stream(),
                                    ctypes.byref(st) if st is not None else None), st)
        return (pots, st.as_dict()) if stats else pots

    def smooth(self, density):
        import torch
        dens = torch.as_tensor(density, dtype=torch.float64, device="cuda").contiguous()
        pots = self._pots()
        ptr = [pots[k].data_ptr() if pots[k] is not None else None for k in KERNELS]
        _check(lib().rrq_smooth_potentials(self.plan.handle, ctypes.byref(self._t), self.kmask,
                                           dens.data_ptr(), ptr[0], ptr[1], ptr[2], ptr[3],
                                           _stream()))
        return pots


def _out_ptrs(asm):
    return [asm.out[k].data_ptr() if asm.out[k] is not None else None for k in KERNELS]


def autotune(asm, flags=RRQ_F_CORRECTION | RRQ_F_ONSURF_PV, cache_path=None):
    """rrq_autotune: pick the tile size and grid of the batched form for this near list."""
    r = TuneResult()
    p = _out_ptrs(asm)
    _check(lib().rrq_autotune(asm.plan.handle, ctypes.byref(asm._t), asm.kmask, flags, p[0], p[1],
                              p[2], p[3], asm.nweights, asm.pair_off.data_ptr(),
                              asm.workspace.data_ptr(), asm.workspace.numel(),
                              cache_path.encode() if cache_path else None, _stream(),
                              ctypes.byref(r)))
    return _struct_dict(r)


class Graph:
    """rrq_graph: one whole step (refit, pair offsets, assembly) captured into a HIP graph."""

    def __init__(self, asm, flags=RRQ_F_CORRECTION | RRQ_F_ONSURF_PV):
        self.asm = asm
        self._s = asm.plan.dsurf.cstruct()
        p = _out_ptrs(asm)
        h = ctypes.c_void_p()
        _check(lib().rrq_graph_create(asm.plan.handle, ctypes.byref(self._s), ctypes.byref(asm._t),
                                      asm.kmask, flags, p[0], p[1], p[2], p[3], asm.nweights,
                                      asm.pair_off.data_ptr(), asm.workspace.data_ptr(),
                                      asm.workspace.numel(), _stream(), ctypes.byref(h)))
        self.handle = h

    def launch(self):
        _check(lib().rrq_graph_launch(self.handle, _stream()))

    def close(self):
        if self.handle:
            _check(lib().rrq_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------------------
# learned initial guess of the singularity-swap Newton solve
# ---------------------------------------------------------------------------------------
def collect_roots(plan, dtg, cap):
    """rrq_collect_roots: (feat [8][n] float32, dt [2][n] float32, t0 [2][n] float64) for the
    near (pair, edge) combinations of this near list, n <= cap."""
    import torch
    t = dtg.cstruct()
    feat = torch.empty((8, cap), dtype=torch.float32, device="cuda")
    dt = torch.empty((2, cap), dtype=torch.float32, device="cuda")
    t0 = torch.empty((2, cap), dtype=torch.float64, device="cuda")
    n = ctypes.c_int64()
    _check(lib().rrq_collect_roots(plan.handle, ctypes.byref(t), cap, feat.data_ptr(),
                                   dt.data_ptr(), t0.data_ptr(), ctypes.byref(n), _stream()))
    n = int(n.value)
    return (feat[:, :n].contiguous(), dt[:, :n].contiguous(), t0[:, :n].contiguous())


def mlp_train(feat, dt, steps=3000, batch=4096, lr=3e-3, seed=1):
    """rrq_mlp_train on samples feat [8][m], dt [2][m]: returns (params, loss_curve)."""
    import torch
    m = feat.shape[1]
    assert feat.shape == (8, m) and dt.shape == (2, m)
    feat, dt = feat.contiguous(), dt.contiguous()
    params = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    curve = torch.empty(steps, dtype=torch.float32, device="cuda")
    cfg = MlpCfg(steps, batch, lr, seed)
    _check(lib().rrq_mlp_train(feat.data_ptr(), dt.data_ptr(), m, ctypes.byref(cfg),
                               params.data_ptr(), curve.data_ptr(), _stream()))
    return params, curve


def mlp_loss_grad(params, feat, dt):
    """rrq_mlp_loss_grad: (loss, gradient) of the mean squared error on n samples."""
    import torch
    n = feat.shape[1]
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    _check(lib().rrq_mlp_loss_grad(params.contiguous().data_ptr(), feat.contiguous().data_ptr(),
                                   dt.contiguous().data_ptr(), n, loss.data_ptr(),
                                   grad.data_ptr(), _stream()))
    return loss, grad


def mlp_predict(params, feat):
    """rrq_mlp_predict: outputs [2][n] for features [8][n]."""
    import torch
    n = feat.shape[1]
    out = torch.empty((2, n), dtype=torch.float32, device="cuda")
    _check(lib().rrq_mlp_predict(params.contiguous().data_ptr(), feat.contiguous().data_ptr(), n,
                                 out.data_ptr(), _stream()))
    return out
