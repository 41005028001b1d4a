"""Python binding of the sd3 C-ABI (include/sd3.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libsd3.so`` built in this directory.  PyTorch provides device
memory and the current HIP stream.  There is no CPU fallback: if the library
is not built, or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsd3.so")

MEM_HOST, MEM_DEVICE = 0, 1
PREC = {"fp32": 0, "fp64": 1}
ORDER = {"bound": 0, "none": 1, "learned": 2}
MLP_NPARAM = 9089
MLP_NIN = 10
LOG_STRIDE = 12

STATUS = {
    0: "SD3_OK", 1: "SD3_E_INVALID_ARG", 2: "SD3_E_INDEX_RANGE", 3: "SD3_E_NONFINITE",
    4: "SD3_E_RANGE", 5: "SD3_E_NOMEM", 6: "SD3_E_DEVICE", 7: "SD3_E_NO_DEVICE",
    8: "SD3_E_CAPACITY",
}

KIND = {"distance": 0, "intersects": 1}
SEG_OP = {"distance": 0, "intersects": 1, "within": 2}
SEMANTICS = {"surface": 0, "solid": 1}
TILES = (32, 64, 128)

EXPORTS = ["sd3_default_opts", "sd3_create", "sd3_destroy", "sd3_distance", "sd3_intersects",
           "sd3_graph_create", "sd3_graph_launch", "sd3_graph_result", "sd3_graph_destroy",
           "sd3_autotune", "sd3_mlp_forward", "sd3_mlp_loss_grad", "sd3_adam_step", "sd3_mlp_score",
           "sd3_validate", "sd3_status_string", "sd3_last_error", "sd3_segments", "sd3_volume",
           "sd3_distance_noalloc"]


class Geoms(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("tri", ctypes.c_void_p), ("v_off", ctypes.c_void_p),
                ("t_off", ctypes.c_void_p), ("count", ctypes.c_int64), ("mem", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("ranker", ctypes.c_void_p), ("log", ctypes.c_void_p),
                ("log_cap", ctypes.c_int64), ("queue_cap", ctypes.c_int64),
                ("rescue_cap", ctypes.c_int64), ("exact_cap", ctypes.c_int64),
                ("semantics", ctypes.c_int32), ("reserved32", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("tile_pairs_total", ctypes.c_int64), ("tile_pairs_candidate", ctypes.c_int64),
                ("tile_pairs_evaluated", ctypes.c_int64), ("tri_pairs_boxed", ctypes.c_int64),
                ("tri_pairs_fp32", ctypes.c_int64), ("tri_pairs_fp64", ctypes.c_int64),
                ("rescued", ctypes.c_int64), ("exact", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("ms_phase", ctypes.c_double * 7),
                ("logged", ctypes.c_int64), ("ms_kernel", ctypes.c_double * 4),
                ("n_kernel", ctypes.c_int64 * 4), ("sort_items", ctypes.c_int64),
                ("sort_item_bytes", ctypes.c_int32), ("sort_passes", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("queue_passes", ctypes.c_int32),
                ("queue_skew", ctypes.c_int64), ("fallback", ctypes.c_int32),
                ("reserved32", ctypes.c_int32), ("tiles_copied", ctypes.c_int64)]

    KERNELS = ("scatter", "tiles", "filter", "pairs")

    PHASES = ("upload", "prep", "queue", "pairs", "rescue", "exact", "finalize")

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("ms_phase", "ms_kernel", "n_kernel")}
        d["ms_phase"] = dict(zip(self.PHASES, list(self.ms_phase)))
        d["ms_kernel"] = dict(zip(self.KERNELS, list(self.ms_kernel)))
        d["n_kernel"] = dict(zip(self.KERNELS, list(self.n_kernel)))
        return d


class TuneReport(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("best", ctypes.c_int32), ("tile", ctypes.c_int32 * 4),
                ("ms", ctypes.c_double * 4)]


class SD3Error(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libsd3.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch provides device memory and streams, so the library must share its
    # HIP runtime: import torch (and let it initialise the device) before the
    # library pulls in libamdhip64.so.7, which the loader then resolves to
    # torch's already loaded copy.
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"sd3 HIP library not built: {path} (run python -m "
                           "paper_1808_09571_amd.build)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.sd3_default_opts.argtypes = [P(Opts)]
    lib.sd3_default_opts.restype = None
    lib.sd3_create.argtypes = [P(ctypes.c_void_p), ctypes.c_int]
    lib.sd3_create.restype = ctypes.c_int
    lib.sd3_destroy.argtypes = [ctypes.c_void_p]
    lib.sd3_destroy.restype = ctypes.c_int
    lib.sd3_distance.argtypes = [ctypes.c_void_p, P(Geoms), P(Geoms), ctypes.c_void_p,
                                 ctypes.c_void_p, P(Opts), P(Stats), ctypes.c_void_p]
    lib.sd3_distance.restype = ctypes.c_int
    lib.sd3_distance_noalloc.argtypes = lib.sd3_distance.argtypes
    lib.sd3_distance_noalloc.restype = ctypes.c_int
    lib.sd3_intersects.argtypes = [ctypes.c_void_p, P(Geoms), P(Geoms), ctypes.c_void_p,
                                   P(Opts), P(Stats), ctypes.c_void_p]
    lib.sd3_intersects.restype = ctypes.c_int
    vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
    lib.sd3_mlp_forward.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.sd3_mlp_forward.restype = ctypes.c_int
    lib.sd3_mlp_score.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.sd3_mlp_score.restype = ctypes.c_int
    lib.sd3_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    lib.sd3_mlp_loss_grad.restype = ctypes.c_int
    lib.sd3_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp]
    lib.sd3_adam_step.restype = ctypes.c_int
    lib.sd3_validate.argtypes = [P(Geoms)]
    lib.sd3_validate.restype = ctypes.c_int
    lib.sd3_graph_create.argtypes = [vp, i32, P(Geoms), P(Geoms), vp, vp, P(Opts), P(vp)]
    lib.sd3_graph_create.restype = ctypes.c_int
    lib.sd3_graph_launch.argtypes = [vp, vp]
    lib.sd3_graph_launch.restype = ctypes.c_int
    lib.sd3_graph_result.argtypes = [vp, P(Stats), vp]
    lib.sd3_graph_result.restype = ctypes.c_int
    lib.sd3_graph_destroy.argtypes = [vp]
    lib.sd3_graph_destroy.restype = ctypes.c_int
    lib.sd3_autotune.argtypes = [vp, i32, P(Geoms), P(Geoms), P(Opts), i32, P(TuneReport), vp]
    lib.sd3_autotune.restype = ctypes.c_int
    lib.sd3_segments.argtypes = [vp, i32, vp, i64, i32, P(Geoms), ctypes.c_double, vp, vp, P(Stats), vp]
    lib.sd3_segments.restype = ctypes.c_int
    lib.sd3_volume.argtypes = [vp, P(Geoms), vp, P(Stats), vp]
    lib.sd3_volume.restype = ctypes.c_int
    lib.sd3_status_string.argtypes = [ctypes.c_int]
    lib.sd3_status_string.restype = ctypes.c_char_p
    lib.sd3_last_error.argtypes = [ctypes.c_void_p]
    lib.sd3_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


@dataclass
class Batch:
    """CSR batch of meshes: ``xyz`` float64 [nv*3] and ``tri`` int32 [nt*3] (host
    numpy arrays or device torch tensors), offsets int64 numpy arrays [G+1]."""
    xyz: object
    tri: object
    v_off: np.ndarray
    t_off: np.ndarray

    @property
    def count(self) -> int:
        return int(self.v_off.shape[0] - 1)

    @property
    def on_device(self) -> bool:
        return not isinstance(self.xyz, np.ndarray)

    @classmethod
    def from_packed(cls, p, device=None):
        """From a synth.Packed (host arrays); ``device`` copies xyz/tri to a torch
        device."""
        v_off = np.ascontiguousarray(p.v_off, dtype=np.int64)
        t_off = np.ascontiguousarray(p.t_off, dtype=np.int64)
        if device is None:
            return cls(np.ascontiguousarray(p.xyz, dtype=np.float64),
                       np.ascontiguousarray(p.tri, dtype=np.int32), v_off, t_off)
        import torch
        return cls(torch.from_numpy(np.ascontiguousarray(p.xyz, dtype=np.float64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(p.tri, dtype=np.int32)).to(device),
                   v_off, t_off)

    def geoms(self) -> Geoms:
        if self.on_device:
            import torch
            assert self.xyz.dtype == torch.float64 and self.tri.dtype == torch.int32
            assert self.xyz.is_contiguous() and self.tri.is_contiguous()
            xp, tp, mem = self.xyz.data_ptr(), self.tri.data_ptr(), MEM_DEVICE
        else:
            assert self.xyz.dtype == np.float64 and self.tri.dtype == np.int32
            xp, tp, mem = self.xyz.ctypes.data, self.tri.ctypes.data, MEM_HOST
        return Geoms(xp, tp, self.v_off.ctypes.data, self.t_off.ctypes.data, self.count, mem)


class Context:
    """An sd3 context on one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        st = self.lib.sd3_create(ctypes.byref(h), int(device))
        if st != 0:
            raise SD3Error(st, self.lib.sd3_status_string(st).decode())
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sd3_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        raise SD3Error(st, self.lib.sd3_last_error(self.handle).decode())

    @staticmethod
    def _opts(precision, order, timing=False, ranker=None, log=None, tile=0, queue_cap=0,
              rescue_cap=0, exact_cap=0, semantics="surface"):
        o = Opts()
        o.semantics = SEMANTICS[semantics]
        o.precision = PREC[precision]
        o.order = ORDER[order]
        o.timing = 1 if timing else 0
        o.tile = int(tile)
        o.queue_cap = int(queue_cap)
        o.rescue_cap = int(rescue_cap)
        o.exact_cap = int(exact_cap)
        if ranker is not None:
            assert ranker.is_cuda and ranker.dtype.itemsize == 4 and ranker.numel() == MLP_NPARAM
            o.ranker = ranker.data_ptr()
        if log is not None:
            assert log.is_cuda and log.dim() == 2 and log.shape[1] == LOG_STRIDE
            o.log = log.data_ptr()
            o.log_cap = log.shape[0]
        return o

    def _stream(self, a: Batch):
        if not a.on_device:
            return None
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(a.xyz.device).cuda_stream)

    def _outputs(self, a: Batch, want_dist: bool):
        G = a.count
        if a.on_device:
            import torch
            d = torch.empty(G, dtype=torch.float64, device=a.xyz.device) if want_dist else None
            h = torch.empty(G, dtype=torch.uint8, device=a.xyz.device)
            return d, h, (d.data_ptr() if want_dist else None), h.data_ptr()
        d = np.empty(G, dtype=np.float64) if want_dist else None
        h = np.empty(G, dtype=np.uint8)
        return d, h, (d.ctypes.data if want_dist else None), h.ctypes.data

    def distance(self, a: Batch, b: Batch, precision="fp32", order="bound", stats=False,
                 timing=False, ranker=None, log=None, tile=0, queue_cap=0, rescue_cap=0,
                 exact_cap=0, semantics="surface"):
        """Row-wise 3D distance (and the exact intersects flag as a by-product).
        order="learned" needs ``ranker`` (float32 [MLP_NPARAM] on the device);
        ``log`` (float32 [cap, LOG_STRIDE] on the device) receives one training
        record per dequeued tile pair.  ``tile``: 32, 64, 128, or 0 (tuned or
        64); ``queue_cap``: candidate tile pairs per queue pass (0: default)."""
        ga, gb = a.geoms(), b.geoms()
        d, h, dp, hp = self._outputs(a, True)
        s = Stats()
        o = self._opts(precision, order, timing, ranker, log, tile, queue_cap, rescue_cap, exact_cap,
                       semantics)
        st = self.lib.sd3_distance(self.handle, ctypes.byref(ga), ctypes.byref(gb), dp, hp,
                                   ctypes.byref(o), ctypes.byref(s), self._stream(a))
        if st != 0:
            self._raise(st)
        return (d, h, s.as_dict()) if stats else (d, h)

    def distance_noalloc(self, a: Batch, b: Batch, out=None, precision="fp32", order="bound",
                         stats=False, ranker=None, tile=0, queue_cap=0, rescue_cap=0, exact_cap=0,
                         semantics="surface"):
        """sd3_distance_noalloc: the same results as ``distance`` with every
        device buffer taken from the library's static scratch (no allocation
        in the call).  ``out``: (dist, hit) outputs of ``a.count`` rows in the
        inputs' memory (float64, uint8), else allocated here."""
        ga, gb = a.geoms(), b.geoms()
        if out is None:
            d, h, dp, hp = self._outputs(a, True)
        else:
            d, h = out
            if a.on_device:
                dp, hp = d.data_ptr(), h.data_ptr()
            else:
                dp, hp = d.ctypes.data, h.ctypes.data
            if len(d) != a.count or len(h) != a.count:
                raise ValueError("outputs must hold one value per row")
        s = Stats()
        o = self._opts(precision, order, False, ranker, None, tile, queue_cap, rescue_cap, exact_cap,
                       semantics)
        st = self.lib.sd3_distance_noalloc(self.handle, ctypes.byref(ga), ctypes.byref(gb), dp, hp,
                                           ctypes.byref(o), ctypes.byref(s), self._stream(a))
        if st != 0:
            self._raise(st)
        return (d, h, s.as_dict()) if stats else (d, h)

    def intersects(self, a: Batch, b: Batch, precision="fp32", order="bound", stats=False,
                   timing=False, tile=0, queue_cap=0, rescue_cap=0, exact_cap=0, semantics="surface"):
        """Row-wise exact 3D intersects."""
        ga, gb = a.geoms(), b.geoms()
        _, h, _, hp = self._outputs(a, False)
        s = Stats()
        o = self._opts(precision, order, timing, tile=tile, queue_cap=queue_cap,
                       rescue_cap=rescue_cap, exact_cap=exact_cap, semantics=semantics)
        st = self.lib.sd3_intersects(self.handle, ctypes.byref(ga), ctypes.byref(gb), hp,
                                     ctypes.byref(o), ctypes.byref(s), self._stream(a))
        if st != 0:
            self._raise(st)
        return (h, s.as_dict()) if stats else h


    def volume(self, g: Batch):
        """Volume of each row (divergence theorem, double-double sums)."""
        G = g.count
        gg = g.geoms()
        if g.on_device:
            import torch
            v = torch.empty(G, dtype=torch.float64, device=g.xyz.device)
            vp_, stream = v.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream(g.xyz.device).cuda_stream)
        else:
            v = np.empty(G, dtype=np.float64)
            vp_, stream = v.ctypes.data, None
        st = self.lib.sd3_volume(self.handle, ctypes.byref(gg), vp_, None, stream)
        if st != 0:
            self._raise(st)
        return v

    def segments(self, op, seg, mesh: Batch, r=0.0, stats=False):
        """Segments (or points, P0 == P1) against one mesh (a Batch of one row).
        ``seg``: float64 [n, 2, 3], a numpy array (host) or a torch tensor on the
        mesh's device.  op "distance" returns (dist, hit), "intersects" and
        "within" (distance <= r) return the flags."""
        if mesh.count != 1:
            raise ValueError("the mesh must be a batch of one row")
        g = mesh.geoms()
        if mesh.on_device:
            import torch
            assert seg.dtype == torch.float64 and seg.is_contiguous() and seg.device == mesh.xyz.device
            n = int(seg.numel() // 6)
            sp, mem = seg.data_ptr(), MEM_DEVICE
            dev = mesh.xyz.device
            d = torch.empty(n, dtype=torch.float64, device=dev)
            f = torch.empty(n, dtype=torch.uint8, device=dev)
            dp, fp = d.data_ptr(), f.data_ptr()
            stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        else:
            seg = np.ascontiguousarray(seg, dtype=np.float64)
            n = int(seg.size // 6)
            sp, mem = seg.ctypes.data, MEM_HOST
            d = np.empty(n, dtype=np.float64)
            f = np.empty(n, dtype=np.uint8)
            dp, fp = d.ctypes.data, f.ctypes.data
            stream = None
        st_ = Stats()
        st = self.lib.sd3_segments(self.handle, SEG_OP[op], sp, n, mem, ctypes.byref(g), float(r),
                                   dp if op == "distance" else None, fp, ctypes.byref(st_), stream)
        if st != 0:
            self._raise(st)
        out = (d, f) if op == "distance" else f
        return (out, st_.as_dict()) if stats else out

    def graph(self, kind, a: Batch, b: Batch, precision="fp32", order="bound", ranker=None,
              tile=0, queue_cap=0):
        """A HIP graph of one whole call over device batches (see Graph)."""
        return Graph(self, kind, a, b, precision, order, ranker, tile, queue_cap)

    def autotune(self, kind, a: Batch, b: Batch, precision="fp32", order="bound", ranker=None,
                 reps=3, queue_cap=0):
        """Time every tile size on this workload, remember the fastest for
        calls with tile=0, and return {"best": size, "ms": {size: median ms}}."""
        ga, gb = a.geoms(), b.geoms()
        o = self._opts(precision, order, ranker=ranker, queue_cap=queue_cap)
        r = TuneReport()
        st = self.lib.sd3_autotune(self.handle, KIND[kind], ctypes.byref(ga), ctypes.byref(gb),
                                   ctypes.byref(o), int(reps), ctypes.byref(r), self._stream(a))
        if st != 0:
            self._raise(st)
        return {"best": r.best, "ms": {r.tile[i]: r.ms[i] for i in range(r.n)}}


class Graph:
    """One call (``kind`` "distance" or "intersects") recorded as a HIP graph
    over device-resident batches: ``launch()`` replays it on the current
    stream without host synchronisation, ``result()`` waits and checks it.
    The outputs ``dist`` (distance) and ``hit`` are fixed device tensors that
    every replay overwrites; the batches' contents may change between
    replays, their shapes may not."""

    def __init__(self, ctx: Context, kind, a: Batch, b: Batch, precision, order, ranker, tile,
                 queue_cap):
        import torch
        assert a.on_device and b.on_device, "graphs need device batches"
        self.ctx, self.lib = ctx, ctx.lib
        self._keep = (a, b, ranker)  # the graph reads these buffers on every replay
        dev = a.xyz.device
        self.dist = torch.empty(a.count, dtype=torch.float64, device=dev) if kind == "distance" else None
        self.hit = torch.empty(a.count, dtype=torch.uint8, device=dev)
        self._ga, self._gb = a.geoms(), b.geoms()
        o = Context._opts(precision, order, ranker=ranker, tile=tile, queue_cap=queue_cap)
        h = ctypes.c_void_p()
        st = self.lib.sd3_graph_create(ctx.handle, KIND[kind], ctypes.byref(self._ga),
                                       ctypes.byref(self._gb),
                                       self.dist.data_ptr() if self.dist is not None else None,
                                       self.hit.data_ptr(), ctypes.byref(o), ctypes.byref(h))
        if st != 0:
            ctx._raise(st)
        self.handle = h
        self.device = dev

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def launch(self):
        st = self.lib.sd3_graph_launch(self.handle, self._stream())
        if st != 0:
            self.ctx._raise(st)

    def result(self, stats=False):
        s = Stats()
        st = self.lib.sd3_graph_result(self.handle, ctypes.byref(s), self._stream())
        if st != 0:
            self.ctx._raise(st)
        return s.as_dict() if stats else None

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sd3_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev(t, n=None, dtype_size=4):
    assert t.is_cuda and t.is_contiguous() and t.element_size() == dtype_size, "device float32"
    if n is not None:
        assert t.numel() == n
    return t.data_ptr()


class Ranker:
    """Hand-written HIP training kernels of the tile-pair ranker MLP, driven
    through the C-ABI (sd3_mlp_forward, sd3_mlp_loss_grad, sd3_adam_step)."""

    def __init__(self, ctx: "Context"):
        self.ctx = ctx
        self.lib = ctx.lib

    def _stream(self, t):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)

    def forward(self, params, x):
        import torch
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        st = self.lib.sd3_mlp_forward(self.ctx.handle, _dev(params, MLP_NPARAM), _dev(x), n,
                                      _dev(y), self._stream(x))
        if st != 0:
            self.ctx._raise(st)
        return y

    def score(self, params, x):
        """The learned seed round's in-kernel scorer on feature rows x."""
        import torch
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        st = self.lib.sd3_mlp_score(self.ctx.handle, _dev(params, MLP_NPARAM), _dev(x), n,
                                    _dev(y), self._stream(x))
        if st != 0:
            self.ctx._raise(st)
        return y

    def loss_grad(self, params, x, t):
        import torch
        n = x.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
        st = self.lib.sd3_mlp_loss_grad(self.ctx.handle, _dev(params, MLP_NPARAM), _dev(x),
                                        _dev(t, n), n, _dev(loss), _dev(grad), self._stream(x))
        if st != 0:
            self.ctx._raise(st)
        return loss, grad

    def adam(self, p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        st = self.lib.sd3_adam_step(self.ctx.handle, _dev(p), _dev(g), _dev(m), _dev(v), p.numel(),
                                    int(step), lr, beta1, beta2, eps, self._stream(p))
        if st != 0:
            self.ctx._raise(st)


def validate(batch: Batch) -> int:
    """Host-side validation status of a host batch (0 = valid)."""
    g = batch.geoms()
    return int(load().sd3_validate(ctypes.byref(g)))
