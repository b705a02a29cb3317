"""ctypes binding of libn2f.so (include/n2f.h), the Noise2Fast GPU library.

Argument marshalling only: every step of the loop runs in the HIP library.
PyTorch supplies device memory (images, the workspace) and the stream.
Importing this module does not load the library; the first call does, and
raises if it has not been built (``python -m paper_2108_10209_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int, c_longlong, c_size_t, c_ulonglong, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libn2f.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC, ECANCELED = 0, -1, -2, -3, -4, -5, -6
WCONSTANT, WCAPPED = 1, 2
FP32, BF16 = 0, 1
DS_CHECKERBOARD, DS_QUAD = 0, 1

SYMBOLS = [
    "n2f_config_default", "n2f_last_error", "n2f_param_count", "n2f_init_params", "n2f_workspace_bytes",
    "n2f_run_create", "n2f_run_destroy", "n2f_train_step", "n2f_validate", "n2f_run_epochs", "n2f_result",
    "n2f_denoise", "n2f_get_state", "n2f_set_state", "n2f_get_grad", "n2f_debug_adam", "n2f_get_progress",
    "n2f_get_history", "n2f_get_lohi", "n2f_get_image", "n2f_profile_begin", "n2f_profile_read",
    "n2f_profile_end", "n2f_run_launch_epochs", "n2f_run_poll", "n2f_batch_workspace_bytes", "n2f_batch_create",
    "n2f_batch_run", "n2f_batch_result", "n2f_batch_progress", "n2f_batch_destroy", "n2f_server_create",
    "n2f_server_submit", "n2f_server_step", "n2f_server_poll", "n2f_server_memory", "n2f_server_destroy",
    "n2f_run_set_clean", "n2f_max_project", "n2f_batch_run_of", "n2f_checkpoint_bytes", "n2f_save_checkpoint",
    "n2f_load_checkpoint", "n2f_batch_add", "n2f_batch_remove", "n2f_server_cancel", "n2f_denoise_noalloc",
    "n2f_server_table_bytes", "n2f_group_grid_get", "n2f_group_grid_set",
]
NOALLOC_MAX_BYTES = 128 << 20   # N2F_NOALLOC_MAX_BYTES
SERVER_SIMULATE = 1
SERVER_GROUPED = 2
K_CONV_FWD, K_BACKWARD, K_ADAM = 0, 1, 2
LITERAL_WIDTHS = (32, 32, 64, 64, 128, 128, 256, 256)   # the Methods' per-layer widths
K_GROUP = 16                # + kind: one grouped launch (see n2f.h)
GROUP_KINDS = ["conv3x3_fwd", "conv3x3_dgrad", "conv3x3_fwd_head", "conv3x3_fwd_val", "conv3x3_fwd_first",
               "conv3x3_wgrad", "conv1_c1", "conv1_c2", "conv1_c3", "wgrad1_c1", "wgrad1_c2", "wgrad1_c3", "adam",
               "decide", "accumulate"]
BATCH_GROUPED = -1          # n_streams of a grouped batch


class N2FError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"n2f error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("n_layers", c_int), ("width", c_int),
        ("lr", c_float), ("eps", c_float), ("beta1", c_double), ("beta2", c_double),
        ("patience", c_int), ("max_epochs", c_int), ("fixed_epochs", c_int),
        ("pair_order", c_int * 4), ("precision", c_int), ("init_seed", c_ulonglong),
        ("use_graph", c_int), ("downsample", c_int), ("exact_targets", c_int), ("widths", c_int * 8),
        ("wgrad_splits", c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2108_10209_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.n2f_config_default.restype = None
        L.n2f_config_default.argtypes = [POINTER(Config)]
        L.n2f_last_error.restype = ctypes.c_char_p
        L.n2f_last_error.argtypes = []
        sig = {
            "n2f_param_count": [c_int, POINTER(Config), POINTER(c_size_t)],
            "n2f_init_params": [c_int, POINTER(Config), c_ulonglong, c_void_p],
            "n2f_workspace_bytes": [c_int, c_int, c_int, POINTER(Config), POINTER(c_size_t)],
            "n2f_run_create": [POINTER(c_void_p), c_void_p, c_int, c_int, c_int, POINTER(Config), c_void_p,
                               c_size_t, c_void_p],
            "n2f_run_destroy": [c_void_p],
            "n2f_train_step": [c_void_p, c_int, c_int],
            "n2f_validate": [c_void_p, c_int, POINTER(c_double), POINTER(c_int), POINTER(c_int)],
            "n2f_run_epochs": [c_void_p, c_int, c_int, POINTER(c_int)],
            "n2f_result": [c_void_p, c_void_p],
            "n2f_denoise": [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(Config), c_void_p, c_size_t,
                            c_void_p],
            "n2f_denoise_noalloc": [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(Config), c_void_p],
            "n2f_get_state": [c_void_p, c_int, c_void_p, c_void_p, c_void_p, POINTER(c_longlong)],
            "n2f_set_state": [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_longlong],
            "n2f_get_grad": [c_void_p, c_int, c_void_p, POINTER(c_double)],
            "n2f_debug_adam": [c_void_p, c_int, c_void_p],
            "n2f_get_progress": [c_void_p, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                 POINTER(c_double)],
            "n2f_get_history": [c_void_p, c_int, c_int, c_void_p],
            "n2f_get_lohi": [c_void_p, POINTER(c_float), POINTER(c_float)],
            "n2f_get_image": [c_void_p, c_int, c_void_p],
            "n2f_profile_begin": [c_int],
            "n2f_profile_read": [c_int, POINTER(c_double), POINTER(c_longlong), POINTER(c_longlong)],
            "n2f_profile_end": [],
            "n2f_run_launch_epochs": [c_void_p, c_int, c_int],
            "n2f_run_poll": [c_void_p, c_int, POINTER(c_int), POINTER(c_int)],
            "n2f_batch_workspace_bytes": [c_int, c_void_p, c_void_p, c_void_p, POINTER(Config), POINTER(c_size_t)],
            "n2f_batch_create": [POINTER(c_void_p), c_int, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(Config),
                                 c_void_p, c_size_t, c_int, c_void_p],
            "n2f_batch_add": [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_size_t, POINTER(c_int)],
            "n2f_batch_remove": [c_void_p, c_int],
            "n2f_batch_run": [c_void_p, c_int, POINTER(c_int)],
            "n2f_batch_result": [c_void_p, c_int, c_void_p],
            "n2f_batch_progress": [c_void_p, c_int, POINTER(c_int), POINTER(c_int)],
            "n2f_batch_destroy": [c_void_p],
            "n2f_server_create": [POINTER(c_void_p), POINTER(Config), c_void_p, c_size_t, c_int, c_int, c_int],
            "n2f_server_table_bytes": [c_int, POINTER(c_size_t)],
            "n2f_server_submit": [c_void_p, c_longlong, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p],
            "n2f_server_cancel": [c_void_p, c_longlong],
            "n2f_server_step": [c_void_p, c_int, POINTER(c_int), POINTER(c_int)],
            "n2f_server_poll": [c_void_p, c_void_p, c_void_p, c_int, POINTER(c_int)],
            "n2f_server_memory": [c_void_p, POINTER(c_size_t), POINTER(c_size_t)],
            "n2f_server_destroy": [c_void_p],
            "n2f_run_set_clean": [c_void_p, c_void_p],
            "n2f_max_project": [c_void_p, c_int, c_longlong, c_void_p, c_void_p],
            "n2f_batch_run_of": [c_void_p, c_int, POINTER(c_void_p)],
            "n2f_checkpoint_bytes": [c_void_p, POINTER(c_size_t)],
            "n2f_save_checkpoint": [c_void_p, c_int, c_void_p, c_size_t],
            "n2f_load_checkpoint": [c_void_p, c_int, c_void_p, c_size_t],
            "n2f_group_grid_get": [c_int, POINTER(c_int)],
            "n2f_group_grid_set": [c_int, c_int],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.restype = c_int
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> int:
    if status < 0:
        raise N2FError(status, lib().n2f_last_error().decode(errors="replace"))
    return status


def default_config(**kw) -> Config:
    cfg = Config()
    lib().n2f_config_default(byref(cfg))
    for k, v in kw.items():
        if k == "pair_order":
            cfg.pair_order = (c_int * 4)(*v)
        elif k == "widths":
            cfg.widths = (c_int * 8)(*v)
        else:
            setattr(cfg, k, v)
    return cfg


def param_count(C: int, cfg: Config | None = None) -> int:
    cfg = cfg or default_config()
    n = c_size_t()
    _check(lib().n2f_param_count(C, byref(cfg), byref(n)))
    return n.value


def init_params(C: int, seed: int, cfg: Config | None = None) -> np.ndarray:
    cfg = cfg or default_config()
    n = param_count(C, cfg)
    out = np.empty((C, n), dtype=np.float32)
    _check(lib().n2f_init_params(C, byref(cfg), c_ulonglong(seed), out.ctypes.data))
    return out


def workspace_bytes(H: int, W: int, C: int, cfg: Config | None = None) -> int:
    cfg = cfg or default_config()
    n = c_size_t()
    _check(lib().n2f_workspace_bytes(H, W, C, byref(cfg), byref(n)))
    return n.value


def _stream_of(t):
    import torch
    return c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_image(x, name="image"):
    """A (C, H, W) FP32 contiguous CUDA tensor, checked on the host before
    any pointer reaches the library (a host pointer read by a kernel faults
    the device)."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() == 3
            and x.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape (C, H, W)")


class Run:
    """One image's run: create, step, validate, read results and state."""

    def __init__(self, x, cfg: Config | None = None, ws=None):
        import torch
        _check_image(x)
        self.cfg = cfg or default_config()
        self.C, self.H, self.W = (int(s) for s in x.shape)
        self.device = x.device
        nbytes = workspace_bytes(self.H, self.W, self.C, self.cfg)
        self.ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        assert self.ws.numel() >= nbytes
        self.nparams = param_count(self.C, self.cfg)
        self._owned = True
        self._ptr = c_void_p()
        self.status = _check(lib().n2f_run_create(byref(self._ptr), c_void_p(x.data_ptr()), self.H, self.W, self.C,
                                                  byref(self.cfg), c_void_p(self.ws.data_ptr()), nbytes,
                                                  _stream_of(x)))

    @classmethod
    def _view(cls, ptr, shape, cfg, device):
        """A handle on a run owned elsewhere (a batch image): state calls
        only, never destroyed from here."""
        r = cls.__new__(cls)
        r.cfg, r.device, r._ptr, r._owned = cfg, device, ptr, False
        r.C, r.H, r.W = shape
        r.nparams = param_count(r.C, cfg)
        r.status = OK
        return r

    def close(self):
        if self._ptr and self._owned:
            lib().n2f_run_destroy(self._ptr)
        self._ptr = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_clean(self, clean):
        """Targets of the "Exact" ablation from the clean image (same shape as
        the input, FP32 CUDA, contiguous); needs exact_targets=1."""
        import torch
        assert clean.is_cuda and clean.dtype == torch.float32 and clean.is_contiguous()
        assert tuple(clean.shape) == (self.C, self.H, self.W)
        _check(lib().n2f_run_set_clean(self._ptr, c_void_p(clean.data_ptr())))

    def train_step(self, net: int, pair: int):
        _check(lib().n2f_train_step(self._ptr, net, pair))

    def validate(self, net: int = 0):
        v, imp, done = c_double(), c_int(), c_int()
        _check(lib().n2f_validate(self._ptr, net, byref(v), byref(imp), byref(done)))
        return v.value, bool(imp.value), bool(done.value)

    def run_epochs(self, net: int, max_now: int):
        done = c_int()
        st = _check(lib().n2f_run_epochs(self._ptr, net, max_now, byref(done)))
        return bool(done.value), st

    def result(self):
        import torch
        out = torch.empty((self.C, self.H, self.W), dtype=torch.float32, device=self.device)
        _check(lib().n2f_result(self._ptr, c_void_p(out.data_ptr())))
        return out

    def get_state(self, net: int = 0):
        th = np.empty(self.nparams, np.float32)
        m = np.empty(self.nparams, np.float32)
        v = np.empty(self.nparams, np.float32)
        t = c_longlong()
        _check(lib().n2f_get_state(self._ptr, net, th.ctypes.data, m.ctypes.data, v.ctypes.data, byref(t)))
        return th, m, v, t.value

    def set_state(self, net: int, theta, m=None, v=None, t: int = 0):
        th = np.ascontiguousarray(theta, np.float32)
        mm = None if m is None else np.ascontiguousarray(m, np.float32)
        vv = None if v is None else np.ascontiguousarray(v, np.float32)
        assert th.size == self.nparams
        _check(lib().n2f_set_state(self._ptr, net, th.ctypes.data, None if mm is None else mm.ctypes.data,
                                   None if vv is None else vv.ctypes.data, int(t)))

    def save_checkpoint(self, net: int = 0) -> np.ndarray:
        """Opaque checkpoint of network `net` (uint8 host array)."""
        nb = c_size_t()
        _check(lib().n2f_checkpoint_bytes(self._ptr, byref(nb)))
        buf = np.empty(nb.value, np.uint8)
        _check(lib().n2f_save_checkpoint(self._ptr, net, buf.ctypes.data, nb.value))
        return buf

    def load_checkpoint(self, net: int, buf) -> None:
        b = np.ascontiguousarray(buf, np.uint8)
        _check(lib().n2f_load_checkpoint(self._ptr, net, b.ctypes.data, b.size))

    def get_grad(self, net: int = 0):
        g = np.empty(self.nparams, np.float32)
        loss = c_double()
        _check(lib().n2f_get_grad(self._ptr, net, g.ctypes.data, byref(loss)))
        return g, loss.value

    def debug_adam(self, net: int, g):
        gg = np.ascontiguousarray(g, np.float32)
        _check(lib().n2f_debug_adam(self._ptr, net, gg.ctypes.data))

    def progress(self, net: int = 0):
        e, be, ns, best = c_int(), c_int(), c_int(), c_double()
        _check(lib().n2f_get_progress(self._ptr, net, byref(e), byref(be), byref(ns), byref(best)))
        return e.value, be.value, ns.value, best.value

    def history(self, net: int = 0):
        e = self.progress(net)[0]
        out = np.empty(e, np.float64)
        _check(lib().n2f_get_history(self._ptr, net, e, out.ctypes.data if e else None))
        return out

    def lohi(self):
        lo, hi = c_float(), c_float()
        _check(lib().n2f_get_lohi(self._ptr, byref(lo), byref(hi)))
        return lo.value, hi.value

    def image(self, which: int):
        import torch
        Hc, Wc = self.H - self.H % 2, self.W - self.W % 2
        if self.cfg.downsample == DS_QUAD:
            shapes = {i: (self.C, Hc // 2, Wc // 2) for i in range(4)}
        else:
            shapes = {0: (self.C, Hc, Wc // 2), 1: (self.C, Hc, Wc // 2), 2: (self.C, Hc // 2, Wc),
                      3: (self.C, Hc // 2, Wc)}
        shapes[4] = (self.C, self.H, self.W)
        for p in range(4):
            shapes[8 + p] = shapes[p]
        shape = shapes.get(which, (self.H, self.W))
        out = torch.empty(shape, dtype=torch.float32, device=self.device)
        _check(lib().n2f_get_image(self._ptr, which, c_void_p(out.data_ptr())))
        return out


def denoise(x, cfg: Config | None = None, ws=None):
    """One-shot denoise of a (C, H, W) FP32 CUDA tensor; returns (y, status)."""
    import torch
    _check_image(x)
    cfg = cfg or default_config()
    C, H, W = (int(s) for s in x.shape)
    nbytes = workspace_bytes(H, W, C, cfg)
    ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    if not (ws.is_cuda and ws.device == x.device and ws.numel() * ws.element_size() >= nbytes):
        raise ValueError("workspace must be a CUDA tensor on the image's device of at least workspace_bytes()")
    out = torch.empty_like(x)
    st = _check(lib().n2f_denoise(c_void_p(x.data_ptr()), c_void_p(out.data_ptr()), H, W, C, byref(cfg),
                                  c_void_p(ws.data_ptr()), nbytes, _stream_of(x)))
    return out, st


def denoise_noalloc(x, cfg: Config | None = None, out=None):
    """One-shot denoise through the entry point that allocates no device
    memory (its workspace is a fixed array inside the library); returns
    (y, status).  Pass `out` (same shape, FP32, contiguous, same device) to
    allocate nothing here either."""
    import torch
    _check_image(x)
    cfg = cfg or default_config()
    C, H, W = (int(s) for s in x.shape)
    if out is None:
        out = torch.empty_like(x)
    _check_image(out, "out")
    if tuple(out.shape) != tuple(x.shape) or out.device != x.device:
        raise ValueError("out must have the image's shape and device")
    st = _check(lib().n2f_denoise_noalloc(c_void_p(x.data_ptr()), c_void_p(out.data_ptr()), H, W, C, byref(cfg),
                                          _stream_of(x)))
    return out, st


def max_project(stack, out=None):
    """Maximum-intensity projection along the first axis of a (Z, ...) FP32
    contiguous CUDA tensor; returns a tensor of the remaining shape."""
    import torch
    assert stack.is_cuda and stack.dtype == torch.float32 and stack.is_contiguous() and stack.dim() >= 2
    nz = int(stack.shape[0])
    npix = stack[0].numel()
    if out is None:
        out = torch.empty(stack.shape[1:], dtype=torch.float32, device=stack.device)
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.numel() == npix
    _check(lib().n2f_max_project(c_void_p(stack.data_ptr()), nz, npix, c_void_p(out.data_ptr()), _stream_of(stack)))
    return out


def profile_begin(every: int = 1):
    _check(lib().n2f_profile_begin(every))


def profile_read(kernel_class: int):
    """(total kernel ms, launches, pixels processed) for one kernel class."""
    ms, n, px = c_double(), c_longlong(), c_longlong()
    _check(lib().n2f_profile_read(kernel_class, byref(ms), byref(n), byref(px)))
    return ms.value, n.value, px.value


def profile_end():
    _check(lib().n2f_profile_end())


MAX_GROUP_GRID = 1024       # N2F_MAX_GROUP_GRID


def group_grid(kind: int) -> int:
    """Hardware blocks of one grouped launch of `kind` (see n2f.h)."""
    g = c_int()
    _check(lib().n2f_group_grid_get(kind, byref(g)))
    return g.value


def set_group_grid(kind: int, grid: int):
    """Set the launch geometry of grouped kind `kind`; results do not change."""
    _check(lib().n2f_group_grid_set(kind, grid))


def _ints(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32))


class Batch:
    """Independent images of uneven sizes trained together (see n2f.h).

    n_streams = 0 runs every image on the caller's current stream;
    n_streams = BATCH_GROUPED (BF16) makes every launch of an epoch one
    grouped launch over all images, replayed as one graph per epoch on the
    caller's current stream; n_streams = -K (K = 2..4, BF16) splits the
    images into K groups launched on K streams of the batch's own."""

    def __init__(self, images, cfg: Config | None = None, n_streams: int = 4):
        import torch
        self.cfg = cfg or default_config()
        self.images = [x.contiguous() for x in images]
        for x in self.images:
            _check_image(x)
        self.shapes = [tuple(int(d) for d in x.shape) for x in self.images]
        self.extra_ws = {}   # workspaces of images joined by add(), kept until removed
        n = len(self.images)
        C = _ints([s[0] for s in self.shapes])
        H = _ints([s[1] for s in self.shapes])
        W = _ints([s[2] for s in self.shapes])
        nb = c_size_t()
        _check(lib().n2f_batch_workspace_bytes(n, H.ctypes.data, W.ctypes.data, C.ctypes.data, byref(self.cfg),
                                               byref(nb)))
        dev = self.images[0].device
        if any(x.device != dev for x in self.images):
            raise ValueError("all images of a batch must be on one device")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        ptrs = (c_void_p * n)(*[x.data_ptr() for x in self.images])
        self._ptr = c_void_p()
        _check(lib().n2f_batch_create(byref(self._ptr), n, ptrs, H.ctypes.data, W.ctypes.data, C.ctypes.data,
                                      byref(self.cfg), c_void_p(self.ws.data_ptr()), nb.value, n_streams,
                                      _stream_of(self.images[0])))

    def add(self, x) -> int:
        """Join image x (C, H, W) at the next epoch boundary; returns its index."""
        import torch
        x = x.contiguous()
        _check_image(x)
        C, H, W = (int(d) for d in x.shape)
        nbytes = workspace_bytes(H, W, C, self.cfg)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        idx = c_int()
        _check(lib().n2f_batch_add(self._ptr, c_void_p(x.data_ptr()), H, W, C, c_void_p(ws.data_ptr()), nbytes,
                                   byref(idx)))
        self.images.append(x)
        self.shapes.append((C, H, W))
        self.extra_ws[idx.value] = ws
        return idx.value

    def remove(self, i: int):
        """Image i leaves the batch; its workspace is released."""
        _check(lib().n2f_batch_remove(self._ptr, i))
        self.extra_ws.pop(i, None)

    def run(self, max_epochs: int = 100000):
        a = c_int()
        _check(lib().n2f_batch_run(self._ptr, max_epochs, byref(a)))
        return a.value

    def result(self, i: int):
        import torch
        out = torch.empty(self.shapes[i], dtype=torch.float32, device=self.images[i].device)
        _check(lib().n2f_batch_result(self._ptr, i, c_void_p(out.data_ptr())))
        return out

    def progress(self, i: int):
        e, f = c_int(), c_int()
        _check(lib().n2f_batch_progress(self._ptr, i, byref(e), byref(f)))
        return e.value, bool(f.value)

    def run_of(self, i: int) -> Run:
        """State-exchange handle on image i's run (valid while the batch lives)."""
        p = c_void_p()
        _check(lib().n2f_batch_run_of(self._ptr, i, byref(p)))
        return Run._view(p, self.shapes[i], self.cfg, self.images[i].device)

    def close(self):
        if self._ptr:
            lib().n2f_batch_destroy(self._ptr)
            self._ptr = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over one device arena (see n2f.h)."""

    def __init__(self, arena_bytes: int, cfg: Config | None = None, n_streams: int = 4, max_active: int = 64,
                 simulate: bool = False, device="cuda:0", grouped: bool = False):
        """grouped=True (BF16): grouped launches over all active requests of a
        channel count; the launch tables are added to arena_bytes here."""
        self.cfg = cfg or default_config()
        self.arena = None
        self._keep = {}   # request id -> (x, out), alive until reported finished
        if grouped and not simulate:
            tb = c_size_t()
            _check(lib().n2f_server_table_bytes(max_active, byref(tb)))
            arena_bytes += tb.value
        ptr = None
        if not simulate:
            import torch
            self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
            ptr = self.arena.data_ptr()
        self._ptr = c_void_p()
        flags = (SERVER_SIMULATE if simulate else 0) | (SERVER_GROUPED if grouped else 0)
        _check(lib().n2f_server_create(byref(self._ptr), byref(self.cfg), ptr, arena_bytes, n_streams, max_active,
                                       flags))

    def submit(self, rid: int, x=None, out=None, H: int = 0, W: int = 0, C: int = 1, sim_epochs: int = 0):
        """Queue request rid.  A real server takes x and out, (C, H, W) FP32
        contiguous CUDA tensors of one shape; both are kept referenced here
        until poll() reports rid, and x is read only after the work already
        queued on the current stream."""
        stream = None
        if x is not None or out is not None:
            _check_image(x, "x")
            _check_image(out, "out")
            if tuple(x.shape) != tuple(out.shape) or x.device != out.device:
                raise ValueError("x and out must have the same shape and device")
            C, H, W = (int(d) for d in x.shape)
            stream = _stream_of(x)
        st = _check(lib().n2f_server_submit(self._ptr, rid, None if x is None else c_void_p(x.data_ptr()),
                                            None if out is None else c_void_p(out.data_ptr()), H, W, C, sim_epochs,
                                            stream))
        if x is not None:
            self._keep[rid] = (x, out)
        return st

    def cancel(self, rid: int):
        """Cancel a queued or active request; poll() reports it as ECANCELED."""
        _check(lib().n2f_server_cancel(self._ptr, rid))

    def step(self, epochs: int = 1):
        a, q = c_int(), c_int()
        _check(lib().n2f_server_step(self._ptr, epochs, byref(a), byref(q)))
        return a.value, q.value

    def poll(self, max_n: int = 4096):
        ids = np.empty(max_n, np.int64)
        st = np.empty(max_n, np.int32)
        n = c_int()
        _check(lib().n2f_server_poll(self._ptr, ids.ctypes.data, st.ctypes.data, max_n, byref(n)))
        done = list(zip(ids[:n.value].tolist(), st[:n.value].tolist()))
        for rid, _ in done:
            self._keep.pop(rid, None)
        return done

    def memory(self):
        u, l = c_size_t(), c_size_t()
        _check(lib().n2f_server_memory(self._ptr, byref(u), byref(l)))
        return u.value, l.value

    def close(self):
        if self._ptr:
            lib().n2f_server_destroy(self._ptr)
            self._ptr = c_void_p()
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
