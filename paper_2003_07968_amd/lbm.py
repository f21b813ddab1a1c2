"""Python binding of the C ABI in include/lbm.h (liblbm.so, HIP for gfx950).

The functions below carry the C names and only marshal arguments: every step
of the lattice update runs in the library's HIP kernels.  PyTorch provides
device memory and the stream.  The library must have been built
(`python -m paper_2003_07968_amd.build`); loading fails loudly otherwise, and
there is no CPU fallback.

Arrays: fields are torch.float64 CUDA tensors of shape (ny, nx), populations
(9, ny, nx), contiguous, on the device of the stream.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
LBM_ERR_INVALID_ARG = -1
LBM_ERR_DOMAIN = -2
LBM_ERR_DEVICE = -3
LBM_ERR_OOM = -4
LBM_ERR_STATE = -5
LBM_STORE_F64 = 0
LBM_STORE_F32_SHIFTED = 1
LBM_STORE_F16_SHIFTED = 2
LBM_STORE_F16_LOCAL = 3
LBM_COLL_BGK = 0
LBM_COLL_MRT = 1

_ALIGN = 256


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("tau", ctypes.c_double), ("G", ctypes.c_double),
        ("epsilon", ctypes.c_double), ("sigma", ctypes.c_double),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double),
        ("eos_c", ctypes.c_double), ("eos_k", ctypes.c_double), ("T", ctypes.c_double),
        ("force_on", ctypes.c_int32), ("m2_trace_alt", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("rho_ref", ctypes.c_double),
        ("collision", ctypes.c_int32),
        ("tau_rho", ctypes.c_double), ("tau_e", ctypes.c_double), ("tau_zeta", ctypes.c_double),
        ("tau_j", ctypes.c_double), ("tau_q", ctypes.c_double),
    ]


class lbm_server_config(ctypes.Structure):
    _fields_ = [("max_resident", ctypes.c_int32), ("quantum", ctypes.c_int32),
                ("max_bypass", ctypes.c_int32)]


class lbm_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("rounds", ctypes.c_int64), ("cell_steps", ctypes.c_int64),
                ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t)]


class LbmError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        text = _load().lbm_status_string(status).decode()
        super().__init__(f"{text}: {message}" if message else text)


_lib = None
_VP = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing; build it with `python -m paper_2003_07968_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(lbm_params)
        H = ctypes.c_void_p
        lib.lbm_workspace_bytes.argtypes = [P]
        lib.lbm_workspace_bytes.restype = ctypes.c_size_t
        lib.lbm_init.argtypes = [P, _VP, ctypes.c_size_t, _VP, _VP, _VP, _VP,
                                 ctypes.POINTER(H)]
        lib.lbm_init.restype = ctypes.c_int
        lib.lbm_step.argtypes = [H, ctypes.c_int64]
        lib.lbm_step.restype = ctypes.c_int
        lib.lbm_sync.argtypes = [H]
        lib.lbm_sync.restype = ctypes.c_int
        lib.lbm_moments.argtypes = [H] + [_VP] * 6
        lib.lbm_moments.restype = ctypes.c_int
        lib.lbm_diagnostics.argtypes = [H, ctypes.POINTER(ctypes.c_double)]
        lib.lbm_diagnostics.restype = ctypes.c_int
        lib.lbm_diagnostics_noalloc.argtypes = [H, ctypes.POINTER(ctypes.c_double)]
        lib.lbm_diagnostics_noalloc.restype = ctypes.c_int
        lib.lbm_get_populations.argtypes = [H, _VP]
        lib.lbm_get_populations.restype = ctypes.c_int
        lib.lbm_set_populations.argtypes = [H, _VP, ctypes.c_int64]
        lib.lbm_set_populations.restype = ctypes.c_int
        lib.lbm_time.argtypes = [H]
        lib.lbm_time.restype = ctypes.c_int64
        lib.lbm_set_launch.argtypes = [H, ctypes.c_int32, ctypes.c_int32]
        lib.lbm_set_launch.restype = ctypes.c_int
        lib.lbm_set_fusion.argtypes = [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.lbm_set_fusion.restype = ctypes.c_int
        lib.lbm_get_fusion.argtypes = [H]
        lib.lbm_get_fusion.restype = ctypes.c_int32
        lib.lbm_get_launch.argtypes = [H, ctypes.POINTER(ctypes.c_int32)]
        lib.lbm_get_launch.restype = ctypes.c_int
        lib.lbm_status_string.argtypes = [ctypes.c_int]
        lib.lbm_status_string.restype = ctypes.c_char_p
        lib.lbm_last_error.argtypes = [H]
        lib.lbm_last_error.restype = ctypes.c_char_p
        lib.lbm_destroy.argtypes = [H]
        lib.lbm_destroy.restype = None
        D3 = ctypes.POINTER(ctypes.c_double)
        lib.lbm_autotune.argtypes = [H, D3]
        lib.lbm_autotune.restype = ctypes.c_int
        B = ctypes.c_void_p
        lib.lbm_batch_workspace_bytes.argtypes = [ctypes.c_int32]
        lib.lbm_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.lbm_batch_create.argtypes = [ctypes.c_int32, _VP, ctypes.c_size_t, _VP,
                                         ctypes.POINTER(B)]
        lib.lbm_batch_create.restype = ctypes.c_int
        lib.lbm_batch_add.argtypes = [B, H]
        lib.lbm_batch_add.restype = ctypes.c_int
        lib.lbm_batch_remove.argtypes = [B, H]
        lib.lbm_batch_remove.restype = ctypes.c_int
        lib.lbm_batch_size.argtypes = [B]
        lib.lbm_batch_size.restype = ctypes.c_int32
        lib.lbm_batch_step.argtypes = [B, ctypes.c_int64]
        lib.lbm_batch_step.restype = ctypes.c_int
        lib.lbm_batch_autotune.argtypes = [B, D3]
        lib.lbm_batch_autotune.restype = ctypes.c_int
        lib.lbm_batch_set_fusion.argtypes = [B, ctypes.c_int32]
        lib.lbm_batch_set_fusion.restype = ctypes.c_int
        lib.lbm_batch_get_fusion.argtypes = [B]
        lib.lbm_batch_get_fusion.restype = ctypes.c_int32
        lib.lbm_batch_set_launch.argtypes = [B, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.lbm_batch_set_launch.restype = ctypes.c_int
        lib.lbm_batch_get_launch.argtypes = [B, ctypes.POINTER(ctypes.c_int32)]
        lib.lbm_batch_get_launch.restype = ctypes.c_int
        lib.lbm_batch_destroy.argtypes = [B]
        lib.lbm_batch_destroy.restype = None
        lib.lbm_probe_stream_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.lbm_probe_stream_bytes.restype = ctypes.c_size_t
        lib.lbm_probe_stream.argtypes = [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         _VP]
        lib.lbm_probe_stream.restype = ctypes.c_int
        S = ctypes.c_void_p
        DP = ctypes.POINTER(ctypes.c_double)
        lib.lbm_server_create.argtypes = [ctypes.POINTER(lbm_server_config), _VP,
                                          ctypes.c_size_t, _VP, ctypes.POINTER(S)]
        lib.lbm_server_create.restype = ctypes.c_int
        lib.lbm_server_job_bytes.argtypes = [P, ctypes.c_int32]
        lib.lbm_server_job_bytes.restype = ctypes.c_size_t
        lib.lbm_server_submit.argtypes = [S, P, DP, ctypes.c_int64, DP, DP,
                                          ctypes.POINTER(ctypes.c_int64)]
        lib.lbm_server_submit.restype = ctypes.c_int
        lib.lbm_server_advance.argtypes = [S, ctypes.POINTER(ctypes.c_int32)]
        lib.lbm_server_advance.restype = ctypes.c_int
        lib.lbm_server_poll.argtypes = [S, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        lib.lbm_server_poll.restype = ctypes.c_int32
        lib.lbm_server_get_stats.argtypes = [S, ctypes.POINTER(lbm_server_stats)]
        lib.lbm_server_get_stats.restype = ctypes.c_int
        lib.lbm_server_destroy.argtypes = [S]
        lib.lbm_server_destroy.restype = None
        _lib = lib
    return _lib


EXPORTED = ("lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_sync", "lbm_moments",
            "lbm_diagnostics", "lbm_diagnostics_noalloc", "lbm_get_populations", "lbm_set_populations", "lbm_time",
            "lbm_set_launch", "lbm_set_fusion", "lbm_get_fusion", "lbm_get_launch", "lbm_autotune", "lbm_batch_workspace_bytes",
            "lbm_batch_create", "lbm_batch_add", "lbm_batch_remove", "lbm_batch_size",
            "lbm_batch_step", "lbm_batch_autotune", "lbm_batch_set_fusion",
            "lbm_batch_get_fusion", "lbm_batch_set_launch", "lbm_batch_get_launch",
            "lbm_batch_destroy", "lbm_status_string",
            "lbm_last_error", "lbm_destroy", "lbm_server_create", "lbm_server_job_bytes",
            "lbm_server_submit", "lbm_server_advance", "lbm_server_poll",
            "lbm_server_get_stats", "lbm_server_destroy", "lbm_probe_stream_bytes",
            "lbm_probe_stream")


def make_params(p: dict) -> lbm_params:
    """lbm_params from a dictionary with the struct's field names."""
    return lbm_params(int(p["nx"]), int(p["ny"]), float(p["tau"]), float(p["G"]),
                      float(p["epsilon"]), float(p["sigma"]), float(p["eos_a"]),
                      float(p["eos_b"]), float(p["eos_c"]), float(p["eos_k"]), float(p["T"]),
                      int(bool(p.get("force_on", True))), int(bool(p.get("m2_trace_alt", False))),
                      int(p.get("storage", LBM_STORE_F64)), float(p.get("rho_ref", 0.0)),
                      int(p.get("collision", LBM_COLL_BGK)),
                      *[float(p.get(k, 1.0)) for k in ("tau_rho", "tau_e", "tau_zeta", "tau_j",
                                                       "tau_q")])


def _dev_ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


# ---- the C functions, one to one ----

def lbm_workspace_bytes(params: lbm_params) -> int:
    return _load().lbm_workspace_bytes(ctypes.byref(params))


def lbm_init(params, workspace, rho0, ux0=None, uy0=None, stream=None):
    """Returns a handle (an opaque integer)."""
    lib = _load()
    h = ctypes.c_void_p()
    ws_ptr = workspace.data_ptr()
    ws_bytes = workspace.numel() * workspace.element_size()
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib.lbm_init(ctypes.byref(params), ctypes.c_void_p(ws_ptr), ws_bytes, _dev_ptr(rho0),
                      _dev_ptr(ux0), _dev_ptr(uy0), ctypes.c_void_p(s.cuda_stream),
                      ctypes.byref(h))
    if st != LBM_OK:
        raise LbmError(st)
    return h.value


def _check(h, st):
    if st != LBM_OK:
        raise LbmError(st, _load().lbm_last_error(h).decode())


def lbm_step(h, nsteps):
    _check(h, _load().lbm_step(h, int(nsteps)))


def lbm_sync(h):
    return _load().lbm_sync(h)


def lbm_moments(h, rho=None, ux=None, uy=None, Fx=None, Fy=None, psi=None):
    _check(h, _load().lbm_moments(h, *[_dev_ptr(t) for t in (rho, ux, uy, Fx, Fy, psi)]))


def lbm_diagnostics(h):
    out = (ctypes.c_double * 6)()
    _check(h, _load().lbm_diagnostics(h, out))
    return list(out)


def lbm_diagnostics_noalloc(h):
    out = (ctypes.c_double * 6)()
    _check(h, _load().lbm_diagnostics_noalloc(h, out))
    return list(out)


def lbm_get_populations(h, f):
    _check(h, _load().lbm_get_populations(h, _dev_ptr(f)))


def lbm_set_populations(h, f, t):
    _check(h, _load().lbm_set_populations(h, _dev_ptr(f), int(t)))


def lbm_time(h):
    return _load().lbm_time(h)


def lbm_set_launch(h, block_x=0, seg_rows=0):
    _check(h, _load().lbm_set_launch(h, int(block_x), int(seg_rows)))


def lbm_set_fusion(h, steps, block_x=0, seg_rows=0):
    _check(h, _load().lbm_set_fusion(h, int(steps), int(block_x), int(seg_rows)))


def lbm_get_fusion(h):
    return _load().lbm_get_fusion(h)


def lbm_get_launch(h):
    out = (ctypes.c_int32 * 3)()
    _check(h, _load().lbm_get_launch(h, out))
    return tuple(out)


def lbm_autotune(h):
    out = (ctypes.c_double * 3)()
    _check(h, _load().lbm_autotune(h, out))
    return int(out[0]), int(out[1]), float(out[2])


def lbm_batch_workspace_bytes(capacity):
    return _load().lbm_batch_workspace_bytes(int(capacity))


def lbm_batch_create(capacity, workspace, stream=None):
    b = ctypes.c_void_p()
    s = stream if stream is not None else torch.cuda.current_stream()
    st = _load().lbm_batch_create(int(capacity), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel() * workspace.element_size(),
                                  ctypes.c_void_p(s.cuda_stream), ctypes.byref(b))
    if st != LBM_OK:
        raise LbmError(st)
    return b.value


def _check_b(st):
    if st != LBM_OK:
        raise LbmError(st)


def lbm_batch_add(b, h):
    _check_b(_load().lbm_batch_add(b, h))


def lbm_batch_remove(b, h):
    _check_b(_load().lbm_batch_remove(b, h))


def lbm_batch_size(b):
    return _load().lbm_batch_size(b)


def lbm_batch_step(b, nsteps):
    _check_b(_load().lbm_batch_step(b, int(nsteps)))


def lbm_batch_autotune(b):
    out = (ctypes.c_double * 3)()
    _check_b(_load().lbm_batch_autotune(b, out))
    return int(out[0]), int(out[1]), float(out[2])


def lbm_batch_set_fusion(b, steps):
    _check_b(_load().lbm_batch_set_fusion(b, int(steps)))


def lbm_batch_get_fusion(b):
    return _load().lbm_batch_get_fusion(b)


def lbm_batch_set_launch(b, steps, block_x, seg_rows=0):
    _check_b(_load().lbm_batch_set_launch(b, int(steps), int(block_x), int(seg_rows)))


def lbm_batch_get_launch(b):
    out = (ctypes.c_int32 * 3)()
    _check_b(_load().lbm_batch_get_launch(b, out))
    return int(out[0]), int(out[1]), int(out[2])


def lbm_probe_stream_bytes(nx, ny):
    return int(_load().lbm_probe_stream_bytes(int(nx), int(ny)))


def lbm_probe_stream(src, dst, nx, ny, seg_rows=32, stream=None):
    """One pulled copy of nine FP64 population planes (the step kernels'
    access pattern without their arithmetic) between two device tensors of
    lbm_probe_stream_bytes(nx, ny) bytes, on `stream` (default: torch's
    current stream)."""
    stream = stream if stream is not None else torch.cuda.current_stream(src.device)
    need = lbm_probe_stream_bytes(nx, ny)
    for t in (src, dst):
        if t.device.type != "cuda" or t.numel() * t.element_size() < need:
            raise ValueError(f"probe buffers must be device tensors of at least {need} bytes")
    st = _load().lbm_probe_stream(_dev_ptr(src), _dev_ptr(dst), int(nx), int(ny), int(seg_rows),
                                  ctypes.c_void_p(stream.cuda_stream))
    if st != LBM_OK:
        raise LbmError(st)


def lbm_batch_destroy(b):
    _load().lbm_batch_destroy(b)


def lbm_server_create(max_resident, quantum, max_bypass, arena, stream):
    srv = ctypes.c_void_p()
    cfg = lbm_server_config(int(max_resident), int(quantum), int(max_bypass))
    _check_b(_load().lbm_server_create(ctypes.byref(cfg), ctypes.c_void_p(arena.data_ptr()),
                                       arena.numel() * arena.element_size(),
                                       ctypes.c_void_p(stream.cuda_stream), ctypes.byref(srv)))
    return srv.value


def lbm_server_job_bytes(params, want_populations=False):
    return _load().lbm_server_job_bytes(ctypes.byref(params), int(bool(want_populations)))


def _host_ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lbm_server_submit(srv, params, rho0, nsteps, rho_out=None, f_out=None):
    """rho0, rho_out, f_out: C-contiguous float64 NumPy arrays on the host."""
    job = ctypes.c_int64()
    _check_b(_load().lbm_server_submit(srv, ctypes.byref(params), _host_ptr(rho0), int(nsteps),
                                       _host_ptr(rho_out), _host_ptr(f_out), ctypes.byref(job)))
    return job.value


def lbm_server_advance(srv):
    n = ctypes.c_int32()
    _check_b(_load().lbm_server_advance(srv, ctypes.byref(n)))
    return n.value


def lbm_server_poll(srv, max_jobs=1024):
    ids = (ctypes.c_int64 * max_jobs)()
    sts = (ctypes.c_int32 * max_jobs)()
    n = _load().lbm_server_poll(srv, ids, sts, max_jobs)
    return [(ids[k], sts[k]) for k in range(n)]


def lbm_server_get_stats(srv):
    out = lbm_server_stats()
    _check_b(_load().lbm_server_get_stats(srv, ctypes.byref(out)))
    return {name: getattr(out, name) for name, _ in out._fields_}


def lbm_server_destroy(srv):
    _load().lbm_server_destroy(srv)


def lbm_last_error(h):
    return _load().lbm_last_error(h).decode()


def lbm_destroy(h):
    _load().lbm_destroy(h)


def _pinned(shape):
    """A float64 numpy array in page-locked host memory."""
    return torch.empty(shape, dtype=torch.float64, pin_memory=True).numpy()


# ---- convenience wrapper owning its torch workspace ----

class Lattice:
    """One periodic lattice on the current CUDA device and stream."""

    def __init__(self, p: dict, rho0, ux0=None, uy0=None, device="cuda", stream=None):
        self.params = make_params(p)
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = lbm_workspace_bytes(self.params)
        if nbytes == 0:
            raise LbmError(LBM_ERR_INVALID_ARG, "parameters rejected")
        # torch's caching allocator hands out 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.workspace.data_ptr() % _ALIGN == 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        if self.stream != torch.cuda.current_stream(device):
            # the library's work runs on self.stream: keep the caching allocator
            # from reusing the workspace before that work is done
            self.workspace.record_stream(self.stream)

        def dev(a):
            if a is None:
                return None
            t = torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
            return t
        self._rho0, self._ux0, self._uy0 = dev(rho0), dev(ux0), dev(uy0)
        if self.stream != torch.cuda.current_stream(device):
            for t in (self._rho0, self._ux0, self._uy0):
                if t is not None:
                    t.record_stream(self.stream)
        self.handle = lbm_init(self.params, self.workspace, self._rho0, self._ux0, self._uy0,
                               self.stream)

    def step(self, n=1):
        lbm_step(self.handle, n)

    def sync(self):
        st = lbm_sync(self.handle)
        if st != LBM_OK:
            raise LbmError(st, lbm_last_error(self.handle))

    @property
    def t(self):
        return lbm_time(self.handle)

    def moments(self):
        shape = (self.ny, self.nx)
        out = {k: torch.empty(shape, dtype=torch.float64, device=self.workspace.device)
               for k in ("rho", "ux", "uy", "Fx", "Fy", "psi")}
        lbm_moments(self.handle, **out)
        return out

    def diagnostics(self):
        v = lbm_diagnostics(self.handle)
        return dict(zip(["mass", "mom_x", "mom_y", "ssc_num", "ssc_den", "umax"], v))

    def populations(self):
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.workspace.device)
        lbm_get_populations(self.handle, f)
        return f

    def set_populations(self, f, t):
        lbm_set_populations(self.handle, f.contiguous(), t)

    def set_launch(self, block_x=0, seg_rows=0):
        lbm_set_launch(self.handle, block_x, seg_rows)

    def set_fusion(self, steps, block_x=0, seg_rows=0):
        lbm_set_fusion(self.handle, steps, block_x, seg_rows)

    def fusion(self):
        return lbm_get_fusion(self.handle)

    def launch(self):
        return lbm_get_launch(self.handle)

    def autotune(self):
        return lbm_autotune(self.handle)

    def close(self):
        if self.handle:
            lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A group of Lattice objects advanced together: one kernel launch covers every
    member, per two time steps (the two-step pass) or per step."""

    def __init__(self, capacity, device="cuda", stream=None):
        self.workspace = torch.empty(lbm_batch_workspace_bytes(capacity), dtype=torch.uint8,
                                     device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        if self.stream != torch.cuda.current_stream(device):
            self.workspace.record_stream(self.stream)
        self.handle = lbm_batch_create(capacity, self.workspace, self.stream)
        self.members = []

    def add(self, lat):
        lbm_batch_add(self.handle, lat.handle)
        self.members.append(lat)

    def remove(self, lat):
        lbm_batch_remove(self.handle, lat.handle)
        self.members.remove(lat)

    def __len__(self):
        return lbm_batch_size(self.handle)

    def step(self, n=1):
        lbm_batch_step(self.handle, n)

    def autotune(self):
        return lbm_batch_autotune(self.handle)

    def set_fusion(self, steps):
        lbm_batch_set_fusion(self.handle, steps)

    def fusion(self):
        return lbm_batch_get_fusion(self.handle)

    def set_launch(self, steps, block_x, seg_rows=0):
        lbm_batch_set_launch(self.handle, steps, block_x, seg_rows)

    def launch(self):
        """(steps per launch, block_x, seg_rows) in use."""
        return lbm_batch_get_launch(self.handle)

    def close(self):
        if self.handle:
            lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching serving loop (include/lbm_server.h) over an arena of
    `arena_bytes` device bytes on a stream of its own.  submit() takes host
    NumPy arrays and keeps the output arrays alive until the job is polled."""

    def __init__(self, arena_bytes, max_resident=256, quantum=64, max_bypass=8, device="cuda",
                 stream=None):
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        # the server's work runs on its own stream, which the caching allocator
        # must wait for before it reuses the arena
        self.arena.record_stream(self.stream)
        self.handle = lbm_server_create(max_resident, quantum, max_bypass, self.arena,
                                        self.stream)
        self._outputs = {}

    def submit(self, p: dict, rho0, nsteps, want_rho=True, want_populations=False):
        params = make_params(p)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (params.ny, params.nx)
        # outputs in page-locked host memory, so the server's copies at
        # retirement are direct DMA; the arrays keep their pinned tensors alive
        rho = _pinned((params.ny, params.nx)) if want_rho else None
        f = _pinned((9, params.ny, params.nx)) if want_populations else None
        job = lbm_server_submit(self.handle, params, rho0, nsteps, rho, f)
        self._outputs[job] = (rho, f)
        return job

    def advance(self):
        return lbm_server_advance(self.handle)

    def poll(self):
        """[(job id, status, rho or None, populations or None)] of jobs finished
        since the last poll."""
        return [(j, st) + self._outputs.pop(j) for j, st in lbm_server_poll(self.handle)]

    def stats(self):
        return lbm_server_get_stats(self.handle)

    def close(self):
        if self.handle:
            lbm_server_destroy(self.handle)   # waits for the server's stream
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
