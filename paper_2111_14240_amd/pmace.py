"""ctypes binding of libpmace.so (include/pmace.h).

Argument marshalling only: every step of the PMACE iteration runs in the HIP
library.  PyTorch supplies device memory (the caller-owned workspace and the
input/output tensors) and the current HIP stream.  If the library has not
been built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmace.so")

PMACE_OK = 0
PMACE_EINVAL = 1
PMACE_EUNSUPPORTED = 2
PMACE_ENOMEM = 3
PMACE_EDEVICE = 4
PMACE_ESTATE = 5
PMACE_EDIVERGED = 6
PMACE_CENTERED_DC = 0x1
PMACE_STAGED_AGENT = 0x2
PMACE_SPLIT_AGENT = 0x4
PMACE_ROWSPEC_AGENT = 0x8
PMACE_METHOD_PMACE = 0
PMACE_METHOD_SHARP_PLUS = 1
PMACE_STOP_NRMSE = 0
PMACE_STOP_DATA_FIT = 1

STATUS_NAMES = {
    0: "PMACE_OK", 1: "PMACE_EINVAL", 2: "PMACE_EUNSUPPORTED", 3: "PMACE_ENOMEM",
    4: "PMACE_EDEVICE", 5: "PMACE_ESTATE", 6: "PMACE_EDIVERGED",
}


class pmace_params(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("np", ctypes.c_int32),
        ("num_pos", ctypes.c_int32), ("alpha", ctypes.c_float), ("kappa", ctypes.c_float),
        ("rho", ctypes.c_float), ("flags", ctypes.c_uint32), ("chunk", ctypes.c_int32),
        ("method", ctypes.c_int32), ("beta", ctypes.c_float), ("ppw", ctypes.c_int32),
    ]


class pmace_stop_rule(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_float), ("min_iter", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("criterion", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class PMACEError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({_status_str(status)})")


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpmace.so and declare the C signatures (raises if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the PMACE path has no CPU fallback)")
    # The device memory and streams passed in come from PyTorch's HIP runtime,
    # which PyTorch ships as its own libamdhip64.  Loaded first, it is the one
    # the library's HIP dependency binds to; loaded after the library, the
    # process holds two HIP runtimes and the library rejects PyTorch's pointers.
    _torch()
    L = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    P = ctypes.POINTER(pmace_params)
    L.pmace_footprint.argtypes = [P]
    L.pmace_footprint.restype = sz
    L.pmace_init.argtypes = [P, vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    L.pmace_init.restype = ctypes.c_int
    for name in ("pmace_reconstruct", "pmace_get_state", "pmace_set_state"):
        getattr(L, name).argtypes = [vp, vp]
        getattr(L, name).restype = ctypes.c_int
    L.pmace_iterate.argtypes = [vp, i32]
    L.pmace_iterate.restype = ctypes.c_int
    L.pmace_sync.argtypes = [vp]
    L.pmace_sync.restype = ctypes.c_int
    L.pmace_destroy.argtypes = [vp]
    L.pmace_destroy.restype = None
    L.pmace_status_str.argtypes = [ctypes.c_int]
    L.pmace_status_str.restype = ctypes.c_char_p
    L.pmace_fft2.argtypes = [i32, i32, vp, vp, i32, vp]
    L.pmace_fft2.restype = ctypes.c_int
    L.pmace_set_reference.argtypes = [vp, vp, vp]
    L.pmace_set_reference.restype = ctypes.c_int
    L.pmace_nrmse.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.pmace_nrmse.restype = ctypes.c_int
    L.pmace_set_stream.argtypes = [vp, vp]
    L.pmace_set_stream.restype = ctypes.c_int
    L.pmace_data_fit.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.pmace_data_fit.restype = ctypes.c_int
    L.pmace_batch_poll_fit.argtypes = [vp, vp, vp, vp, vp]
    L.pmace_batch_poll_fit.restype = ctypes.c_int
    L.pmace_batch_footprint.argtypes = [ctypes.POINTER(vp), i32]
    L.pmace_batch_footprint.restype = sz
    L.pmace_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(pmace_stop_rule), vp, sz,
                                     ctypes.POINTER(vp)]
    L.pmace_batch_create.restype = ctypes.c_int
    L.pmace_batch_step.argtypes = [vp, i32]
    L.pmace_batch_step.restype = ctypes.c_int
    L.pmace_batch_poll.argtypes = [vp, vp, vp, vp]
    L.pmace_batch_poll.restype = ctypes.c_int
    L.pmace_batch_destroy.argtypes = [vp]
    L.pmace_batch_destroy.restype = None
    L.pmace_simulate_footprint.argtypes = [i32, i32]
    L.pmace_simulate_footprint.restype = sz
    L.pmace_simulate.argtypes = [i32, i32, i32, i32, vp, vp, vp, ctypes.c_double, ctypes.c_uint64, vp,
                                 vp, sz, ctypes.POINTER(ctypes.c_double), vp]
    L.pmace_simulate.restype = ctypes.c_int
    L.pmace_simulate_static_max_bytes.argtypes = []
    L.pmace_simulate_static_max_bytes.restype = sz
    L.pmace_simulate_static.argtypes = [i32, i32, i32, i32, vp, vp, vp, ctypes.c_double, ctypes.c_uint64,
                                        vp, ctypes.POINTER(ctypes.c_double), vp]
    L.pmace_simulate_static.restype = ctypes.c_int
    L.pmace_agent_kind.argtypes = [vp]
    L.pmace_agent_kind.restype = i32
    L.pmace_philox4x32_10.argtypes = [vp, i32, vp]
    L.pmace_philox4x32_10.restype = ctypes.c_int
    L.pmace_poisson.argtypes = [vp, vp, i32, ctypes.c_uint64, vp]
    L.pmace_poisson.restype = ctypes.c_int
    _lib = L
    return L


def _status_str(s: int) -> str:
    try:
        return load_library().pmace_status_str(s).decode()
    except Exception:
        return "?"


def _check(status: int, where: str):
    if status != PMACE_OK:
        raise PMACEError(status, where)


def make_params(n1, n2, np_, num_pos, alpha, kappa=1.25, rho=0.5, flags=0, chunk=0,
                method=PMACE_METHOD_PMACE, beta=0.0, ppw=0) -> pmace_params:
    return pmace_params(int(n1), int(n2), int(np_), int(num_pos), float(alpha), float(kappa),
                        float(rho), int(flags), int(chunk), int(method), float(beta), int(ppw))


# Thin wrappers with the C names -------------------------------------------

def pmace_footprint(params: pmace_params) -> int:
    return int(load_library().pmace_footprint(ctypes.byref(params)))


def pmace_init(params, probe_ptr, pos_ptr, intensity_ptr, x0_ptr, ws_ptr, ws_bytes, stream_ptr):
    ctx = ctypes.c_void_p()
    st = load_library().pmace_init(ctypes.byref(params), probe_ptr, pos_ptr, intensity_ptr,
                                   x0_ptr, ws_ptr, ws_bytes, stream_ptr, ctypes.byref(ctx))
    return st, ctx


def pmace_iterate(ctx, n_iter: int) -> int:
    return load_library().pmace_iterate(ctx, int(n_iter))


def pmace_reconstruct(ctx, xhat_ptr) -> int:
    return load_library().pmace_reconstruct(ctx, xhat_ptr)


def pmace_get_state(ctx, v_ptr) -> int:
    return load_library().pmace_get_state(ctx, v_ptr)


def pmace_set_state(ctx, v_ptr) -> int:
    return load_library().pmace_set_state(ctx, v_ptr)


def pmace_sync(ctx) -> int:
    return load_library().pmace_sync(ctx)


def pmace_destroy(ctx) -> None:
    load_library().pmace_destroy(ctx)


def pmace_status_str(s: int) -> str:
    return _status_str(s)


def pmace_fft2(np_, count, in_ptr, out_ptr, inverse, stream_ptr) -> int:
    return load_library().pmace_fft2(int(np_), int(count), in_ptr, out_ptr, int(inverse), stream_ptr)


def pmace_set_reference(ctx, xref_ptr, mask_ptr) -> int:
    return load_library().pmace_set_reference(ctx, xref_ptr, mask_ptr)


def pmace_nrmse(ctx):
    out = ctypes.c_double()
    st = load_library().pmace_nrmse(ctx, ctypes.byref(out))
    return st, out.value


def pmace_set_stream(ctx, stream_ptr):
    return load_library().pmace_set_stream(ctx, stream_ptr)


def pmace_data_fit(ctx):
    out = ctypes.c_double()
    st = load_library().pmace_data_fit(ctx, ctypes.byref(out))
    return st, out.value


def _ctx_array(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), arr


def pmace_batch_footprint(ctxs) -> int:
    p, _keep = _ctx_array(ctxs)
    return int(load_library().pmace_batch_footprint(p, len(ctxs)))


def pmace_batch_create(ctxs, rule: pmace_stop_rule, ws_ptr, ws_bytes):
    p, _keep = _ctx_array(ctxs)
    out = ctypes.c_void_p()
    st = load_library().pmace_batch_create(p, len(ctxs), ctypes.byref(rule), ws_ptr, ws_bytes,
                                           ctypes.byref(out))
    return st, out


def pmace_batch_step(batch, n_iter: int) -> int:
    return load_library().pmace_batch_step(batch, int(n_iter))


def pmace_batch_poll(batch, n: int):
    done = (ctypes.c_int32 * n)()
    nr = (ctypes.c_double * n)()
    it = (ctypes.c_int32 * n)()
    st = load_library().pmace_batch_poll(batch, ctypes.cast(done, ctypes.c_void_p),
                                         ctypes.cast(nr, ctypes.c_void_p), ctypes.cast(it, ctypes.c_void_p))
    return st, np.array(done[:], dtype=np.int32), np.array(nr[:]), np.array(it[:], dtype=np.int32)


def pmace_batch_poll_fit(batch, n: int):
    done = (ctypes.c_int32 * n)()
    nr = (ctypes.c_double * n)()
    it = (ctypes.c_int32 * n)()
    fit = (ctypes.c_double * n)()
    st = load_library().pmace_batch_poll_fit(batch, ctypes.cast(done, ctypes.c_void_p),
                                             ctypes.cast(nr, ctypes.c_void_p),
                                             ctypes.cast(it, ctypes.c_void_p),
                                             ctypes.cast(fit, ctypes.c_void_p))
    return (st, np.array(done[:], dtype=np.int32), np.array(nr[:]), np.array(it[:], dtype=np.int32),
            np.array(fit[:]))


def pmace_batch_destroy(batch) -> None:
    load_library().pmace_batch_destroy(batch)


# Torch-facing helpers ------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def to_device_c64(a, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.complex64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex64))).to(device)


def fft2(x, inverse: bool = False, stream=None):
    """Orthonormal 2-D DFT (or its inverse) of a (count, np, np) complex64 CUDA tensor."""
    torch = _torch()
    x = x.contiguous()
    out = torch.empty_like(x)
    _check(pmace_fft2(x.shape[-1], x.numel() // (x.shape[-1] ** 2), ctypes.c_void_p(x.data_ptr()),
                      ctypes.c_void_p(out.data_ptr()), 1 if inverse else 0, _stream_ptr(stream)),
           "pmace_fft2")
    return out


def simulate(x, probe, pos, peak, seed: int, device="cuda", stream=None, out=None, workspace=None):
    """Intensities |F D P_j x|^2 (eq. (1)) on the device, Poisson at peak rate
    `peak` with the global-max scaling of eq. (16) when peak > 0.
    Returns (z float32 CUDA tensor (J, Np, Np), scale = peak / max I).
    `out` (float32, (J, Np, Np), contiguous) and `workspace` (uint8, at least
    pmace_simulate_footprint bytes) are used instead of new allocations."""
    torch = _torch()
    dev = torch.device(device)
    x_t = to_device_c64(x, dev)
    d_t = to_device_c64(probe, dev)
    pos_t = (pos if isinstance(pos, torch.Tensor) and pos.dtype == torch.int32
             else torch.as_tensor(np.asarray(pos, dtype=np.int32))).to(dev).contiguous()
    n1, n2 = x_t.shape
    np_ = d_t.shape[-1]
    J = pos_t.shape[0]
    fp = int(load_library().pmace_simulate_footprint(np_, J))
    if out is None:
        z = torch.empty((J, np_, np_), dtype=torch.float32, device=dev)
    else:
        if (out.dtype != torch.float32 or tuple(out.shape) != (J, np_, np_) or not out.is_contiguous()
                or out.device != x_t.device):
            raise ValueError(f"out must be a contiguous float32 ({J},{np_},{np_}) tensor on {x_t.device}")
        z = out
    if workspace is None:
        ws = torch.empty(fp, dtype=torch.uint8, device=dev)
    else:
        if workspace.dtype != torch.uint8 or workspace.numel() < fp or workspace.device != x_t.device:
            raise ValueError(f"workspace must be a uint8 tensor of at least {fp} bytes on {x_t.device}")
        ws = workspace
    scale = ctypes.c_double()
    _check(load_library().pmace_simulate(n1, n2, np_, J, ctypes.c_void_p(d_t.data_ptr()),
                                         ctypes.c_void_p(pos_t.data_ptr()),
                                         ctypes.c_void_p(x_t.data_ptr()), float(peak or 0.0),
                                         int(seed), ctypes.c_void_p(z.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(scale),
                                         _stream_ptr(stream)), "pmace_simulate")
    return z, scale.value


def simulate_static(x, probe, pos, peak, seed: int, device="cuda", stream=None, out=None):
    """As simulate(), through the allocation-free entry point: the library
    uses its per-device static scratch instead of a workspace (Np > 128 then
    needs J*Np*Np*8 <= simulate_static_max_bytes()).  Returns (z, scale)."""
    torch = _torch()
    dev = torch.device(device)
    x_t = to_device_c64(x, dev)
    d_t = to_device_c64(probe, dev)
    pos_t = (pos if isinstance(pos, torch.Tensor) and pos.dtype == torch.int32
             else torch.as_tensor(np.asarray(pos, dtype=np.int32))).to(dev).contiguous()
    n1, n2 = x_t.shape
    np_ = d_t.shape[-1]
    J = pos_t.shape[0]
    if out is None:
        z = torch.empty((J, np_, np_), dtype=torch.float32, device=dev)
    else:
        if (out.dtype != torch.float32 or tuple(out.shape) != (J, np_, np_) or not out.is_contiguous()
                or out.device != x_t.device):
            raise ValueError(f"out must be a contiguous float32 ({J},{np_},{np_}) tensor on {x_t.device}")
        z = out
    scale = ctypes.c_double()
    _check(load_library().pmace_simulate_static(n1, n2, np_, J, ctypes.c_void_p(d_t.data_ptr()),
                                                ctypes.c_void_p(pos_t.data_ptr()),
                                                ctypes.c_void_p(x_t.data_ptr()), float(peak or 0.0),
                                                int(seed), ctypes.c_void_p(z.data_ptr()),
                                                ctypes.byref(scale), _stream_ptr(stream)),
           "pmace_simulate_static")
    return z, scale.value


def simulate_static_max_bytes() -> int:
    """Largest Np > 128 frame buffer (J*Np*Np*8 bytes) simulate_static accepts."""
    return int(load_library().pmace_simulate_static_max_bytes())


def simulated_problem(n, np_, scan, step, peak, seed, device="cuda"):
    """A synth problem (object, probe, positions from the seeded generator)
    whose intensities are simulated on the device; z stays a CUDA tensor and
    the probe carries the photon scaling."""
    from . import synth
    rng = np.random.default_rng(seed)
    x = synth.make_object(n, n, rng)
    d = synth.make_probe(np_)
    pos = synth.make_positions(n, np_, scan, step, rng)
    z, scale = simulate(x, d, pos, peak, seed, device=device)
    return synth.Problem(x_true=x, probe=d * np.sqrt(scale), pos=pos, z=z, peak_photons=peak,
                         name=f"sim{seed}")


def philox4x32_10(records):
    """Philox4x32-10 on the device for (n, 6) uint32 records (counter[4], key[2])."""
    torch = _torch()
    r = np.ascontiguousarray(np.asarray(records, dtype=np.uint32))
    t = torch.from_numpy(r.view(np.int32)).cuda()
    _check(load_library().pmace_philox4x32_10(ctypes.c_void_p(t.data_ptr()), r.shape[0],
                                              _stream_ptr()), "pmace_philox4x32_10")
    return t.cpu().numpy().view(np.uint32)[:, :4]


def poisson(lam, seed: int):
    """The device Poisson sampler on given means (element i uses stream i)."""
    torch = _torch()
    lam_t = torch.as_tensor(np.asarray(lam, dtype=np.float64)).cuda().contiguous()
    out = torch.empty(lam_t.numel(), dtype=torch.float32, device="cuda")
    _check(load_library().pmace_poisson(ctypes.c_void_p(lam_t.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), lam_t.numel(), int(seed),
                                        _stream_ptr()), "pmace_poisson")
    return out.cpu().numpy()


class Reconstruction:
    """One PMACE reconstruction whose state stays resident on the GPU.

    probe (Np,Np) complex, pos (J,2) int (row, col), z (J,Np,Np) float
    intensities (numpy or torch); x0 (N1,N2) complex or None for ones."""

    def __init__(self, n1, n2, probe, pos, z, alpha, kappa=1.25, rho=0.5, x0=None,
                 flags=0, chunk=0, device="cuda", stream=None, workspace=None,
                 method=PMACE_METHOD_PMACE, beta=0.0, ppw=0):
        torch = _torch()
        self.device = torch.device(device)
        self.stream = stream
        probe_t = to_device_c64(probe, self.device)
        pos_t = torch.as_tensor(np.asarray(pos, dtype=np.int32) if not isinstance(pos, torch.Tensor) else pos,
                                dtype=torch.int32).to(self.device).contiguous()
        z_t = (z if isinstance(z, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(z, dtype=np.float32)))
        z_t = z_t.to(device=self.device, dtype=torch.float32).contiguous()
        np_ = probe_t.shape[-1]
        J = pos_t.shape[0]
        if z_t.shape != (J, np_, np_):
            raise ValueError(f"intensities must be ({J},{np_},{np_}), got {tuple(z_t.shape)}")
        x0_t = None if x0 is None else to_device_c64(x0, self.device)
        self.params = make_params(n1, n2, np_, J, alpha, kappa, rho, flags, chunk, method, beta, ppw)
        fp = pmace_footprint(self.params)
        if fp == 0:
            raise PMACEError(PMACE_EINVAL, "pmace_footprint")
        self.footprint = fp
        if workspace is None:
            workspace = torch.empty(fp, dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        st, ctx = pmace_init(self.params, ctypes.c_void_p(probe_t.data_ptr()),
                             ctypes.c_void_p(pos_t.data_ptr()), ctypes.c_void_p(z_t.data_ptr()),
                             ctypes.c_void_p(0 if x0_t is None else x0_t.data_ptr()),
                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                             _stream_ptr(stream))
        _check(st, "pmace_init")
        self.ctx = ctx
        self.n1, self.n2, self.np, self.J = int(n1), int(n2), int(np_), int(J)

    def iterate(self, n: int = 1):
        _check(pmace_iterate(self.ctx, n), "pmace_iterate")

    @property
    def agent(self) -> str:
        """'whole patch', 'three-pass', 'split' (coset blocks) or 'row-spectrum'
        (states kept as row DFTs): the agent this reconstruction runs."""
        k = load_library().pmace_agent_kind(self.ctx)
        return {0: "whole patch", 1: "three-pass", 2: "split", 3: "row-spectrum"}[k]

    def reconstruct(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n1, self.n2), dtype=torch.complex64, device=self.device)
        _check(pmace_reconstruct(self.ctx, ctypes.c_void_p(out.data_ptr())), "pmace_reconstruct")
        return out

    def get_state(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.J, self.np, self.np), dtype=torch.complex64, device=self.device)
        _check(pmace_get_state(self.ctx, ctypes.c_void_p(out.data_ptr())), "pmace_get_state")
        return out

    def set_state(self, v):
        v_t = to_device_c64(v, self.device)
        _check(pmace_set_state(self.ctx, ctypes.c_void_p(v_t.data_ptr())), "pmace_set_state")
        self.sync()          # keep v_t alive until the copy has run

    def sync(self):
        _check(pmace_sync(self.ctx), "pmace_sync")

    def set_stream(self, stream):
        """Queue later work on `stream` (a torch stream or None for the null stream)."""
        _check(pmace_set_stream(self.ctx, _stream_ptr(stream)), "pmace_set_stream")
        self.stream = stream

    def set_reference(self, xref, mask=None):
        """NRMSE reference object (and optional boolean region); kept alive here."""
        torch = _torch()
        if xref is None:
            self._ref = None
            _check(pmace_set_reference(self.ctx, ctypes.c_void_p(0), ctypes.c_void_p(0)),
                   "pmace_set_reference")
            return
        xr = to_device_c64(xref, self.device)
        mk = None
        if mask is not None:
            m = mask if isinstance(mask, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(mask))
            mk = m.to(device=self.device, dtype=torch.uint8).contiguous()
        self._ref = (xr, mk)
        _check(pmace_set_reference(self.ctx, ctypes.c_void_p(xr.data_ptr()),
                                   ctypes.c_void_p(0 if mk is None else mk.data_ptr())),
               "pmace_set_reference")

    def nrmse(self) -> float:
        st, v = pmace_nrmse(self.ctx)
        _check(st, "pmace_nrmse")
        return v

    def data_fit(self) -> float:
        """Data-fit cost of eq. (4) at the current reconstruction (sigma_n = 1)."""
        st, v = pmace_data_fit(self.ctx)
        _check(st, "pmace_data_fit")
        return v

    def close(self):
        """Release the context.  A batch that holds this reconstruction must be
        closed first (it launches from the context's tables)."""
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            live = [b for b in getattr(self, "_batches", ()) if b.batch is not None]
            if live:
                raise RuntimeError("close the Batch holding this Reconstruction first")
            pmace_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several Reconstructions (same device and stream) advanced together: one
    graph launch per iteration, NRMSE and the stop rule kept on the device."""

    def __init__(self, recons, tol=1e-4, min_iter=2, max_iter=500, workspace=None,
                 criterion=PMACE_STOP_NRMSE, check_every=1):
        torch = _torch()
        self.recons = list(recons)
        self.ctxs = [r.ctx for r in self.recons]
        fp = pmace_batch_footprint(self.ctxs)
        if fp == 0:
            raise PMACEError(PMACE_EINVAL, "pmace_batch_footprint")
        if workspace is None:
            workspace = torch.empty(fp, dtype=torch.uint8, device=self.recons[0].device)
        self.workspace = workspace
        self.rule = pmace_stop_rule(float(tol), int(min_iter), int(max_iter), int(criterion),
                                    int(check_every))
        st, b = pmace_batch_create(self.ctxs, self.rule, ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel())
        _check(st, "pmace_batch_create")
        self.batch = b
        import weakref
        for r in self.recons:
            if not hasattr(r, "_batches"):
                r._batches = weakref.WeakSet()
            r._batches.add(self)

    def step(self, n: int = 1):
        _check(pmace_batch_step(self.batch, n), "pmace_batch_step")

    def poll(self):
        """(done flags, last NRMSE, counted iterations) per member, numpy arrays."""
        st, done, nr, it = pmace_batch_poll(self.batch, len(self.ctxs))
        _check(st, "pmace_batch_poll")
        return done, nr, it

    def poll_fit(self):
        """poll() plus the last data-fit cost the stop rule evaluated."""
        st, done, nr, it, fit = pmace_batch_poll_fit(self.batch, len(self.ctxs))
        _check(st, "pmace_batch_poll_fit")
        return done, nr, it, fit

    def close(self):
        if getattr(self, "batch", None) is not None and self.batch.value:
            pmace_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
