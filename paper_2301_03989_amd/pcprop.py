"""Python binding of libpcprop (include/pcprop.h): argument marshalling only.

Every step of the propagation runs in the HIP kernels of ``csrc/``; PyTorch only
provides device memory (tensors) and the stream.  There is no CPU fallback: if the
library is not built, or no GPU is present, calls raise.

Method: Masat, Colombo, Boutonnet, arXiv 2301.03989 (batched Picard-Chebyshev
propagation of many initial conditions; Sec. 2.2 iteration, Sec. 3 augmentation).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcprop.so")

PC_OK, PC_EINVAL, PC_ENOTCONV, PC_ENONFINITE, PC_EHIP, PC_ENOMEM = 0, 1, 2, 3, 4, 5
PC_ITER_NOTCONV, PC_ITER_NONFINITE = -1, -2
INIT = {"kepler": 0, "cold": 1, "guess": 2}
TOL_MODE = {"rel": 0, "abs": 1}
PATH = {"fused": 0, "plain": 1}
PRECISION = {"fp64": 0, "fp32-fp64": 1}
CONV = {"ic": 0, "group": 1}

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class PcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pcprop error {code}: {msg}")
        self.code = code


class _Model(ctypes.Structure):
    _fields_ = [("mu_sun", ctypes.c_double), ("n_pert", ctypes.c_int32),
                ("pert", _dp), ("epoch", ctypes.c_double), ("inv_c2", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("init", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("path", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("tile_pairs", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("switch_tol", ctypes.c_double), ("max_fp32", ctypes.c_int32), ("job_list", ctypes.c_int32),
                ("conv", ctypes.c_int32), ("streams", ctypes.c_int32), ("order", ctypes.c_int32),
                ("feedback", ctypes.c_int32), ("guess", ctypes.c_void_p), ("refine", ctypes.c_int32),
                ("flyby_hill", ctypes.c_double)]


class _Group(ctypes.Structure):
    _fields_ = [("ic_offset", ctypes.c_int64), ("n_ic", ctypes.c_int64),
                ("t0", ctypes.c_double), ("tf", ctypes.c_double),
                ("nodes", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("tol", ctypes.c_double)]


_lib = None

EXPORTS = ("pc_default_opts", "pc_ctx_create", "pc_ctx_destroy", "pc_workspace_bytes",
           "pc_propagate", "pc_propagate_batched", "pc_get_operator", "pc_apply_operator",
           "pc_eval_force", "pc_eval_kepler", "pc_set_timing", "pc_last_kernel_ms", "pc_autotune",
           "pc_set_tile_pairs", "pc_get_tile_pairs", "pc_adjoint", "pc_strerror", "pc_last_error",
           "pc_version", "pc_graph_captures", "pc_measure_ceilings",
           "pc_set_job_list", "pc_get_job_list", "pc_propagate_batched_noalloc", "pc_flyby_ratio")


def load_library(path: str = LIB_PATH):
    """Load libpcprop.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run `python -m paper_2301_03989_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.pc_default_opts.argtypes = [P(_Opts)]
    lib.pc_default_opts.restype = None
    lib.pc_ctx_create.argtypes = [ctypes.c_int, P(_vp)]
    lib.pc_ctx_destroy.argtypes = [_vp]
    lib.pc_ctx_destroy.restype = None
    lib.pc_workspace_bytes.argtypes = [_vp, P(_Group), ctypes.c_int32, P(_Model), P(_Opts),
                                       P(ctypes.c_size_t)]
    lib.pc_propagate.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_double, P(_Model), P(_Opts),
                                 _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pc_propagate_batched.argtypes = [_vp, _vp, ctypes.c_int64, P(_Group), ctypes.c_int32,
                                         P(_Model), P(_Opts), _vp, _vp, ctypes.c_int32, _vp, _vp,
                                         ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    lib.pc_propagate_batched_noalloc.argtypes = [_vp, _vp, ctypes.c_int64, P(_Group), ctypes.c_int32,
                                                 P(_Model), P(_Opts), _vp, _vp, ctypes.c_int32, _vp, _vp,
                                                 ctypes.c_int32, _vp]
    lib.pc_flyby_ratio.argtypes = [_vp, _vp, ctypes.c_int64, P(_Group), ctypes.c_int32, P(_Model), ctypes.c_int32,
                                   _vp, _vp, ctypes.c_size_t, _vp]
    lib.pc_get_operator.argtypes = [_vp, ctypes.c_int32, _dp]
    lib.pc_apply_operator.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, _vp, _vp, ctypes.c_double,
                                      _vp, _vp]
    lib.pc_eval_force.argtypes = [_vp, _vp, _vp, ctypes.c_int64, P(_Model), _vp, _vp]
    lib.pc_eval_kepler.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
    lib.pc_autotune.argtypes = [_vp, _vp, ctypes.c_int64, P(_Group), ctypes.c_int32, P(_Model), _vp, _vp,
                                ctypes.c_size_t, _vp, P(ctypes.c_int32)]
    lib.pc_set_tile_pairs.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
    lib.pc_adjoint.argtypes = [_vp, ctypes.c_int64, P(_Group), ctypes.c_int32, P(_Model), P(_Opts), _vp,
                               ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                               _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pc_get_tile_pairs.argtypes = [_vp, ctypes.c_int32, P(ctypes.c_int32)]
    lib.pc_set_job_list.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
    lib.pc_get_job_list.argtypes = [_vp, ctypes.c_int32, P(ctypes.c_int32)]
    lib.pc_graph_captures.argtypes = [_vp, P(ctypes.c_int64)]
    lib.pc_measure_ceilings.argtypes = [_vp, _vp, ctypes.c_size_t, _vp, _dp]
    lib.pc_set_timing.argtypes = [_vp, ctypes.c_int]
    lib.pc_last_kernel_ms.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
    lib.pc_strerror.argtypes = [ctypes.c_int]
    lib.pc_strerror.restype = ctypes.c_char_p
    lib.pc_last_error.argtypes = [_vp]
    lib.pc_last_error.restype = ctypes.c_char_p
    lib.pc_version.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass
class Model:
    """Point-mass force model: central body mu_sun plus perturbers on Keplerian orbits.
    ``pert``: [P, 7] rows (mu_p, a, e, inc, raan, argp, M0), radians, M0 at ``epoch``.
    ``inv_c2`` > 0: the Einstein-Infeld-Hoffmann dynamics with 1/c^2 = inv_c2."""
    mu_sun: float = 1.0
    pert: np.ndarray | None = None
    epoch: float = 0.0
    inv_c2: float = 0.0

    def _c(self):
        pert = np.zeros((0, 7)) if self.pert is None else np.ascontiguousarray(self.pert, dtype=np.float64).reshape(-1, 7)
        self._keep = pert
        m = _Model()
        m.mu_sun = float(self.mu_sun)
        m.n_pert = int(pert.shape[0])
        m.pert = pert.ctypes.data_as(_dp) if pert.size else ctypes.cast(None, _dp)
        m.epoch = float(self.epoch)
        m.inv_c2 = float(self.inv_c2)
        return m


@dataclass
class Group:
    ic_offset: int
    n_ic: int
    t0: float
    tf: float
    nodes: int
    segments: int
    tol: float


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t, name, shape=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """Owns a pc_ctx on one device (cached operators K_N) and a reusable workspace."""

    def __init__(self, device=None):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("pcprop needs a HIP GPU; none is available")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = ctypes.c_void_p()
        rc = self.lib.pc_ctx_create(self.device.index, ctypes.byref(h))
        if rc != PC_OK:
            raise PcError(rc, self.lib.pc_strerror(rc).decode())
        self.handle = h
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.pc_ctx_destroy(h)
            self.handle = None

    def _raise(self, rc):
        raise PcError(rc, f"{self.lib.pc_strerror(rc).decode()}: {self.lib.pc_last_error(self.handle).decode()}")

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=self.device)
        return self._ws

    @staticmethod
    def opts(init="kepler", max_iter=64, tol_mode="rel", path="fused", fixed_iters=0,
             tile_pairs=0, precision="fp64", graph=False, switch_tol=0.0, max_fp32=0, job_list=0, conv="ic",
             streams=1, order=1, feedback=0, guess=None, refine=0, flyby_hill=0.0):
        o = _Opts()
        o.init, o.max_iter, o.tol_mode = INIT[init], int(max_iter), TOL_MODE[tol_mode]
        o.precision, o.path, o.fixed_iters = PRECISION[precision], PATH[path], int(fixed_iters)
        o.tile_pairs, o.graph = int(tile_pairs), int(bool(graph))
        o.switch_tol, o.max_fp32, o.job_list = float(switch_tol), int(max_fp32), int(job_list)
        o.conv = CONV[conv]
        o.streams = int(streams)
        o.order, o.feedback = int(order), int(feedback)
        o.refine = int(refine)
        o.flyby_hill = float(flyby_hill)
        if guess is not None:   # init "guess": device node states [n, S_max, N_max, 6]
            _check_tensor(guess, "guess")
            o.guess = guess.data_ptr()
        return o

    def workspace_bytes(self, groups, model, **opts):
        garr = (_Group * len(groups))(*[_Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)
                                       for g in groups])
        mc, oc = model._c(), self.opts(**opts)
        nb = ctypes.c_size_t()
        rc = self.lib.pc_workspace_bytes(self.handle, garr, len(groups), ctypes.byref(mc), ctypes.byref(oc),
                                         ctypes.byref(nb))
        if rc != PC_OK:
            self._raise(rc)
        return nb.value

    def _outputs(self, ics, groups, want_bounds, want_nodes, out, iters_out=None, bounds_out=None,
                 nodes_out=None):
        """Output tensors of a call: the caller's (out, iters_out, bounds_out, nodes_out; kept
        across calls, e.g. for graph replay, whose signature includes the output pointers) or
        new ones."""
        _check_tensor(ics, "ics")
        if ics.dim() != 2 or ics.shape[1] != 6:
            raise ValueError("ics must be [n, 6]")
        n = ics.shape[0]
        S_max = max(g.segments for g in groups)
        N_max = max(g.nodes for g in groups)
        dev = ics.device
        if out is not None:
            _check_tensor(out, "out", (n, 6))
        if iters_out is not None:
            _check_tensor(iters_out, "iters_out", (n, S_max), torch.int32)
        if bounds_out is not None:
            _check_tensor(bounds_out, "bounds_out", (n, S_max + 1, 6))
        if nodes_out is not None:
            _check_tensor(nodes_out, "nodes_out", (n, S_max, N_max, 6))
        states = out if out is not None else torch.empty((n, 6), dtype=torch.float64, device=dev)
        # a caller's iters_out keeps its contents in the columns past a group's segments
        iters = iters_out if iters_out is not None else torch.zeros((n, S_max), dtype=torch.int32, device=dev)
        bounds = bounds_out if bounds_out is not None else (
            torch.empty((n, S_max + 1, 6), dtype=torch.float64, device=dev) if want_bounds else None)
        nodes = nodes_out if nodes_out is not None else (
            torch.empty((n, S_max, N_max, 6), dtype=torch.float64, device=dev) if want_nodes else None)
        garr = (_Group * len(groups))(*[_Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)
                                       for g in groups])
        return n, S_max, N_max, states, iters, bounds, nodes, garr

    @staticmethod
    def _result(rc, states, iters, bounds, nodes):
        res = {"states": states, "iters": iters, "status": rc}
        if bounds is not None:
            res["bounds"] = bounds
        if nodes is not None:
            res["nodes"] = nodes
        return res

    def propagate_batched(self, ics, groups, model=None, *, want_bounds=False, want_nodes=False,
                          raise_on_status=False, out=None, iters_out=None, bounds_out=None, nodes_out=None,
                          **opts):
        """Two-level augmented propagation (Sec. 3.2).  Returns a dict with
        ``states`` [n,6], ``iters`` [n,S_max] (int32), ``status`` and, when asked,
        ``bounds`` [n,S_max+1,6] and ``nodes`` [n,S_max,N_max,6].  ``out``,
        ``iters_out``, ``bounds_out`` and ``nodes_out`` give the output tensors."""
        model = model or Model()
        want_bounds = want_bounds or bool(opts.get("refine", 0))   # refinement rewrites the boundary records
        n, S_max, N_max, states, iters, bounds, nodes, garr = self._outputs(
            ics, groups, want_bounds, want_nodes, out, iters_out, bounds_out, nodes_out)
        mc, oc = model._c(), self.opts(**opts)
        nb = ctypes.c_size_t()
        rc = self.lib.pc_workspace_bytes(self.handle, garr, len(groups), ctypes.byref(mc), ctypes.byref(oc),
                                         ctypes.byref(nb))
        if rc != PC_OK:
            self._raise(rc)
        ws = self.workspace(nb.value)
        rc = self.lib.pc_propagate_batched(
            self.handle, ctypes.c_void_p(ics.data_ptr()), n, garr, len(groups), ctypes.byref(mc),
            ctypes.byref(oc), ctypes.c_void_p(states.data_ptr()), ctypes.c_void_p(iters.data_ptr()), S_max,
            ctypes.c_void_p(bounds.data_ptr() if bounds is not None else 0),
            ctypes.c_void_p(nodes.data_ptr() if nodes is not None else 0), N_max,
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(ics.device))
        if rc not in (PC_OK, PC_ENOTCONV, PC_ENONFINITE) or (raise_on_status and rc != PC_OK):
            self._raise(rc)
        return self._result(rc, states, iters, bounds, nodes)

    def propagate_batched_noalloc(self, ics, groups, model=None, *, out, iters_out, bounds_out=None,
                                  nodes_out=None, raise_on_status=False, **opts):
        """pc_propagate_batched_noalloc: the fused path with the library's static device
        scratch as its workspace, for callers that cannot allocate.  Every output tensor is
        the caller's (``out`` [n,6], ``iters_out`` [n,S_max] int32, optional ``bounds_out``,
        ``nodes_out``); the call allocates nothing.  Same result dict as propagate_batched."""
        model = model or Model()
        n, S_max, N_max, states, iters, bounds, nodes, garr = self._outputs(
            ics, groups, bounds_out is not None, nodes_out is not None, out, iters_out, bounds_out, nodes_out)
        mc, oc = model._c(), self.opts(**opts)
        rc = self.lib.pc_propagate_batched_noalloc(
            self.handle, ctypes.c_void_p(ics.data_ptr()), n, garr, len(groups), ctypes.byref(mc),
            ctypes.byref(oc), ctypes.c_void_p(states.data_ptr()), ctypes.c_void_p(iters.data_ptr()), S_max,
            ctypes.c_void_p(bounds.data_ptr() if bounds is not None else 0),
            ctypes.c_void_p(nodes.data_ptr() if nodes is not None else 0), N_max, _stream_ptr(ics.device))
        if rc not in (PC_OK, PC_ENOTCONV, PC_ENONFINITE) or (raise_on_status and rc != PC_OK):
            self._raise(rc)
        return self._result(rc, states, iters, bounds, nodes)

    def flyby_ratio(self, ics, groups, model, samples=16):
        """pc_flyby_ratio: per IC, the smallest distance of its two-body prediction to any
        perturber in Hill radii ([n] float64 tensor; +inf outside the groups)."""
        _check_tensor(ics, "ics")
        garr = (_Group * len(groups))(*[_Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)
                                       for g in groups])
        mc = model._c()
        ratio = torch.full((ics.shape[0],), float("inf"), dtype=torch.float64, device=ics.device)
        nb = ctypes.c_size_t()
        oc = self.opts()
        rc = self.lib.pc_workspace_bytes(self.handle, garr, len(groups), ctypes.byref(mc), ctypes.byref(oc),
                                         ctypes.byref(nb))
        if rc != PC_OK:
            self._raise(rc)
        ws = self.workspace(nb.value)
        rc = self.lib.pc_flyby_ratio(self.handle, ctypes.c_void_p(ics.data_ptr()), ics.shape[0], garr, len(groups),
                                     ctypes.byref(mc), int(samples), ctypes.c_void_p(ratio.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(ics.device))
        if rc != PC_OK:
            self._raise(rc)
        return ratio

    def propagate(self, ics, t0, tf, nodes, segments, tol, model=None, **kw):
        g = Group(0, int(ics.shape[0]), float(t0), float(tf), int(nodes), int(segments), float(tol))
        r = self.propagate_batched(ics, [g], model, **kw)
        return r["states"], r["iters"], r["status"]

    def set_timing(self, enable=True):
        rc = self.lib.pc_set_timing(self.handle, int(bool(enable)))
        if rc != PC_OK:
            self._raise(rc)

    def measure_ceilings(self, mib=1024):
        """On-chip ceilings: (FP64 matrix-core TFLOP/s, FP64 vector FMA TFLOP/s, device copy
        GB/s read + written) from pc_measure_ceilings, with a scratch of ``mib`` MiB."""
        buf = torch.empty(int(mib) << 20, dtype=torch.uint8, device=self.device)
        out = np.zeros(3)
        rc = self.lib.pc_measure_ceilings(self.handle, ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                          _stream_ptr(self.device), out.ctypes.data_as(_dp))
        if rc != PC_OK:
            self._raise(rc)
        return float(out[0]), float(out[1]), float(out[2])

    def graph_captures(self):
        """HIP graphs captured so far by graph=True calls of this context."""
        v = ctypes.c_int64()
        rc = self.lib.pc_graph_captures(self.handle, ctypes.byref(v))
        if rc != PC_OK:
            self._raise(rc)
        return v.value

    def last_kernel_ms(self):
        ms = ctypes.c_double()
        rc = self.lib.pc_last_kernel_ms(self.handle, ctypes.byref(ms))
        if rc != PC_OK:
            self._raise(rc)
        return ms.value

    def autotune(self, ics, groups, model=None):
        """Tune the job shape and the per-node-count job lengths for this batch (pc_autotune);
        returns the chosen tile_pairs (the job lengths: ``job_list(padded_nodes)``)."""
        model = model or Model()
        _check_tensor(ics, "ics")
        garr = (_Group * len(groups))(*[_Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)
                                       for g in groups])
        mc, oc = model._c(), self.opts()
        nb = ctypes.c_size_t()
        rc = self.lib.pc_workspace_bytes(self.handle, garr, len(groups), ctypes.byref(mc), ctypes.byref(oc),
                                         ctypes.byref(nb))
        if rc != PC_OK:
            self._raise(rc)
        ws = self.workspace(nb.value)
        scratch = torch.empty((ics.shape[0], 6), dtype=torch.float64, device=ics.device)
        chosen = ctypes.c_int32()
        rc = self.lib.pc_autotune(self.handle, ctypes.c_void_p(ics.data_ptr()), ics.shape[0], garr, len(groups),
                                  ctypes.byref(mc), ctypes.c_void_p(scratch.data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(ics.device),
                                  ctypes.byref(chosen))
        if rc != PC_OK:
            self._raise(rc)
        return chosen.value

    def adjoint(self, ckpt, gbar_final, groups, model=None, gbar_nodes=None, adj_tol=1e-12,
                adj_max_iter=200, raise_on_status=False, fwd_nodes=None, **opts):
        """pc_adjoint: dL/dy0 [n, 6] from the forward call's segment-boundary states ``ckpt``
        [n, S+1, 6] and the seeds dL/d(final state) [n, 6] (and dL/d(node states)
        [n, S, N, 6]).  ``fwd_nodes``: the forward call's node states [n, S, N, 6]; given,
        the segments are read instead of re-solved.  Returns (grad, adjoint sweeps per
        segment [n, S], status)."""
        model = model or Model()
        _check_tensor(ckpt, "ckpt")
        _check_tensor(gbar_final, "gbar_final")
        n = ckpt.shape[0]
        S_max = max(g.segments for g in groups)
        N_max = max(g.nodes for g in groups)
        if ckpt.shape != (n, S_max + 1, 6) or gbar_final.shape != (n, 6):
            raise ValueError("ckpt must be [n, S+1, 6] and gbar_final [n, 6]")
        if gbar_nodes is not None:
            _check_tensor(gbar_nodes, "gbar_nodes", (n, S_max, N_max, 6))
        if fwd_nodes is not None:
            _check_tensor(fwd_nodes, "fwd_nodes", (n, S_max, N_max, 6))
        garr = (_Group * len(groups))(*[_Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)
                                       for g in groups])
        mc, oc = model._c(), self.opts(**opts)
        oc.tile_pairs = 2048
        nb = ctypes.c_size_t()
        rc = self.lib.pc_workspace_bytes(self.handle, garr, len(groups), ctypes.byref(mc), ctypes.byref(oc),
                                         ctypes.byref(nb))
        if rc != PC_OK:
            self._raise(rc)
        ws = self.workspace(nb.value)
        grad = torch.empty((n, 6), dtype=torch.float64, device=ckpt.device)
        adj_it = torch.zeros((n, S_max), dtype=torch.int32, device=ckpt.device)
        rc = self.lib.pc_adjoint(self.handle, n, garr, len(groups), ctypes.byref(mc), ctypes.byref(oc),
                                 ctypes.c_void_p(ckpt.data_ptr()), S_max, ctypes.c_void_p(gbar_final.data_ptr()),
                                 ctypes.c_void_p(gbar_nodes.data_ptr() if gbar_nodes is not None else 0),
                                 ctypes.c_void_p(fwd_nodes.data_ptr() if fwd_nodes is not None else 0), N_max,
                                 float(adj_tol), int(adj_max_iter), ctypes.c_void_p(grad.data_ptr()),
                                 ctypes.c_void_p(adj_it.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream_ptr(ckpt.device))
        if rc not in (PC_OK, PC_ENOTCONV, PC_ENONFINITE) or (raise_on_status and rc != PC_OK):
            self._raise(rc)
        return grad, adj_it, rc

    def tile_pairs(self, padded_nodes):
        v = ctypes.c_int32()
        rc = self.lib.pc_get_tile_pairs(self.handle, int(padded_nodes), ctypes.byref(v))
        if rc != PC_OK:
            self._raise(rc)
        return v.value

    def job_list(self, padded_nodes):
        v = ctypes.c_int32()
        rc = self.lib.pc_get_job_list(self.handle, int(padded_nodes), ctypes.byref(v))
        if rc != PC_OK:
            self._raise(rc)
        return v.value

    def set_job_list(self, padded_nodes, blocks):
        rc = self.lib.pc_set_job_list(self.handle, int(padded_nodes), int(blocks))
        if rc != PC_OK:
            self._raise(rc)

    def set_tile_pairs(self, padded_nodes, pairs):
        rc = self.lib.pc_set_tile_pairs(self.handle, int(padded_nodes), int(pairs))
        if rc != PC_OK:
            self._raise(rc)

    def get_operator(self, nodes):
        K = np.zeros((nodes, nodes))
        rc = self.lib.pc_get_operator(self.handle, int(nodes), K.ctypes.data_as(_dp))
        if rc != PC_OK:
            self._raise(rc)
        return K

    def apply_operator(self, F, y0, scale, nodes):
        _check_tensor(F, "F")
        _check_tensor(y0, "y0")
        if F.dim() != 2 or F.shape[0] != nodes or y0.shape != (F.shape[1],):
            raise ValueError("F must be [nodes, n_cols] and y0 [n_cols]")
        Y = torch.empty_like(F)
        rc = self.lib.pc_apply_operator(self.handle, int(nodes), int(F.shape[1]), ctypes.c_void_p(F.data_ptr()),
                                        ctypes.c_void_p(y0.data_ptr()), float(scale),
                                        ctypes.c_void_p(Y.data_ptr()), _stream_ptr(F.device))
        if rc != PC_OK:
            self._raise(rc)
        return Y

    def eval_force(self, r, t, model=None):
        model = model or Model()
        _check_tensor(r, "r")
        _check_tensor(t, "t")
        n = t.shape[0]
        if r.shape != (3, n):
            raise ValueError("r must be [3, n] and t [n]")
        a = torch.empty_like(r)
        mc = model._c()
        rc = self.lib.pc_eval_force(self.handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(t.data_ptr()), n,
                                    ctypes.byref(mc), ctypes.c_void_p(a.data_ptr()), _stream_ptr(r.device))
        if rc != PC_OK:
            self._raise(rc)
        return a

    def eval_kepler(self, y0, dt):
        _check_tensor(y0, "y0")
        _check_tensor(dt, "dt")
        n = dt.shape[0]
        if y0.shape != (6, n):
            raise ValueError("y0 must be [6, n] and dt [n]")
        y = torch.empty_like(y0)
        ok = torch.empty(n, dtype=torch.int32, device=y0.device)
        rc = self.lib.pc_eval_kepler(self.handle, ctypes.c_void_p(y0.data_ptr()), ctypes.c_void_p(dt.data_ptr()), n,
                                     ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ok.data_ptr()),
                                     _stream_ptr(y0.device))
        if rc != PC_OK:
            self._raise(rc)
        return y, ok


_default_ctx = {}


def context(device=None) -> Context:
    """Per-device default context."""
    key = torch.cuda.current_device() if device is None else device
    if key not in _default_ctx:
        _default_ctx[key] = Context(key)
    return _default_ctx[key]


def propagate(ics, t0, tf, nodes, segments, tol, model=None, **kw):
    """pc_propagate: returns (states [n,6], iters [n,segments], status)."""
    return context(ics.device.index).propagate(ics, t0, tf, nodes, segments, tol, model, **kw)


def propagate_batched(ics, groups, model=None, **kw):
    """pc_propagate_batched: see Context.propagate_batched."""
    return context(ics.device.index).propagate_batched(ics, groups, model, **kw)
