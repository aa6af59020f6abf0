"""Python binding of the C ABI: torch device tensors in, torch device tensors out.

Argument marshalling only -- every step of the evaluation runs in the HIP
kernels of libbeagle.so.  Calls are enqueued on torch's current stream of the
tensors' device.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib

_FIT_NAMES = {"mse": _lib.FIT_MSE, "corr": _lib.FIT_CORR, "point": _lib.FIT_POINT, "r4": _lib.FIT_R4}


def _kind(kind) -> int:
    """Fitness kind as the C enum value; unknown integers pass through so the
    library reports them."""
    if isinstance(kind, str):
        if kind not in _FIT_NAMES:
            raise ValueError(f"unknown fitness kind {kind!r}")
        return _FIT_NAMES[kind]
    return int(kind)


class BeagleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"beagle error {code}: {msg}")
        self.code = code


def _check(code: int):
    if code != _lib.OK:
        lib = _lib.load()
        raise BeagleError(code, lib.beagle_last_error().decode())


class Context:
    """A library context (device workspace) on one HIP device."""

    def __init__(self, device: int = 0, max_workspace_bytes: int = 0):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.beagle_ctx_create(ctypes.byref(h), device, max_workspace_bytes))
        self.handle = h

    def enable_timing(self, enable: bool = True):
        _check(self.lib.beagle_ctx_enable_timing(self.handle, 1 if enable else 0))

    def kernel_time(self):
        """(total ms, launches) of the main evaluation kernel since timing was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.beagle_ctx_kernel_time(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def set_tuning(self, policy: str = "auto"):
        """Tile-width policy: "auto" (measure once per shape bucket), "wide" or "narrow"."""
        names = {"auto": _lib.TUNE_AUTO, "wide": _lib.TUNE_WIDE, "narrow": _lib.TUNE_NARROW}
        code = names.get(policy, -1) if isinstance(policy, str) else int(policy)
        _check(self.lib.beagle_ctx_set_tuning(self.handle, code))

    def set_decoder(self, decoder: str = "wave"):
        """Decoder of the programs of at most 64 tokens: "wave" (one wave per
        program, the default) or "thread" (one thread per program)."""
        names = {"wave": _lib.DECODE_WAVE, "thread": _lib.DECODE_THREAD}
        code = names.get(decoder, -1) if isinstance(decoder, str) else int(decoder)
        _check(self.lib.beagle_ctx_set_decoder(self.handle, code))

    def tile_width(self, kind, D: int, M: int, n_tokens: int, n_programs: int) -> int:
        """Cases per lane beagle_eval uses for this shape (0: not measured yet)."""
        out = ctypes.c_int32()
        _check(self.lib.beagle_ctx_tile_width(self.handle, _kind(kind), D, M, n_tokens, n_programs,
                                              ctypes.byref(out)))
        return int(out.value)

    def graph_stats(self):
        """(graphs captured, graph launches) of batched evaluation."""
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        _check(self.lib.beagle_ctx_graph_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def close(self):
        if self.handle:
            self.lib.beagle_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def context(device: int = 0) -> Context:
    ctx = _contexts.get(device)
    if ctx is None:
        ctx = Context(device)
        _contexts[device] = ctx
    return ctx


@dataclasses.dataclass
class DevicePrograms:
    """A population in the library's packed layout, resident on a GPU.

    tokens are stored as int16 tensors holding the uint16 token bits.
    """

    tokens: torch.Tensor        # int16 [n_tokens]
    tok_offset: torch.Tensor    # int64 [N]
    tok_len: torch.Tensor       # int32 [N]
    consts: torch.Tensor        # float32 [n_consts]
    const_offset: torch.Tensor  # int64 [N]
    const_count: torch.Tensor   # int32 [N]

    @property
    def n(self) -> int:
        return int(self.tok_len.shape[0])

    @property
    def device(self) -> torch.device:
        return self.tok_len.device

    @staticmethod
    def from_arrays(tokens, tok_offset, tok_len, consts, const_offset, const_count, device="cuda") -> "DevicePrograms":
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(tokens, dtype=np.uint16)).view(np.int16))
        return DevicePrograms(
            t.to(device),
            torch.as_tensor(np.asarray(tok_offset, dtype=np.int64)).to(device),
            torch.as_tensor(np.asarray(tok_len, dtype=np.int32)).to(device),
            torch.as_tensor(np.asarray(consts, dtype=np.float32)).to(device),
            torch.as_tensor(np.asarray(const_offset, dtype=np.int64)).to(device),
            torch.as_tensor(np.asarray(const_count, dtype=np.int32)).to(device))

    @staticmethod
    def from_programset(ps, device="cuda") -> "DevicePrograms":
        return DevicePrograms.from_arrays(ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset,
                                          ps.const_count, device)

    @staticmethod
    def from_fixed(tokens: torch.Tensor, lens: torch.Tensor, consts: torch.Tensor,
                   const_count: torch.Tensor) -> "DevicePrograms":
        """View fixed-capacity slot arrays ([N, max_len], [N, max_consts]) as a population."""
        N, max_len = tokens.shape
        max_c = consts.shape[1]
        dev = tokens.device
        return DevicePrograms(tokens.reshape(-1), torch.arange(N, device=dev, dtype=torch.int64) * max_len,
                              lens, consts.reshape(-1), torch.arange(N, device=dev, dtype=torch.int64) * max_c,
                              const_count)

    def struct(self) -> _lib.Programs:
        for name, t, dt in (("tokens", self.tokens, torch.int16), ("tok_offset", self.tok_offset, torch.int64),
                            ("tok_len", self.tok_len, torch.int32), ("consts", self.consts, torch.float32),
                            ("const_offset", self.const_offset, torch.int64),
                            ("const_count", self.const_count, torch.int32)):
            if t.dtype != dt:
                raise TypeError(f"{name} must be {dt}, got {t.dtype}")
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
            if t.device != self.device:
                raise ValueError(f"{name} is on {t.device}, expected {self.device}")
        if self.device.type != "cuda":
            raise ValueError("programs must live on a GPU")
        return _lib.Programs(self.tokens.data_ptr(), self.tokens.numel(), self.tok_offset.data_ptr(),
                             self.tok_len.data_ptr(), self.consts.data_ptr(), self.consts.numel(),
                             self.const_offset.data_ptr(), self.const_count.data_ptr(), self.n)


def _dataset(X: torch.Tensor, y: torch.Tensor, device) -> _lib.Dataset:
    if X.dtype != torch.float32 or y.dtype != torch.float32:
        raise TypeError("X and y must be float32")
    if X.dim() != 2 or y.dim() != 1 or y.shape[0] != X.shape[0]:
        raise ValueError("X must be [M, D] and y [M]")
    if not X.is_contiguous() or not y.is_contiguous():
        raise ValueError("X and y must be contiguous")
    if X.device != device or y.device != device:
        raise ValueError("X and y must be on the programs' device")
    return _lib.Dataset(X.data_ptr(), y.data_ptr(), X.shape[0], X.shape[1])


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ctx_for(device: torch.device, ctx: Optional[Context]) -> Context:
    return ctx if ctx is not None else context(device.index or 0)


def evaluate(progs: DevicePrograms, X: torch.Tensor, y: torch.Tensor, kind="mse", *,
             with_status: bool = False, ctx: Optional[Context] = None):
    """fitness float64 [N] (and int8 status [N]) -- beagle_eval."""
    dev = progs.device
    c = _ctx_for(dev, ctx)
    ps = progs.struct()
    ds = _dataset(X, y, dev)
    fit = torch.empty(progs.n, dtype=torch.float64, device=dev)
    st = torch.empty(progs.n, dtype=torch.int8, device=dev) if with_status else None
    _check(c.lib.beagle_eval(c.handle, ctypes.byref(ps), ctypes.byref(ds), _kind(kind), fit.data_ptr(),
                             st.data_ptr() if st is not None else None, _stream(dev)))
    return (fit, st) if with_status else fit


def evaluate_static(progs: DevicePrograms, X: torch.Tensor, y: torch.Tensor, kind="mse", *,
                    fitness: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None):
    """beagle_eval_static: the evaluation without a context or any device
    allocation by the library (workspace in its static per-device array);
    pass preallocated `fitness` (float64 [N]) and `status` (int8 [N]) to keep
    the call allocation-free on the Python side too."""
    dev = progs.device
    lib = _lib.load()
    ps = progs.struct()
    ds = _dataset(X, y, dev)
    fit = fitness if fitness is not None else torch.empty(progs.n, dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        _check(lib.beagle_eval_static(ctypes.byref(ps), ctypes.byref(ds), _kind(kind), fit.data_ptr(),
                                      status.data_ptr() if status is not None else None, _stream(dev)))
    return fit


def evaluate_batched(problems, kind="mse", *, with_status: bool = False, ctx: Optional[Context] = None,
                     out=None):
    """Fitness of several independent problems in one batched launch --
    beagle_eval_batched.  problems: sequence of (DevicePrograms, X, y) on one
    device.  Returns a list of float64 [N_q] tensors (and of int8 status
    tensors).  `out`, if given, is a list of preallocated fitness tensors
    (reusing them lets repeated calls replay the same captured graph)."""
    problems = list(problems)
    n = len(problems)
    if n == 0:
        return ([], []) if with_status else []
    dev = problems[0][0].device
    c = _ctx_for(dev, ctx)
    P = (_lib.Programs * n)()
    D = (_lib.Dataset * n)()
    fits = []
    sts = []
    for q, (pr, X, y) in enumerate(problems):
        if pr.device != dev:
            raise ValueError("every problem must be on the same device")
        P[q] = pr.struct()
        D[q] = _dataset(X, y, dev)
        f = out[q] if out is not None else torch.empty(pr.n, dtype=torch.float64, device=dev)
        if f.dtype != torch.float64 or f.numel() != pr.n or f.device != dev or not f.is_contiguous():
            raise ValueError(f"out[{q}] must be a contiguous float64 tensor of {pr.n} elements on {dev}")
        fits.append(f)
        sts.append(torch.empty(pr.n, dtype=torch.int8, device=dev) if with_status else None)
    fptr = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fits])
    sptr = (ctypes.c_void_p * n)(*[s_.data_ptr() for s_ in sts]) if with_status else None
    _check(c.lib.beagle_eval_batched(c.handle, P, D, n, _kind(kind), fptr, sptr, _stream(dev)))
    return (fits, sts) if with_status else fits


def eval_workspace_bytes(progs: DevicePrograms, X: torch.Tensor, y: torch.Tensor, kind="mse") -> int:
    lib = _lib.load()
    ps = progs.struct()
    ds = _dataset(X, y, progs.device)
    out = ctypes.c_size_t()
    _check(lib.beagle_eval_workspace_size(ctypes.byref(ps), ctypes.byref(ds), _kind(kind), ctypes.byref(out)))
    return int(out.value)


def predict(progs: DevicePrograms, X: torch.Tensor, *, with_status: bool = False, ctx: Optional[Context] = None):
    """Per-case outputs float32 [N, M] -- beagle_predict."""
    dev = progs.device
    c = _ctx_for(dev, ctx)
    ps = progs.struct()
    y = torch.zeros(X.shape[0], dtype=torch.float32, device=dev)
    ds = _dataset(X, y, dev)
    out = torch.empty((progs.n, X.shape[0]), dtype=torch.float32, device=dev)
    st = torch.empty(progs.n, dtype=torch.int8, device=dev) if with_status else None
    _check(c.lib.beagle_predict(c.handle, ctypes.byref(ps), ctypes.byref(ds), out.data_ptr(),
                                st.data_ptr() if st is not None else None, _stream(dev)))
    return (out, st) if with_status else out


@dataclasses.dataclass
class GenParams:
    """beagle_gen_params: selection and variation settings."""

    tournament: int = 4
    p_crossover: float = 0.9
    p_mutation: float = 0.1
    max_len: int = 128
    max_consts: int = 8
    const_lo: float = -5.0
    const_hi: float = 5.0
    init_depth_min: int = 2
    init_depth_max: int = 6
    op_set: int = 0  # 0: + - * / sin cos exp log sqrt; 1: and x^2 1/x tan asin acos atan tanh

    def struct(self) -> _lib.GenParams:
        return _lib.GenParams(self.tournament, self.p_crossover, self.p_mutation, self.max_len, self.max_consts,
                              self.const_lo, self.const_hi, self.init_depth_min, self.init_depth_max, self.op_set)


@dataclasses.dataclass
class Slots:
    """A population in fixed-capacity slots (what initialisation and the
    generation step write): tokens [N, max_len] (uint16 bits in int16),
    len [N], consts [N, max_consts], const_count [N]."""

    tokens: torch.Tensor
    len: torch.Tensor
    consts: torch.Tensor
    const_count: torch.Tensor

    @staticmethod
    def empty(n: int, max_len: int, max_consts: int, device="cuda") -> "Slots":
        return Slots(torch.empty((n, max_len), dtype=torch.int16, device=device),
                     torch.empty(n, dtype=torch.int32, device=device),
                     torch.empty((n, max(max_consts, 1)), dtype=torch.float32, device=device)[:, :max_consts],
                     torch.empty(n, dtype=torch.int32, device=device))

    @property
    def n(self) -> int:
        return int(self.len.shape[0])

    def programs(self) -> DevicePrograms:
        return DevicePrograms.from_fixed(self.tokens, self.len, self.consts.contiguous(), self.const_count)


def init_population(n: int, D: int, params: GenParams, seed: int, problem: int = 0, device="cuda",
                    ctx: Optional[Context] = None) -> Slots:
    """Ramped half-and-half population -- beagle_init_population."""
    dev = torch.device(device)
    c = _ctx_for(dev, ctx)
    out = Slots.empty(n, params.max_len, params.max_consts, dev)
    p = params.struct()
    _check(c.lib.beagle_init_population(c.handle, ctypes.byref(p), n, D, seed, problem, out.tokens.data_ptr(),
                                        out.len.data_ptr(), out.consts.data_ptr(), out.const_count.data_ptr(),
                                        _stream(dev)))
    return out


def generation(parents: DevicePrograms, fitness: torch.Tensor, params: GenParams, D: int, seed: int,
               generation_index: int, problem: int = 0, out: Optional[Slots] = None,
               ctx: Optional[Context] = None) -> Slots:
    """One selection + variation step -- beagle_generation."""
    dev = parents.device
    c = _ctx_for(dev, ctx)
    if fitness.dtype != torch.float64 or fitness.device != dev or fitness.numel() != parents.n:
        raise ValueError("fitness must be float64 [N] on the parents' device")
    if out is None:
        out = Slots.empty(parents.n, params.max_len, params.max_consts, dev)
    ps = parents.struct()
    p = params.struct()
    _check(c.lib.beagle_generation(c.handle, ctypes.byref(ps), fitness.data_ptr(), ctypes.byref(p), D, seed,
                                   generation_index, problem, out.tokens.data_ptr(), out.len.data_ptr(),
                                   out.consts.data_ptr(), out.const_count.data_ptr(), _stream(dev)))
    return out


def generation_microcosm(parents: DevicePrograms, fitness: torch.Tensor, params: GenParams, D: int, seed: int,
                         generation_index: int, n_children: int, *, sample: int = 100, keep: float = 0.5,
                         problem: int = 0, out: Optional[Slots] = None, with_selection: bool = False,
                         ctx: Optional[Context] = None):
    """One generation under microcosm selection -- beagle_generation_microcosm.
    Returns the child slots, and with `with_selection` also the threshold
    (float64 [1]) and the survivor count (int32 [1]) as device tensors."""
    dev = parents.device
    c = _ctx_for(dev, ctx)
    if fitness.dtype != torch.float64 or fitness.device != dev or fitness.numel() != parents.n:
        raise ValueError("fitness must be float64 [N] on the parents' device")
    if out is None:
        out = Slots.empty(n_children, params.max_len, params.max_consts, dev)
    if out.n != n_children:
        raise ValueError("out must hold n_children slots")
    tau = torch.empty(1, dtype=torch.float64, device=dev)
    ns = torch.empty(1, dtype=torch.int32, device=dev)
    ps = parents.struct()
    p = params.struct()
    _check(c.lib.beagle_generation_microcosm(c.handle, ctypes.byref(ps), fitness.data_ptr(), ctypes.byref(p), D,
                                             sample, keep, seed, generation_index, problem, n_children,
                                             out.tokens.data_ptr(), out.len.data_ptr(), out.consts.data_ptr(),
                                             out.const_count.data_ptr(), tau.data_ptr(), ns.data_ptr(), _stream(dev)))
    return (out, tau, ns) if with_selection else out


def evaluate_score(progs: DevicePrograms, X: torch.Tensor, y: torch.Tensor, kind="point", max_score: float = 1000.0,
                   *, with_status: bool = False, ctx: Optional[Context] = None):
    """float64 [N] scores (higher is better) -- beagle_eval_score: "point" the
    sum over cases of the paper's Eq. 3, "r4" its Eq. 2; y may hold NaN/Inf."""
    dev = progs.device
    c = _ctx_for(dev, ctx)
    ps = progs.struct()
    ds = _dataset(X, y, dev)
    out = torch.empty(progs.n, dtype=torch.float64, device=dev)
    st = torch.empty(progs.n, dtype=torch.int8, device=dev) if with_status else None
    _check(c.lib.beagle_eval_score(c.handle, ctypes.byref(ps), ctypes.byref(ds), _kind(kind), float(max_score),
                                   out.data_ptr(), st.data_ptr() if st is not None else None, _stream(dev)))
    return (out, st) if with_status else out


def evaluate_grad(progs: DevicePrograms, X: torch.Tensor, y: torch.Tensor, kind="mse", *,
                  with_status: bool = False, ctx: Optional[Context] = None):
    """(fitness float64 [N], dF/dconsts float32 [n_consts]) -- beagle_eval_grad.

    Program p's gradient occupies consts[const_offset[p] : + const_count[p]]
    of the returned array; the programs' constant ranges must not overlap.
    """
    dev = progs.device
    c = _ctx_for(dev, ctx)
    ps = progs.struct()
    ds = _dataset(X, y, dev)
    fit = torch.empty(progs.n, dtype=torch.float64, device=dev)
    grad = torch.zeros(progs.consts.numel(), dtype=torch.float32, device=dev)
    st = torch.empty(progs.n, dtype=torch.int8, device=dev) if with_status else None
    _check(c.lib.beagle_eval_grad(c.handle, ctypes.byref(ps), ctypes.byref(ds), _kind(kind), fit.data_ptr(),
                                  grad.data_ptr(), st.data_ptr() if st is not None else None, _stream(dev)))
    return (fit, grad, st) if with_status else (fit, grad)
