"""Python binding of the AC library: torch tensors in, C ABI calls out.

Every step of the evaluation runs in the HIP kernels of ``libqkc.so``; this
module only checks shapes, dtypes and devices, allocates outputs and
workspaces with torch, and passes raw device pointers plus the current HIP
stream.  There is no CPU fallback: without the library (or a GPU) the calls
raise.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .blob import to_blob
from .compiler import CompiledAC, compile_circuit

_CDTYPE = {"c64": (L.AC_C64, torch.complex64), "c128": (L.AC_C128, torch.complex128)}


def _as_words(x):
    """Evidence words as an int64 tensor holding the uint64 bit patterns."""
    if isinstance(x, np.ndarray):
        return torch.from_numpy(np.ascontiguousarray(x).astype(np.uint64, copy=False).view(np.int64))
    if isinstance(x, torch.Tensor) and x.dtype == getattr(torch, "uint64", None):
        return x.view(torch.int64)
    return x


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class ACGraph:
    """A compiled arithmetic circuit resident on one GPU."""

    def __init__(self, source, device: int = 0):
        if isinstance(source, (bytes, bytearray)):
            blob = bytes(source)
            self.compiled = None
        else:
            compiled = source if isinstance(source, CompiledAC) else compile_circuit(source)
            blob = to_blob(compiled)
            self.compiled = compiled
        self.blob = blob
        self.device = int(device)
        self._h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        L.check(L.lib().ac_load(buf, len(blob), self.device, ctypes.byref(self._h)))
        inf = L.ACInfo()
        L.check(L.lib().ac_info(self._h, ctypes.byref(inf)))
        self.info = inf.as_dict()
        self._ws = {}

    # ------------------------------------------------------------------ util
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().ac_free(self._h)
            self._h = ctypes.c_void_p()
        self._ws = {}

    def release_workspaces(self):
        """Drop the cached per-(dtype, op) workspaces (they can be tens of GB
        for large batches); later calls allocate again as needed."""
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)

    def workspace_size(self, dtype: str, batch: int, op: int) -> int:
        return int(L.lib().ac_workspace_size(self._h, _CDTYPE[dtype][0], int(batch), int(op)))

    def workspace_size_share(self, dtype: str, batch: int, op: int, share: float) -> int:
        """Workspace bytes for the call run on ``share`` of the device's
        workgroups (smaller, slower, same results)."""
        n = int(L.lib().ac_workspace_size_share(self._h, _CDTYPE[dtype][0], int(batch), int(op), float(share)))
        if n == 0:
            raise L.ACError(L.AC_ERR_INVALID_ARG, L.lib().ac_last_error().decode())
        return n

    def sample_shape(self, dtype: str, chains: int):
        """(kernel, chains advanced at once) that ``sample`` uses for this many
        chains: kernel is "stream", "lds" or "global"."""
        kind, conc = ctypes.c_int32(), ctypes.c_int64()
        L.check(L.lib().ac_sample_shape(self._h, _CDTYPE[dtype][0], int(chains), ctypes.byref(kind),
                                        ctypes.byref(conc)))
        return ("stream", "lds", "global")[kind.value], int(conc.value)

    def workspace(self, dtype: str, batch: int, op: int, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The workspace for one call: ``ws`` if given, else a buffer cached
        per (dtype, op) on this graph.  The cached buffer is shared by every
        call on the graph, so callers that run the same graph on several
        streams at once pass their own ``ws``.  A ``ws`` smaller than
        ``workspace_size`` runs the call on fewer workgroups at once (the
        library refuses one below a single workgroup's region)."""
        need = self.workspace_size(dtype, batch, op)
        if ws is not None:
            if ws.device != self.torch_device or ws.dtype != torch.uint8:
                raise ValueError(f"workspace must be a uint8 tensor on {self.torch_device}")
            return ws
        key = (dtype, op)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.torch_device)
            self._ws[key] = ws
        return ws

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.torch_device).cuda_stream)

    def _dev(self, t, dtype, name, shape=None):
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.torch_device, dtype=dtype).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _inputs(self, theta, evidence, param_of, noise, validate=True):
        K = self.info["n_angles"]
        theta = self._dev(theta, torch.float64, "theta")
        if theta.dim() == 1:
            theta = theta.reshape(1, -1)
        if theta.shape[1] != K:
            raise ValueError(f"theta must have {K} columns, got {theta.shape[1]}")
        P = theta.shape[0]
        evidence = _as_words(evidence)
        evidence = self._dev(evidence, torch.int64, "evidence")
        if evidence.dim() == 1:
            evidence = evidence.reshape(1, -1)
        if evidence.shape[1] != self.info["n_words"]:
            raise ValueError(f"evidence must have {self.info['n_words']} words per row")
        B = evidence.shape[0]
        if param_of is None:
            if P != 1:
                raise ValueError("param_of is required when theta has more than one row")
            param_of = torch.zeros(B, dtype=torch.int32, device=self.torch_device)
        param_of = self._dev(param_of, torch.int32, "param_of", (B,))
        if validate and B > 0 and (int(param_of.min()) < 0 or int(param_of.max()) >= P):
            raise ValueError("param_of entries must lie in [0, P)")
        if noise is not None:
            noise = self._dev(noise, torch.float64, "noise", (self.info["n_noise"],))
            if validate and noise.numel() and (float(noise.min()) < 0.0 or float(noise.max()) > 1.0):
                raise ValueError("noise strengths must lie in [0, 1]")
        return theta, evidence, param_of, noise, P, B

    # ------------------------------------------------------------- queries
    def eval(self, theta, evidence, param_of=None, noise=None, dtype: str = "c64", prob: bool = True,
             validate: bool = True, ws: Optional[torch.Tensor] = None):
        """Amplitudes f(evidence[b]; theta[param_of[b]]) and optionally |f|^2 (FP64).
        validate=False skips the host-side range checks of param_of and noise
        (they synchronise with the device); only for inputs known to be valid."""
        code, cdt = _CDTYPE[dtype]
        theta, evidence, param_of, noise, P, B = self._inputs(theta, evidence, param_of, noise, validate)
        amp = torch.empty(B, dtype=cdt, device=self.torch_device)
        pr = torch.empty(B, dtype=torch.float64, device=self.torch_device) if prob else None
        ws = self.workspace(dtype, B, L.AC_OP_EVAL, ws)
        L.check(L.lib().ac_eval_batch(self._h, code, _ptr(theta), P, _ptr(noise), _ptr(param_of),
                                      _ptr(evidence), B, _ptr(amp), _ptr(pr), _ptr(ws), ws.numel(),
                                      self._stream()))
        return amp, pr

    def eval_static(self, theta, evidence, param_of=None, noise=None, dtype: str = "c64",
                    prob: bool = True, validate: bool = True, out=None):
        """``eval`` through ac_eval_batch_static: the library's own static
        scratch instead of a workspace, so the C call allocates nothing.
        ``out`` = (amp, prob) tensors to write into (the binding allocates
        them otherwise).  Calls on one GPU share that scratch: do not run two
        at once."""
        code, cdt = _CDTYPE[dtype]
        theta, evidence, param_of, noise, P, B = self._inputs(theta, evidence, param_of, noise, validate)
        if out is not None:
            amp, pr = out
            if amp.dtype != cdt or amp.numel() < B or (prob and (pr is None or pr.numel() < B)):
                raise ValueError("out: amplitudes of the dtype and probabilities of at least B entries")
        else:
            amp = torch.empty(B, dtype=cdt, device=self.torch_device)
            pr = torch.empty(B, dtype=torch.float64, device=self.torch_device) if prob else None
        L.check(L.lib().ac_eval_batch_static(self._h, code, _ptr(theta), P, _ptr(noise), _ptr(param_of),
                                             _ptr(evidence), B, _ptr(amp), _ptr(pr if prob else None),
                                             self._stream()))
        return amp, pr

    def mpe(self, theta, evidence, param_of=None, noise=None, validate: bool = True,
            ws: Optional[torch.Tensor] = None):
        """Most probable noise events for each element's outcome (see
        ac_mpe_batch; complex128, an AC compiled with the events decided
        first): (max_k |f(x, k)|^2 float64 [B], evidence words of (x, k*)
        uint64-as-int64 [B, n_words])."""
        theta, evidence, param_of, noise, P, B = self._inputs(theta, evidence, param_of, noise, validate)
        prob = torch.empty(B, dtype=torch.float64, device=self.torch_device)
        words = torch.empty((B, self.info["n_words"]), dtype=torch.int64, device=self.torch_device)
        ws = self.workspace("c128", B, L.AC_OP_MPE, ws)
        L.check(L.lib().ac_mpe_batch(self._h, _ptr(theta), P, _ptr(noise), _ptr(param_of), _ptr(evidence), B,
                                     _ptr(prob), _ptr(words), _ptr(ws), ws.numel(), self._stream()))
        return prob, words

    def grad(self, theta, evidence, param_of=None, mode: str = "cotangent", cotangent=None,
             weight=None, noise=None, dtype: str = "c64", want_amp=False, want_dfdtheta=False,
             want_dind=False, validate: bool = True, ws: Optional[torch.Tensor] = None):
        """Gradient in theta of a loss of the amplitudes (see ac_grad_batch)."""
        code, cdt = _CDTYPE[dtype]
        theta, evidence, param_of, noise, P, B = self._inputs(theta, evidence, param_of, noise, validate)
        m = {"cotangent": L.AC_GRAD_COTANGENT, "prob": L.AC_GRAD_PROB, "logprob": L.AC_GRAD_LOGPROB}[mode]
        cot = self._dev(cotangent, cdt, "cotangent", (B,)) if m == L.AC_GRAD_COTANGENT else None
        w = self._dev(weight, torch.float64, "weight", (B,)) if m != L.AC_GRAD_COTANGENT else None
        K = self.info["n_angles"]
        dev = self.torch_device
        grad = torch.empty((P, K), dtype=torch.float64, device=dev)
        amp = torch.empty(B, dtype=cdt, device=dev) if want_amp else None
        dft = torch.empty((B, K), dtype=cdt, device=dev) if want_dfdtheta else None
        dind = torch.empty((B, self.info["n_indicator_leaves"]), dtype=cdt, device=dev) if want_dind else None
        ws = self.workspace(dtype, B, L.AC_OP_GRAD, ws)
        L.check(L.lib().ac_grad_batch(self._h, code, _ptr(theta), P, _ptr(noise), _ptr(param_of),
                                      _ptr(evidence), B, m, _ptr(cot), _ptr(w), _ptr(grad), _ptr(amp),
                                      _ptr(dft), _ptr(dind), _ptr(ws), ws.numel(), self._stream()))
        return dict(grad=grad, amp=amp, dfdtheta=dft, dind=dind)

    def sample(self, theta, chains_per_param: int, samples_per_chain: int = 1, burn_in: int = 20,
               thin: int = 1, seed: int = 1, cost_edges: Optional[Sequence] = None, noise=None,
               dtype: str = "c64", want_states=False, want_cost=False, want_rounds=False,
               validate: bool = True, ws: Optional[torch.Tensor] = None, init_states=None,
               first_sweep: int = 0, first_var: int = 0, chain_offset: int = 0):
        """Gibbs samples of the output bits (see ac_sample).  ``init_states``
        (uint64/int64 [P * chains_per_param, n_words], e.g. the last sample's
        ``states`` of a previous call) starts every chain from a given state;
        ``first_sweep`` numbers this call's first sweep for the RNG, so a call
        resumed with the previous call's sweep count continues its chains.
        ``first_var`` > 0 keeps variables 0 .. first_var - 1 at their start
        values (conditional sampling, e.g. noise events given an outcome).
        ``chain_offset`` numbers this call's first chain for the RNG, so a
        request split into parts (by parameter sets or by chains of one set)
        draws exactly the chains of the whole request."""
        code, _ = _CDTYPE[dtype]
        K = self.info["n_angles"]
        theta = self._dev(theta, torch.float64, "theta")
        if theta.dim() == 1:
            theta = theta.reshape(1, -1)
        if theta.shape[1] != K:
            raise ValueError(f"theta must have {K} columns")
        P = theta.shape[0]
        if noise is not None:
            noise = self._dev(noise, torch.float64, "noise", (self.info["n_noise"],))
        dev = self.torch_device
        S = chains_per_param * samples_per_chain
        nwq = (self.info["n_qubits"] + 63) // 64
        i64 = torch.int64
        samples = torch.empty((P, S, nwq), dtype=i64, device=dev)
        states = torch.empty((P, S, self.info["n_words"]), dtype=i64, device=dev) if want_states else None
        edges_t = None
        if cost_edges is not None and len(cost_edges):
            edges_t = self._dev(torch.as_tensor(cost_edges, dtype=torch.int32).reshape(-1, 2), torch.int32, "edges")
            if validate and (int(edges_t.min()) < 0 or int(edges_t.max()) >= self.info["n_qubits"]):
                raise ValueError("cost edges must name qubits")
        cost = torch.empty((P, S), dtype=torch.float64, device=dev) if want_cost else None
        if want_cost and edges_t is None:
            raise ValueError("want_cost needs cost_edges")
        rounds = torch.empty(P * chains_per_param, dtype=i64, device=dev) if want_rounds else None
        init_t = None
        if init_states is not None:
            init_t = torch.as_tensor(_as_words(init_states))
            if init_t.numel() != P * chains_per_param * self.info["n_words"]:
                raise ValueError(f"init_states must hold {P * chains_per_param} x {self.info['n_words']} words")
            init_t = self._dev(init_t.reshape(P * chains_per_param, self.info["n_words"]), torch.int64,
                               "init_states")
        cfg = L.SampleCfg(int(chains_per_param), int(samples_per_chain), int(burn_in), int(thin),
                          int(seed) & ((1 << 64) - 1), 0 if edges_t is None else int(edges_t.shape[0]), 0,
                          None if edges_t is None else edges_t.data_ptr(),
                          None if init_t is None else init_t.data_ptr(), int(first_sweep), int(first_var),
                          int(chain_offset))
        ws = self.workspace(dtype, P * chains_per_param, L.AC_OP_SAMPLE, ws)
        L.check(L.lib().ac_sample(self._h, code, _ptr(theta), P, _ptr(noise), ctypes.byref(cfg),
                                  _ptr(samples), _ptr(states), _ptr(cost), _ptr(rounds), _ptr(ws),
                                  ws.numel(), self._stream()))
        return dict(samples=samples, states=states, cost=cost, rounds=rounds)


class ACAmplitude(torch.autograd.Function):
    """f = AC(evidence; theta[param_of]) with a hand-written adjoint backward."""

    @staticmethod
    def forward(ctx, theta, graph: ACGraph, evidence, param_of, dtype, noise):
        amp, _ = graph.eval(theta.detach(), evidence, param_of, noise, dtype, prob=False)
        ctx.graph, ctx.dtype = graph, dtype
        ctx.save_for_backward(theta.detach(), evidence, param_of)
        ctx.noise = noise
        return amp

    @staticmethod
    def backward(ctx, grad_amp):
        theta, evidence, param_of = ctx.saved_tensors
        out = ctx.graph.grad(theta, evidence, param_of, mode="cotangent",
                             cotangent=grad_amp.contiguous(), noise=ctx.noise, dtype=ctx.dtype)
        g = out["grad"].to(theta.dtype).reshape(theta.shape)
        return g, None, None, None, None, None


def amplitudes(graph: ACGraph, theta: torch.Tensor, evidence, param_of=None, dtype="c64", noise=None):
    """Differentiable amplitudes (theta may require grad)."""
    if param_of is None:
        param_of = torch.zeros(evidence.shape[0], dtype=torch.int32, device=graph.torch_device)
    return ACAmplitude.apply(theta, graph, evidence, param_of, dtype, noise)
