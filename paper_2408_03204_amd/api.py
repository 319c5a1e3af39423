"""Python surface of the MI355X renderer: schedule, render (autograd Function), MRSTFT loss.

Mirrors the paper's example API (Sec. 4, Fig. 2a): `Schedule(...)` stands in for
`compute_render_data` (Algorithm 1 preprocessing, on the host in C++), `render(...)` for
`render_grafx` (the batched render loop, HIP kernels), with the hand-written adjoint behind
`torch.autograd.Function`. Every step runs in libgrafx; this module only marshals arguments.
PyTorch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, load

TYPE_CODES = {"in": 0, "out": 1, "mix": 2, "gain_pan": 3, "eq": 4, "compressor": 5, "imager": 6,
              "delay": 7, "tanh": 8, "noisegate": 9, "compressor_ar": 10, "reverb": 11,
              "delay_long": 12}
N_PARAMS = (0, 0, 0, 2, 1024, 4, 1, 220, 1, 4, 5, 768, 880)
NUM_TYPES = _lib.NUM_TYPES
METHODS = {"one_by_one": 0, "greedy": 1, "beam": 2, "optimal": 3}


def _iptr(a):
    return None if a is None else a.ctypes.data_as(_lib.c_i32p)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Schedule:
    """A scheduled graph: the type string, the node reordering and the read/write index lists,
    computed on the host by libgrafx (`grafx_schedule`)."""

    def __init__(self, node_type, edges, method: str | int = "beam", beam_width: int = 32,
                 state_limit: int = 1 << 20, edge_type=None, lengths=None):
        """`lengths` (optional, per node in node order): signal length of each node, for graphs
        of different lengths merged into one schedule (`merge_graphs`); the render's T is then
        the row stride (>= every length)."""
        lib = load()
        nt = np.ascontiguousarray(np.asarray(node_type), dtype=np.int32)
        e = np.asarray(edges, dtype=np.int32).reshape(2, -1)
        src, dst = np.ascontiguousarray(e[0]), np.ascontiguousarray(e[1])
        et = None if edge_type is None else np.ascontiguousarray(
            np.asarray(edge_type), dtype=np.int32).reshape(-1)
        m = METHODS[method] if isinstance(method, str) else int(method)
        h = ctypes.c_void_p()
        if lengths is None:
            check(lib.grafx_schedule(nt.shape[0], _iptr(nt), e.shape[1], _iptr(src), _iptr(dst),
                                     _iptr(et), m, beam_width, state_limit, ctypes.byref(h)))
        else:
            ln = np.ascontiguousarray(np.asarray(lengths), dtype=np.int32).reshape(-1)
            if ln.shape[0] != nt.shape[0]:
                raise ValueError("lengths must have one entry per node")
            check(lib.grafx_schedule_with_lengths(nt.shape[0], _iptr(nt), e.shape[1], _iptr(src),
                                                  _iptr(dst), _iptr(et), _iptr(ln), m, beam_width,
                                                  state_limit, ctypes.byref(h)))
        self._h = h
        s = _lib.ScheduleSizes()
        check(lib.grafx_schedule_query(h, ctypes.byref(s)))
        self.num_nodes, self.num_edges, self.num_steps = s.num_nodes, s.num_edges, s.num_steps
        self.num_inputs, self.num_outputs = s.num_inputs, s.num_outputs
        self.type_count = list(s.type_count)
        self.plan_bytes = int(s.plan_bytes)
        self.max_len = int(s.max_len)
        V, E, N = s.num_nodes, s.num_edges, s.num_steps
        arr = lambda n: np.zeros(max(n, 1), dtype=np.int32)  # noqa: E731
        self.step_type, self.step_ptr, self.perm = arr(N + 1), arr(N + 2), arr(V)
        self.in_ptr, self.in_src, self.out_ptr, self.out_dst = arr(V + 1), arr(E), arr(V + 1), arr(E)
        self.param_row = arr(V)
        check(lib.grafx_schedule_export(h, *[_iptr(a) for a in (
            self.step_type, self.step_ptr, self.perm, self.in_ptr, self.in_src, self.out_ptr,
            self.out_dst, self.param_row)]))
        self.in_src, self.out_dst = self.in_src[:E], self.out_dst[:E]
        # per-node lengths in reordered (sigma) order, or None when every node has the render's T
        self.len_sigma = None if lengths is None else ln[self.perm]
        self.out_begin = int(self.step_ptr[N])
        self._plans: dict = {}
        self._rv_noise, self.reverb_len = None, 0  # set_reverb_noise

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().grafx_schedule_free(h)
            except Exception:  # interpreter shutdown: the process releases the memory anyway
                pass
            self._h = None

    def type_string(self) -> tuple:
        return tuple(int(t) for t in self.step_type)

    def plan(self, device) -> torch.Tensor:
        """Device copy of the index lists (uploaded once per device, on the current stream)."""
        device = torch.device(device)
        if device not in self._plans:
            t = torch.empty(max(self.plan_bytes, 256), dtype=torch.uint8, device=device)
            check(load().grafx_plan_upload(self._h, t.data_ptr(), t.numel(), _stream(device)))
            self._plans[device] = t
        return self._plans[device]

    TUNE_POINTWISE_UNROLL = 0
    TUNE_AR_MAX_PASSES = 1
    TUNE_WAIT_POLLS = 2
    TUNE_EQ_ORDER = 3
    TUNE_DYN_ORDER = 4
    TUNE_TAP_TILES = 5

    def set_tuning(self, knob: int, value: int) -> None:
        """A tuning setting of the schedule (see include/grafx.h, grafx_schedule_set_tuning)."""
        check(load().grafx_schedule_set_tuning(self._h, knob, value))

    def get_tuning(self, knob: int) -> int:
        v = ctypes.c_int32()
        check(load().grafx_schedule_get_tuning(self._h, knob, ctypes.byref(v)))
        return int(v.value)

    def set_reverb_noise(self, noise) -> None:
        """The reverb's noise realisation: a float32 CUDA tensor [2, L] (mid, side) shared by
        every reverb node, or None to clear it. The schedule keeps a reference to the tensor,
        which the library borrows (see grafx_schedule_set_reverb_noise)."""
        if noise is None:
            check(load().grafx_schedule_set_reverb_noise(self._h, None, 0))
            self._rv_noise, self.reverb_len = None, 0
            return
        if not (torch.is_tensor(noise) and noise.is_cuda and noise.dtype == torch.float32
                and noise.dim() == 2 and noise.shape[0] == 2 and noise.is_contiguous()):
            raise ValueError("reverb noise must be a contiguous float32 CUDA tensor [2, L]")
        check(load().grafx_schedule_set_reverb_noise(self._h, noise.data_ptr(), noise.shape[1]))
        self._rv_noise, self.reverb_len = noise, int(noise.shape[1])

    def set_delay_surrogate(self, enable: bool) -> None:
        """Straight-through gradient of the delay phasors through the delay-time surrogate
        (see grafx_schedule_set_delay_surrogate); off by default (phasor gradients are 0)."""
        check(load().grafx_schedule_set_delay_surrogate(self._h, int(bool(enable))))

    def workspace_bytes(self, T: int, with_backward: bool) -> int:
        n = ctypes.c_size_t()
        check(load().grafx_workspace_bytes(self._h, T, int(with_backward), ctypes.byref(n)))
        return int(n.value)


def set_schedule_threads(n: int) -> int:
    """Host threads a beam or optimal search may use (0: the default, the host's concurrency up
    to 16); returns the previous setting. The schedule is the same for every count."""
    if n < 0:
        raise ValueError("thread count must be >= 0")
    return int(load().grafx_set_schedule_threads(int(n)))


def schedule_many(graphs, method: str | int = "beam", beam_width: int = 32, workers: int = 8):
    """Schedules of several graphs, computed concurrently on host threads (each call into the
    library releases the interpreter lock), in the order given. `graphs`: (node_type, edges) or
    (node_type, edges, lengths) per graph. Concurrent or not, each schedule is the one
    `Schedule` computes alone."""
    import concurrent.futures

    def one(g):
        lengths = g[2] if len(g) > 2 else None
        return Schedule(g[0], g[1], method, beam_width, lengths=lengths)

    graphs = list(graphs)
    if workers <= 1 or len(graphs) <= 1:
        return [one(g) for g in graphs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as pool:
        return list(pool.map(one, graphs))


def _param_list(sched: Schedule, P) -> list:
    out = [None] * NUM_TYPES
    for k, v in (P or {}).items():
        t = TYPE_CODES[k] if isinstance(k, str) else int(k)
        if not 0 <= t < NUM_TYPES:
            if v is not None and v.shape[0] == 0:
                continue  # an empty tensor of a type the library has no node of
            raise ValueError(f"unknown node type {t}")
        out[t] = v
    for t in range(NUM_TYPES):
        if N_PARAMS[t] and sched.type_count[t] > 0:
            p = out[t]
            if p is None:
                raise ValueError(f"missing parameters for node type {t}")
            if p.dtype != torch.float32 or not p.is_contiguous() or \
                    tuple(p.shape) != (sched.type_count[t], N_PARAMS[t]):
                raise ValueError(f"parameters of type {t} must be contiguous float32 "
                                 f"[{sched.type_count[t]}, {N_PARAMS[t]}]")
        elif N_PARAMS[t] == 0 or sched.type_count[t] == 0:
            out[t] = None
    return out


def _ptrs(tensors) -> "_lib.ptr_array":
    return _lib.ptr_array(*[(t.data_ptr() if t is not None else None) for t in tensors])


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sched: Schedule, holder: list, S: torch.Tensor, *P):
        dev = S.device
        K, T = sched.num_inputs, int(S.shape[-1])
        if S.dtype != torch.float32 or not S.is_contiguous() or tuple(S.shape) != (K, 2, T):
            raise ValueError(f"sources must be contiguous float32 [{K}, 2, T]")
        want_bwd = any(ctx.needs_input_grad[2:])
        U = torch.empty((sched.num_nodes, 2, T), dtype=torch.float32, device=dev)
        ws = torch.empty(max(sched.workspace_bytes(T, want_bwd), 256), dtype=torch.uint8,
                         device=dev)
        check(load().grafx_render(sched._h, sched.plan(dev).data_ptr(), T, S.data_ptr(),
                                  _ptrs(P), U.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream(dev)))
        ctx.sched, ctx.U, ctx.ws = sched, U, ws
        ctx.save_for_backward(S, *[p if p is not None else torch.empty(0) for p in P])
        ctx.present = [p is not None for p in P]
        holder.append(U)
        return U[sched.out_begin:]

    @staticmethod
    def backward(ctx, gY):
        sched, U, ws = ctx.sched, ctx.U, ctx.ws
        S, *P = ctx.saved_tensors
        P = [p if ok else None for p, ok in zip(P, ctx.present)]
        dev, T = U.device, U.shape[-1]
        dY = gY.contiguous() if gY is not None else torch.zeros_like(U[sched.out_begin:])
        dU = torch.empty_like(U)
        dS = torch.empty_like(S) if ctx.needs_input_grad[2] else None
        dP = [torch.empty_like(p) if (p is not None and ctx.needs_input_grad[3 + t]) else None
              for t, p in enumerate(P)]
        check(load().grafx_render_backward(
            sched._h, sched.plan(dev).data_ptr(), T, S.data_ptr(), _ptrs(P), U.data_ptr(),
            dY.data_ptr(), dU.data_ptr(), dS.data_ptr() if dS is not None else None, _ptrs(dP),
            ws.data_ptr(), ws.numel(), _stream(dev)))
        return (None, None, dS, *dP)


def delay_phasor_regularise(delay_type, P: torch.Tensor, dP: torch.Tensor,
                            weight: float) -> None:
    """grafx_delay_phasor_regularise, in place on dP: unit-length phasor gradients plus the
    gradient of weight * (|z| - 1)^2 (delay_type: "delay" / "delay_long" or their codes)."""
    t = TYPE_CODES[delay_type] if isinstance(delay_type, str) else int(delay_type)
    for x in (P, dP):
        if x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2 or \
                x.shape[1] != N_PARAMS[t]:
            raise ValueError(f"P and dP must be contiguous float32 [n, {N_PARAMS[t]}]")
    if P.shape != dP.shape:
        raise ValueError("P and dP must have one shape")
    check(load().grafx_delay_phasor_regularise(t, P.shape[0], P.data_ptr(), dP.data_ptr(),
                                               float(weight), _stream(dP.device)))


def render(sched: Schedule, S: torch.Tensor, P: dict, return_U: bool = False):
    """Batched render of the scheduled graph (paper Algorithm 1). S: [K, 2, T] float32 on the
    GPU; P: type (code or name) -> float32 [|V_t|, N_t]. Returns Y [|V_N|, 2, T] (and U
    [|V|, 2, T] in reordered order, whose input rows [0, K) are not written)."""
    holder: list = []
    Y = _Render.apply(sched, holder, S, *_param_list(sched, P))
    return (Y, holder[0]) if return_U else Y


def render_noalloc(sched: Schedule, plan: torch.Tensor, S: torch.Tensor, P: dict,
                   U: torch.Tensor) -> torch.Tensor:
    """grafx_render_noalloc: the render of `render` into the caller's U [|V|, 2, T] (float32,
    sigma order) with the library's static scratch as workspace, so the call allocates no device
    memory. `plan` is the schedule's device plan (`sched.plan(device)`, uploaded beforehand).
    Returns the output rows of U. Calls that overlap on one GPU share the scratch and race."""
    T = int(S.shape[-1])
    if tuple(U.shape) != (sched.num_nodes, 2, T) or U.dtype != torch.float32 or \
            not U.is_contiguous():
        raise ValueError(f"U must be contiguous float32 [{sched.num_nodes}, 2, {T}]")
    check(load().grafx_render_noalloc(sched._h, plan.data_ptr(), T, S.data_ptr(),
                                      _ptrs(_param_list(sched, P)), U.data_ptr(),
                                      _stream(U.device)))
    return U[sched.out_begin:]


class _MRSTFT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Y, target):
        rows, T = int(Y.shape[0]), int(Y.shape[-1])
        for t in (Y, target):
            if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (rows, 2, T):
                raise ValueError("Y and target must be contiguous float32 [rows, 2, T]")
        n = ctypes.c_size_t()
        lib = load()
        check(lib.grafx_mrstft_workspace_bytes(rows, T, ctypes.byref(n)))
        ws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=Y.device)
        loss = torch.empty((), dtype=torch.float32, device=Y.device)
        check(lib.grafx_mrstft_loss(rows, T, Y.data_ptr(), target.data_ptr(), loss.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream(Y.device)))
        ctx.save_for_backward(Y, target)
        ctx.ws = ws
        return loss

    @staticmethod
    def backward(ctx, gL):
        Y, target = ctx.saved_tensors
        rows, T = int(Y.shape[0]), int(Y.shape[-1])
        g = gL.detach().to(dtype=torch.float32).contiguous()
        dY = torch.empty_like(Y)
        check(load().grafx_mrstft_backward(rows, T, Y.data_ptr(), target.data_ptr(),
                                           g.data_ptr(), dY.data_ptr(), ctx.ws.data_ptr(),
                                           ctx.ws.numel(), _stream(Y.device)))
        return dY, None


def mrstft_loss(Y: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Multi-resolution STFT loss (512/1024/2048) between [rows, 2, T] signals."""
    return _MRSTFT.apply(Y.contiguous(), target.contiguous())


class RenderBuffers:
    """Explicit-buffer interface to the C ABI without autograd: owns U, the workspace and the
    adjoint buffer for one schedule, signal length and device. `forward`, `backward`, and the
    single-step calls enqueue on the current stream (used for live per-step timing)."""

    def __init__(self, sched: Schedule, T: int, device="cuda", with_backward: bool = True):
        self.sched, self.T, self.device = sched, int(T), torch.device(device)
        self.U = torch.empty((sched.num_nodes, 2, T), dtype=torch.float32, device=device)
        self.dU = torch.empty_like(self.U) if with_backward else None
        self.ws = torch.empty(max(sched.workspace_bytes(T, with_backward), 256),
                              dtype=torch.uint8, device=device)
        self.plan = sched.plan(device)

    @property
    def Y(self) -> torch.Tensor:
        return self.U[self.sched.out_begin:]

    def forward(self, S, P):
        Pl = _param_list(self.sched, P)
        check(load().grafx_render(self.sched._h, self.plan.data_ptr(), self.T, S.data_ptr(),
                                  _ptrs(Pl), self.U.data_ptr(), self.ws.data_ptr(),
                                  self.ws.numel(), _stream(self.device)))

    def backward(self, S, P, dY, dP: dict | None = None, dS=None):
        Pl = _param_list(self.sched, P)
        dPl = [None] * NUM_TYPES
        for k, v in (dP or {}).items():
            dPl[TYPE_CODES[k] if isinstance(k, str) else int(k)] = v
        check(load().grafx_render_backward(
            self.sched._h, self.plan.data_ptr(), self.T, S.data_ptr(), _ptrs(Pl),
            self.U.data_ptr(), dY.data_ptr(), self.dU.data_ptr(),
            dS.data_ptr() if dS is not None else None, _ptrs(dPl), self.ws.data_ptr(),
            self.ws.numel(), _stream(self.device)))

    def step(self, S, P, n: int):
        check(load().grafx_render_step(self.sched._h, self.plan.data_ptr(), self.T, S.data_ptr(),
                                       _ptrs(_param_list(self.sched, P)), self.U.data_ptr(),
                                       self.ws.data_ptr(), self.ws.numel(), n,
                                       _stream(self.device)))

    def error_word(self) -> int:
        """The dynamics kernels' error word of this workspace (bit 0: a chunk wait gave up, bit 1:
        tickets were not reset); waits for the current stream."""
        w = torch.zeros((), dtype=torch.int32, device=self.device)
        check(load().grafx_workspace_error(self.sched._h, self.T, self.ws.data_ptr(),
                                           self.ws.numel(), w.data_ptr(), _stream(self.device)))
        return int(w.item()) & 0xFFFFFFFF

    def backward_step(self, S, P, dY, n: int):
        check(load().grafx_render_backward_step(
            self.sched._h, self.plan.data_ptr(), self.T, S.data_ptr(),
            _ptrs(_param_list(self.sched, P)), self.U.data_ptr(), dY.data_ptr(),
            self.dU.data_ptr(), self.ws.data_ptr(), self.ws.numel(), n, _stream(self.device)))


class GradStep:
    """One gradient step of the mixing application (paper Sec. 4) with every buffer allocated up
    front: batched render of the scheduled graph, MRSTFT loss against a fixed target, the loss
    adjoint and the render adjoint down to per-type parameter gradients (`grads`).

    `run()` enqueues the step's launches on the current stream. `capture()` records the same
    launches once into a HIP graph and `replay()` re-issues them without host work per launch.
    Sources, parameters and target are read through their fixed addresses, so in-place updates
    between replays (an optimiser step on the parameters) are seen by the next replay; the loss
    lands in `loss`, the gradients in `grads[type]`."""

    def __init__(self, sched: Schedule, S: torch.Tensor, P: dict, target: torch.Tensor):
        self.sched, self.dev = sched, S.device
        T = int(S.shape[-1])
        K, rows = sched.num_inputs, sched.num_outputs
        if S.dtype != torch.float32 or not S.is_contiguous() or tuple(S.shape) != (K, 2, T):
            raise ValueError(f"sources must be contiguous float32 [{K}, 2, T]")
        if target.dtype != torch.float32 or not target.is_contiguous() or \
                tuple(target.shape) != (rows, 2, T):
            raise ValueError(f"target must be contiguous float32 [{rows}, 2, T]")
        self.S, self.target, self.T = S, target, T
        self.P = _param_list(sched, P)
        self.buf = RenderBuffers(sched, T, self.dev, with_backward=True)
        n = ctypes.c_size_t()
        check(load().grafx_mrstft_workspace_bytes(rows, T, ctypes.byref(n)))
        self.mws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=self.dev)
        self.loss = torch.empty((), dtype=torch.float32, device=self.dev)
        self.dloss = torch.ones((), dtype=torch.float32, device=self.dev)
        self.dY = torch.empty((rows, 2, T), dtype=torch.float32, device=self.dev)
        self.grads = {t: torch.empty_like(p) for t, p in enumerate(self.P) if p is not None}
        self._dP = [self.grads.get(t) for t in range(NUM_TYPES)]
        self.graph = None

    def run(self) -> torch.Tensor:
        lib, st, b, rows = load(), _stream(self.dev), self.buf, self.sched.num_outputs
        check(lib.grafx_render(self.sched._h, b.plan.data_ptr(), self.T, self.S.data_ptr(),
                               _ptrs(self.P), b.U.data_ptr(), b.ws.data_ptr(), b.ws.numel(), st))
        Y = b.Y
        check(lib.grafx_mrstft_loss(rows, self.T, Y.data_ptr(), self.target.data_ptr(),
                                    self.loss.data_ptr(), self.mws.data_ptr(), self.mws.numel(),
                                    st))
        check(lib.grafx_mrstft_backward(rows, self.T, Y.data_ptr(), self.target.data_ptr(),
                                        self.dloss.data_ptr(), self.dY.data_ptr(),
                                        self.mws.data_ptr(), self.mws.numel(), st))
        check(lib.grafx_render_backward(
            self.sched._h, b.plan.data_ptr(), self.T, self.S.data_ptr(), _ptrs(self.P),
            b.U.data_ptr(), self.dY.data_ptr(), b.dU.data_ptr(), None, _ptrs(self._dP),
            b.ws.data_ptr(), b.ws.numel(), st))
        return self.loss

    def capture(self) -> None:
        """Record `run()` into a HIP graph (after one eager run on a side stream, as graph capture
        requires)."""
        side = torch.cuda.Stream(self.dev)
        side.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.dev).wait_stream(side)
        torch.cuda.synchronize(self.dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()

    def replay(self) -> torch.Tensor:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self.loss


def merge_graphs(graphs):
    """Disconnected union of several graphs, so that one schedule renders them all (paper Sec. 2,
    "Batched processing": a batch of graphs is processed as one graph).

    `graphs`: sequence of (node_type, edges [2, E], T). Nodes and edges are concatenated in graph
    order, so the merged sources, parameters and outputs are plain concatenations too. Returns a
    dict: node_type, edges, lengths (each node's graph T), T (the row stride, the largest T), and
    per graph: node offset, input-row offset (into S), output-row offset (into Y) and, per node
    type, the parameter-row offset (into P[type])."""
    nts, eds, lens = [], [], []
    off = {"node": [], "input": [], "output": [], "param": []}
    n = 0
    cnt = np.zeros(NUM_TYPES, dtype=np.int64)
    for node_type, edges, T in graphs:
        nt = np.asarray(node_type, dtype=np.int32).reshape(-1)
        e = np.asarray(edges, dtype=np.int64).reshape(2, -1)
        off["node"].append(n)
        off["input"].append(int(cnt[TYPE_CODES["in"]]))
        off["output"].append(int(cnt[TYPE_CODES["out"]]))
        off["param"].append(cnt.copy())
        nts.append(nt)
        eds.append(e + n)
        lens.append(np.full(nt.shape[0], int(T), dtype=np.int32))
        n += nt.shape[0]
        cnt += np.bincount(nt, minlength=NUM_TYPES)
    return {"node_type": np.concatenate(nts), "edges": np.concatenate(eds, axis=1).astype(np.int32),
            "lengths": np.concatenate(lens), "T": int(max(int(g[2]) for g in graphs)),
            "node_offset": off["node"], "input_offset": off["input"],
            "output_offset": off["output"], "param_offset": off["param"]}


def merge_inputs(merged, sources, params):
    """Concatenate per-graph sources ([K_g, 2, T_g] each, zero-padded to the merged T) and
    parameters (dicts type -> [n_t, N_t]) in graph order, as numpy arrays."""
    T = merged["T"]
    S = np.concatenate([np.pad(np.asarray(s, dtype=np.float32),
                               ((0, 0), (0, 0), (0, T - np.asarray(s).shape[-1])))
                        for s in sources], axis=0)
    P = {}
    for t in range(NUM_TYPES):
        rows = [np.asarray(p[t], dtype=np.float32) for p in params if t in p]
        rows = [r for r in rows if r.shape[0] > 0]
        if rows:
            P[t] = np.ascontiguousarray(np.concatenate(rows, axis=0))
    return S, P
