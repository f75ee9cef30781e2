"""Python binding of libttc.so: builds C descriptors from torch tensors,
allocates outputs and scratch with torch, and calls the C ABI on torch's
current HIP stream.  It does no arithmetic of its own."""
from __future__ import annotations

import ctypes
import sys
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import torch

from . import _abi
from ._abi import TT, TTM, Pair, TTCError

_lib = _abi.load()

_DT = {torch.float64: _abi.TTC_F64, torch.float32: _abi.TTC_F32, torch.bfloat16: _abi.TTC_BF16}


def _check(status: int):
    if status != _abi.TTC_OK:
        raise TTCError(status, _lib.ttc_last_error().decode())


def _stream(dev) -> c_void_p:
    return c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ws(nbytes: int, dev) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)


def _ptr(t) -> c_void_p:
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _i32(vals):
    return (c_int32 * max(len(vals), 1))(*[int(v) for v in vals])


def _check_cores(cores, name, dims):
    if len(cores) < 1:
        raise ValueError(f"{name}: empty core list")
    dev = cores[0].device
    dt = cores[0].dtype
    if dev.type != "cuda":
        raise ValueError(f"{name}: cores must be on a GPU device")
    if dt not in _DT:
        raise ValueError(f"{name}: dtype {dt} not supported")
    for c in cores:
        if c.device != dev or c.dtype != dt or not c.is_contiguous() or c.dim() != dims:
            raise ValueError(f"{name}: every core must be a contiguous {dims}-D {dt} tensor on {dev}")
    return dev, dt


class TTDesc:
    """C descriptor of a TT given as a list of (R, I, R') tensors."""

    def __init__(self, cores, name="tt", modes=None, ranks=None, check=True):
        self.cores = list(cores)
        if check:
            self.device, self.dtype = _check_cores(self.cores, name, 3)
        else:
            self.device, self.dtype = self.cores[0].device, self.cores[0].dtype
        if modes is None:
            modes = [int(c.shape[1]) for c in self.cores]
        if ranks is None:
            ranks = [int(self.cores[0].shape[0])] + [int(c.shape[2]) for c in self.cores]
        self.modes, self.ranks = list(modes), list(ranks)
        self._m = _i32(self.modes)
        self._r = _i32(self.ranks)
        self._c = (c_void_p * len(self.cores))(*[c.data_ptr() for c in self.cores])
        self.s = TT(len(self.cores), self._m, self._r, _DT[self.dtype], self._c)

    @property
    def ref(self):
        return byref(self.s)


class TTMDesc:
    """C descriptor of a TT-matrix given as a list of (R, I, J, R') tensors."""

    def __init__(self, cores, name="ttm"):
        self.cores = list(cores)
        self.device, self.dtype = _check_cores(self.cores, name, 4)
        self.rows = [int(c.shape[1]) for c in self.cores]
        self.cols = [int(c.shape[2]) for c in self.cores]
        self.ranks = [int(self.cores[0].shape[0])] + [int(c.shape[3]) for c in self.cores]
        self._rows, self._cols, self._r = _i32(self.rows), _i32(self.cols), _i32(self.ranks)
        self._c = (c_void_p * len(self.cores))(*[c.data_ptr() for c in self.cores])
        self.s = TTM(len(self.cores), self._rows, self._cols, self._r, _DT[self.dtype], self._c)

    @property
    def ref(self):
        return byref(self.s)


def _comp_dtype(dt):
    return torch.float64 if dt == torch.float64 else torch.float32


# ------------------------------------------------------------------ calls
def tt_contract_inner(x, y, prec: str = "auto") -> torch.Tensor:
    """<X, Y> as a 0-dim float64 tensor on the cores' device."""
    dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
    p = _abi.PREC[prec]
    need = c_size_t(0)
    _check(_lib.tt_contract_inner_query(dx.ref, dy.ref, p, byref(need)))
    out = torch.empty((), dtype=torch.float64, device=dx.device)
    ws = _ws(need.value, dx.device)
    _check(_lib.tt_contract_inner(dx.ref, dy.ref, p, _ptr(out), _ptr(ws), need.value, _stream(dx.device)))
    return out


def tt_contract_inner_noalloc(x, y, out: torch.Tensor, prec: str = "auto") -> torch.Tensor:
    """<X, Y> into `out` (a 0-dim float64 tensor on the cores' device) with
    the library's fixed workspace: nothing is allocated by this call."""
    dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
    if out.dtype != torch.float64 or out.numel() != 1 or out.device != dx.device:
        raise ValueError("out must be one float64 element on the cores' device")
    _check(_lib.tt_contract_inner_noalloc(dx.ref, dy.ref, _abi.PREC[prec], _ptr(out), _stream(dx.device)))
    return out


def tt_svd_query(dims, dtype=torch.float64, max_rank: int = 0):
    """(rank capacity per bond, workspace bytes) of tt_svd for a dense tensor
    of shape `dims`."""
    n = len(dims)
    cap = (c_int32 * (n + 1))()
    need = c_size_t(0)
    _check(_lib.tt_svd_query(n, _i32(dims), _DT[dtype], int(max_rank), cap, byref(need)))
    return list(cap), need.value


def tt_svd(x: torch.Tensor, eps: float = 0.0, max_rank: int = 0):
    """TT-SVD (Algorithm 1) of the dense tensor x (FP64 or FP32, on a GPU):
    list of cores (R_k, I_k, R_{k+1}) on x's device."""
    if x.device.type != "cuda" or not x.is_contiguous():
        raise ValueError("x must be a contiguous GPU tensor")
    dims = list(x.shape)
    cap, need = tt_svd_query(dims, x.dtype, max_rank)
    bufs = [torch.empty(cap[k] * dims[k] * cap[k + 1], dtype=x.dtype, device=x.device) for k in range(len(dims))]
    ptrs = (c_void_p * len(dims))(*[b.data_ptr() for b in bufs])
    ranks = (c_int32 * (len(dims) + 1))()
    ws = _ws(need, x.device)
    _check(_lib.tt_svd(_ptr(x), len(dims), _i32(dims), _DT[x.dtype], float(eps), int(max_rank), ranks, ptrs,
                       _ptr(ws), need, _stream(x.device)))
    r = list(ranks)
    return [bufs[k][: r[k] * dims[k] * r[k + 1]].view(r[k], dims[k], r[k + 1]) for k in range(len(dims))]


def tt_round(x, eps: float = 0.0, max_rank: int = 0):
    """TT-rounding of the cores x (FP64 or FP32): list of new cores on x's
    device, ranks chosen by Algorithm 1's delta rule."""
    dx = TTDesc(x, "x")
    n = len(x)
    cap = (c_int32 * (n + 1))()
    need = c_size_t(0)
    _check(_lib.tt_round_query(dx.ref, int(max_rank), cap, byref(need)))
    bufs = [torch.empty(cap[k] * dx.modes[k] * cap[k + 1], dtype=dx.dtype, device=dx.device) for k in range(n)]
    ptrs = (c_void_p * n)(*[b.data_ptr() for b in bufs])
    ranks = (c_int32 * (n + 1))()
    ws = _ws(need.value, dx.device)
    _check(_lib.tt_round(dx.ref, float(eps), int(max_rank), ranks, ptrs, _ptr(ws), need.value, _stream(dx.device)))
    r = list(ranks)
    return [bufs[k][: r[k] * dx.modes[k] * r[k + 1]].view(r[k], dx.modes[k], r[k + 1]) for k in range(n)]


def tt_contract_modes_query(x, y, modes, form: str = "junction", prec: str = "auto"):
    dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
    m = _i32(modes)
    order = c_int32(0)
    N = len(x)
    om = (c_int32 * (2 * N + 2))()
    orr = (c_int32 * (2 * N + 3))()
    elems = c_int64(0)
    need = c_size_t(0)
    _check(_lib.tt_contract_modes_query(dx.ref, dy.ref, m, len(modes), _abi.FORM[form], _abi.PREC[prec],
                                        byref(order), om, orr, byref(elems), byref(need)))
    n = order.value
    return {"order": n, "modes": list(om[:n]), "ranks": list(orr[: n + 1]) if form != "junction" else list(orr[:2]),
            "elems": elems.value, "ws": need.value}


def tt_contract_modes(x, y, modes, form: str = "junction", prec: str = "auto"):
    """Contraction over shared positions `modes` (0-based).  Returns the
    scalar when every position is contracted; else the junction matrix K,
    the list of natural-order cores, or the dense tensor.  prec "bf16" (BF16
    cores): the sweep on BF16 MFMA."""
    dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
    q = tt_contract_modes_query(x, y, modes, form, prec)
    dev = dx.device
    cdt = _comp_dtype(dx.dtype)
    ws = _ws(q["ws"], dev)
    m = _i32(modes)
    f, p = _abi.FORM[form], _abi.PREC[prec]
    st = _stream(dev)
    if len(set(int(v) for v in modes)) == len(x) and q["order"] == 0:
        out = torch.empty((), dtype=torch.float64, device=dev)
        _check(_lib.tt_contract_modes(dx.ref, dy.ref, m, len(modes), f, p, None, None, None, _ptr(out), _ptr(ws),
                                      q["ws"], st))
        return out
    if form == "junction":
        K = torch.empty(q["ranks"][0], q["ranks"][1], dtype=cdt, device=dev)
        _check(_lib.tt_contract_modes(dx.ref, dy.ref, m, len(modes), f, p, _ptr(K), None, None, None, _ptr(ws),
                                      q["ws"], st))
        return K
    if form == "natural":
        md, rk = q["modes"], q["ranks"]
        cores = [torch.empty(rk[k], md[k], rk[k + 1], dtype=cdt, device=dev) for k in range(q["order"])]
        od = TTDesc(cores, "out")
        _check(_lib.tt_contract_modes(dx.ref, dy.ref, m, len(modes), f, p, None, od.ref, None, None, _ptr(ws),
                                      q["ws"], st))
        return cores
    Z = torch.empty(*q["modes"], dtype=cdt, device=dev)
    _check(_lib.tt_contract_modes(dx.ref, dy.ref, m, len(modes), f, p, None, None, _ptr(Z), None, _ptr(ws), q["ws"],
                                  st))
    return Z


def tt_contract_pairs_query(x, y, xmodes, ymodes, form: str = "junction"):
    dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
    n = len(x) + len(y)
    order = c_int32(0)
    om = (c_int32 * (n + 2))()
    orr = (c_int32 * (n + 3))()
    elems = c_int64(0)
    need = c_size_t(0)
    _check(_lib.tt_contract_pairs_query(dx.ref, dy.ref, _i32(xmodes), _i32(ymodes), len(xmodes), _abi.FORM[form],
                                        byref(order), om, orr, byref(elems), byref(need)))
    k = order.value
    return {"order": k, "modes": list(om[:k]), "ranks": list(orr[:2]) if form == "junction" else list(orr[:k + 1]),
            "elems": elems.value, "ws": need.value}


def tt_contract_pairs(x, y, xmodes, ymodes, form: str = "junction"):
    """Contraction of X's modes `xmodes` with Y's modes `ymodes` (0-based,
    pairwise; eq. (8) once per pair).  Returns the scalar when every mode of
    both is contracted; else the junction T, the natural-order cores, or the
    dense tensor."""
    if len(xmodes) != len(ymodes):
        raise ValueError("one Y mode per X mode")
    dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
    q = tt_contract_pairs_query(x, y, xmodes, ymodes, form)
    dev = dx.device
    cdt = _comp_dtype(dx.dtype)
    ws = _ws(q["ws"], dev)
    xm, ym = _i32(xmodes), _i32(ymodes)
    f = _abi.FORM[form]
    st = _stream(dev)
    n = len(xmodes)
    if q["order"] == 0:
        out = torch.empty((), dtype=torch.float64, device=dev)
        _check(_lib.tt_contract_pairs(dx.ref, dy.ref, xm, ym, n, f, None, None, None, _ptr(out), _ptr(ws), q["ws"],
                                      st))
        return out
    if form == "junction":
        T = torch.empty(q["ranks"][0], q["ranks"][1], dtype=cdt, device=dev)
        _check(_lib.tt_contract_pairs(dx.ref, dy.ref, xm, ym, n, f, _ptr(T), None, None, None, _ptr(ws), q["ws"], st))
        return T
    if form == "natural":
        md, rk = q["modes"], q["ranks"]
        cores = [torch.empty(rk[k], md[k], rk[k + 1], dtype=cdt, device=dev) for k in range(q["order"])]
        od = TTDesc(cores, "out")
        _check(_lib.tt_contract_pairs(dx.ref, dy.ref, xm, ym, n, f, None, od.ref, None, None, _ptr(ws), q["ws"], st))
        return cores
    Z = torch.empty(*q["modes"], dtype=cdt, device=dev)
    _check(_lib.tt_contract_pairs(dx.ref, dy.ref, xm, ym, n, f, None, None, _ptr(Z), None, _ptr(ws), q["ws"], st))
    return Z


def tt_mode_n_product(x, modes, mats):
    """X x_n A_n for each (n, A_n); returns the new core list (unchanged cores
    are the input tensors themselves)."""
    dx = TTDesc(x, "x")
    modes = [int(v) for v in modes]
    if len(mats) != len(modes):
        raise ValueError("one matrix per mode")
    for A in mats:
        if A.device != dx.device or A.dtype != dx.dtype or not A.is_contiguous() or A.dim() != 2:
            raise ValueError("matrices must be contiguous 2-D tensors with the cores' dtype and device")
    out = list(x)
    J = []
    for n, A in zip(modes, mats):
        J.append(int(A.shape[0]))
        out[n] = torch.empty(x[n].shape[0], A.shape[0], x[n].shape[2], dtype=dx.dtype, device=dx.device)
    dy = TTDesc(out, "y")
    Ap = (c_void_p * len(mats))(*[A.data_ptr() for A in mats])
    _check(_lib.tt_mode_n_product(dx.ref, len(modes), _i32(modes), Ap, _i32(J), dy.ref, _stream(dx.device)))
    return out


def ttm_apply(w, v, prec: str = "auto"):
    """TT-matrix (cores (R, I, J, R')) times TT-vector; returns the output cores."""
    dm, dv = TTMDesc(w, "w"), TTDesc(v, "v")
    N = len(w)
    orr = (c_int32 * (N + 1))()
    elems = c_int64(0)
    _check(_lib.ttm_apply_query(dm.ref, dv.ref, orr, byref(elems)))
    cdt = _comp_dtype(dv.dtype)
    cores = [torch.empty(orr[k], dm.rows[k], orr[k + 1], dtype=cdt, device=dv.device) for k in range(N)]
    od = TTDesc(cores, "out")
    _check(_lib.ttm_apply(dm.ref, dv.ref, _abi.PREC[prec], od.ref, _stream(dv.device)))
    return cores


def ttm_apply_dense_query(w, batch: int, prec: str = "auto", sched: str = "auto", backward: bool = False) -> int:
    """Workspace bytes of ttm_apply_dense (backward False) or its backward."""
    dm = TTMDesc(w, "w")
    need = c_size_t(0)
    _check(_lib.ttm_apply_dense_query(dm.ref, int(batch), _abi.PREC[prec], _abi.SCHED[sched], int(backward),
                                      byref(need)))
    return need.value


def _layer_ws(ws, need: int, dev):
    if ws is None:
        return _ws(need, dev)
    if ws.device != dev or not ws.is_contiguous() or ws.numel() * ws.element_size() < need:
        raise ValueError("ws must be a contiguous tensor of at least the queried bytes on the cores' device")
    return ws


def ttm_apply_dense(w, x: torch.Tensor, prec: str = "auto", sched: str = "auto", ws=None) -> torch.Tensor:
    """Y = X W^T for a batch X (batch x prod J, little-endian rows).  ws:
    the workspace (a device tensor of at least ttm_apply_dense_query bytes;
    required for sched "cores_saved", whose backward reads it)."""
    dm = TTMDesc(w, "w")
    if x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2 or x.device != dm.device:
        raise ValueError("x must be a contiguous 2-D float32 tensor on the cores' device")
    if sched == "cores_saved" and ws is None:
        raise ValueError('sched "cores_saved" needs a workspace kept for the backward')
    B = int(x.shape[0])
    need = c_size_t(0)
    p, s = _abi.PREC[prec], _abi.SCHED[sched]
    _check(_lib.ttm_apply_dense_query(dm.ref, B, p, s, 0, byref(need)))
    rows = 1
    for r in dm.rows:
        rows *= r
    y = torch.empty(B, rows, dtype=torch.float32, device=dm.device)
    ws = _layer_ws(ws, need.value, dm.device)
    _check(_lib.ttm_apply_dense(dm.ref, _ptr(x), B, _ptr(y), p, s, _ptr(ws), need.value, _stream(dm.device)))
    return y


def ttm_apply_dense_bwd(w, x: torch.Tensor, dy: torch.Tensor, prec: str = "auto", sched: str = "auto",
                        need_dx: bool = True, need_dw: bool = True, ws=None):
    dm = TTMDesc(w, "w")
    for t in (x, dy):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2 or t.device != dm.device:
            raise ValueError("x and dy must be contiguous 2-D float32 tensors on the cores' device")
    if sched == "cores_saved" and ws is None:
        raise ValueError('sched "cores_saved" needs the forward\'s workspace')
    B = int(x.shape[0])
    need = c_size_t(0)
    p, s = _abi.PREC[prec], _abi.SCHED[sched]
    _check(_lib.ttm_apply_dense_query(dm.ref, B, p, s, 1, byref(need)))
    dx = torch.empty_like(x) if need_dx else None
    dcores = [torch.empty(c.shape, dtype=torch.float32, device=dm.device) for c in w] if need_dw else None
    dptr = (c_void_p * len(w))(*[c.data_ptr() for c in dcores]) if need_dw else None
    ws = _layer_ws(ws, need.value, dm.device)
    _check(_lib.ttm_apply_dense_bwd(dm.ref, _ptr(x), _ptr(dy), B, _ptr(dx), dptr, p, s, _ptr(ws), need.value,
                                    _stream(dm.device)))
    return dx, dcores


def ttc_mse_loss(y: torch.Tensor, t: torch.Tensor, need_grad: bool = True):
    """(L = mean((y - t)^2) as a 0-dim float64 tensor, dL/dy or None)."""
    if y.shape != t.shape or y.dtype != torch.float32 or t.dtype != torch.float32:
        raise ValueError("y and t must be float32 tensors of one shape")
    if not (y.is_contiguous() and t.is_contiguous()) or y.device != t.device:
        raise ValueError("y and t must be contiguous on one device")
    n = y.numel()
    need = c_size_t(0)
    _check(_lib.ttc_mse_loss_query(n, byref(need)))
    loss = torch.empty((), dtype=torch.float64, device=y.device)
    dy = torch.empty_like(y) if need_grad else None
    ws = _ws(need.value, y.device)
    _check(_lib.ttc_mse_loss(_ptr(y), _ptr(t), n, _ptr(loss), _ptr(dy), _ptr(ws), need.value, _stream(y.device)))
    return loss, dy


def tt_contract_inner_bwd(x, y, gz, ckpt_stride: int = 0, need_x: bool = True, need_y: bool = True):
    """Gradients of gz * <X, Y> with respect to every core of X and Y."""
    dx_, dy_ = TTDesc(x, "x"), TTDesc(y, "y")
    dev = dx_.device
    if not torch.is_tensor(gz):
        # a device fill, not a host-to-device copy (which would wait for the
        # stream's earlier work)
        gz = torch.full((), float(gz), dtype=torch.float64, device=dev)
    gz = gz.to(device=dev, dtype=torch.float64).reshape(())
    need = c_size_t(0)
    _check(_lib.tt_contract_inner_bwd_query(dx_.ref, dy_.ref, int(ckpt_stride), byref(need)))
    cdt = _comp_dtype(dx_.dtype)
    gx = [torch.empty(c.shape, dtype=cdt, device=dev) for c in x] if need_x else None
    gy = [torch.empty(c.shape, dtype=cdt, device=dev) for c in y] if need_y else None
    px = (c_void_p * len(x))(*[t.data_ptr() for t in gx]) if need_x else None
    py = (c_void_p * len(y))(*[t.data_ptr() for t in gy]) if need_y else None
    ws = _ws(need.value, dev)
    _check(_lib.tt_contract_inner_bwd(dx_.ref, dy_.ref, _ptr(gz), px, py, int(ckpt_stride), _ptr(ws), need.value,
                                      _stream(dev)))
    return gx, gy


class BatchPlan:
    """Plan for many (X, Y) pairs in one persistent launch (see tt_batch_plan_create)."""

    def __init__(self, pairs, ops=_abi.OP_INNER | _abi.OP_SUFFIX2, prec: str = "auto"):
        self.pairs = [(list(x), list(y)) for x, y in pairs]
        self.n = len(self.pairs)
        self._descs = []
        arr = (Pair * self.n)()
        dev = None
        for p, (x, y) in enumerate(self.pairs):
            dx, dy = TTDesc(x, "x"), TTDesc(y, "y")
            dev = dx.device
            self._descs.append((dx, dy))
            arr[p].x = dx.s
            arr[p].y = dy.s
        self.device = dev
        self._arr = arr
        self.ops = ops
        h = c_void_p(0)
        _check(_lib.tt_batch_plan_create(arr, self.n, ops, _abi.PREC[prec], byref(h)))
        self._h = h
        offs = (c_int64 * (self.n + 1))()
        fl, by = c_double(0), c_double(0)
        _check(_lib.tt_batch_plan_info(self._h, offs, byref(fl), byref(by)))
        self.junction_offsets = list(offs)
        self.flops, self.bytes = fl.value, by.value
        m, t, pc = c_int32(), c_int32(), c_int32()
        _check(_lib.tt_batch_plan_config(self._h, byref(m), byref(t), byref(pc)))
        self.config = {"mode": ("persistent", "levels", "lds", "lds1", "lds1b")[m.value], "threads": t.value, "wg_per_cu": pc.value}

    def outputs(self):
        inner = torch.empty(self.n, dtype=torch.float64, device=self.device)
        junc = torch.empty(max(self.junction_offsets[-1], 1), dtype=torch.float32, device=self.device)
        return inner, junc

    def run(self, inner=None, junction=None, plain: bool = False):
        if inner is None:
            inner, junction = self.outputs()
        f = _lib.tt_batch_run_plain if plain else _lib.tt_batch_run
        _check(f(self._h, _ptr(inner), _ptr(junction), _stream(self.device)))
        return inner, junction

    def run_traced(self, inner=None, junction=None):
        """Run once with tracing; returns (inner, junction, clock, steps):
        clock[p] = (start, end, workgroup) and steps[p, j] the clock after
        sweep step j (the final product at j = N-1), in GPU shader cycles."""
        if inner is None:
            inner, junction = self.outputs()
        n = self.n
        clk = torch.zeros(35 * n, dtype=torch.int64, device=self.device)
        _check(_lib.tt_batch_run_traced(self._h, _ptr(inner), _ptr(junction), _ptr(clk), _stream(self.device)))
        c = clk.cpu()
        per = torch.stack([c[0:2 * n:2], c[1:2 * n:2], c[2 * n:3 * n]], dim=1)
        return inner, junction, per, c[3 * n:].view(n, 32)

    def junction(self, junction, p):
        x, y = self.pairs[p]
        N = len(x)
        R, P = int(x[N - 2].shape[0]), int(y[N - 2].shape[0])
        o = self.junction_offsets[p]
        return junction[o:o + R * P].view(R, P)

    def __del__(self, _destroy=_lib.tt_batch_plan_destroy, _finalizing=sys.is_finalizing):
        # at interpreter exit ctypes may already be torn down; the process
        # ending releases the plan's device memory anyway
        h = getattr(self, "_h", None)
        if h is not None and h.value and not _finalizing():
            _destroy(h)
            self._h = c_void_p(0)


def version() -> str:
    return _lib.ttc_version().decode()
