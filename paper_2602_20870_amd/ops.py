"""Torch-facing wrapper of the FGFRFT C ABI: device memory and streams from
PyTorch, every computation in the HIP library (argument marshalling only).

    plan = Plan(F_cuda, L)                 # offline stage, Algorithm 1
    Q = plan.update(alphas)                # Q_L^alpha for many orders (Definition 1)
    Y = plan.apply(alphas, X)              # Q_L^alpha X (Definition 2)
    Y = plan.apply_direct(alphas, cols, X) # the same without forming Q (one order per column)
    da, dX = plan.grad(alphas, X, GY)      # Proposition 4
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import P_double, check, lib

STACK_TYPES = {"fp32": 0, "bf16x2": 1, "fp16x2": 2}
FORMS = {"split": 0, "standard": 1}


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _alphas(alphas) -> np.ndarray:
    if isinstance(alphas, torch.Tensor):
        alphas = alphas.detach().cpu().numpy()
    return np.ascontiguousarray(np.atleast_1d(np.asarray(alphas, dtype=np.float64)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _on_device(dev, **tensors) -> None:
    """Every buffer handed to the library is read or written by its kernels as a raw pointer, so each
    must be device memory on the GPU the call runs on (None entries are skipped)."""
    for name, t in tensors.items():
        if t is not None and (not t.is_cuda or t.device != dev):
            raise ValueError(f"{name} must be a cuda tensor on {dev}")


def _caller_ws(ws, need: int, dev):
    """(workspace, temporary): the caller's workspace when it is large enough, else a new one.  A
    caller's workspace must be contiguous uint8 memory on `dev` (its size is counted in bytes)."""
    if ws is not None:
        _on_device(dev, ws=ws)
        if ws.dtype != torch.uint8 or not ws.is_contiguous():
            raise ValueError("ws must be a contiguous uint8 tensor")
        if ws.numel() >= need:
            return ws, None
    tmp = _workspace(need, dev)
    return tmp, tmp


def _keep(stream, *tensors) -> None:
    """Temporaries allocated here on the current stream but used by work queued on `stream`: tell
    the caching allocator, so their memory is not handed out again before that work has run."""
    if stream is not None:
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


class Plan:
    """Offline stage of Algorithm 1 on the GPU for a unitary F.

    F: cuda tensor, float64 (real orthogonal F) or complex128, shape [N, N].
    The persistent buffer (power stack M_1..M_L and P) is a torch tensor owned
    by this object; the FP64 planning scratch is released when planning ends.
    """

    def __init__(self, F: torch.Tensor, L: int, stacktype: str = "fp32", tau: float = 0.0, stream=None,
                 form: str = "split"):
        if not F.is_cuda:
            raise ValueError("F must be a cuda tensor")
        if stacktype not in STACK_TYPES:
            raise ValueError(f"stacktype must be one of {sorted(STACK_TYPES)}")
        if form not in FORMS:
            raise ValueError(f"form must be one of {sorted(FORMS)}")
        if F.dtype == torch.float64:
            intype = 1
        elif F.dtype == torch.complex128:
            intype = 0
        else:
            raise TypeError("F must be float64 or complex128")
        F = F.contiguous()
        N = F.shape[0]
        if F.shape != (N, N):
            raise ValueError("F must be square")
        L_ = lib()
        pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        check(L_.fgfrft_plan_bytes(N, L, intype, STACK_TYPES[stacktype], ctypes.byref(pb), ctypes.byref(sb)),
              "fgfrft_plan_bytes")
        self.device = F.device
        self.persistent = _workspace(pb.value, F.device)
        scratch = _workspace(sb.value, F.device)
        h = ctypes.c_void_p()
        check(L_.fgfrft_plan(_ptr(F), N, L, intype, STACK_TYPES[stacktype], FORMS[form], float(tau),
                             _ptr(self.persistent),
                             pb.value, _ptr(scratch), sb.value, _stream(stream), ctypes.byref(h)), "fgfrft_plan")
        del scratch
        self._h = h
        self._destroy = L_.fgfrft_destroy   # held here: module globals may be gone when __del__ runs at exit
        self.N, self.L = N, L
        self.complex = intype == 0
        self.stacktype = stacktype
        self.form = form

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    # ------------------------------------------------------------------ info
    def info(self) -> dict:
        r = ctypes.c_int()
        u, d, sn, lp, tu = (ctypes.c_double() for _ in range(5))
        check(lib().fgfrft_plan_info(self._h, ctypes.byref(r), ctypes.byref(u), ctypes.byref(d), ctypes.byref(sn),
                                     ctypes.byref(lp), ctypes.byref(tu)), "fgfrft_plan_info")
        return dict(r_minus1=r.value, unitarity_defect=u.value, drift=d.value, stop_norm=sn.value,
                    last_pivot_norm=lp.value, tau_used=tu.value)

    @property
    def r_minus1(self) -> int:
        return self.info()["r_minus1"]

    def buffers(self):
        """(stack, P) as torch views of the resident data: stack[n-1] = F^n P_c and
        stack[L+n-1] = F^{-n} P_c = (F^n P_c)^H for n = 1..L (typed views for the FP32 stack)."""
        N, L = self.N, self.L
        s, p = ctypes.c_void_p(), ctypes.c_void_p()
        check(lib().fgfrft_plan_buffers(self._h, ctypes.byref(s), ctypes.byref(p)), "fgfrft_plan_buffers")
        base = self.persistent.data_ptr()
        es = 8 if self.complex else 4
        stack = self.persistent[: 2 * L * N * N * es]
        poff = p.value - base
        P = self.persistent[poff: poff + N * N * es]
        if self.stacktype == "fp32":
            dt = torch.complex64 if self.complex else torch.float32
            stack = stack.view(dt).view(2 * L, N, N)
        P = P.view(torch.complex64 if self.complex else torch.float32).view(N, N)
        return stack, P

    # ------------------------------------------------------------------ online stage
    def update(self, alphas, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        a = _alphas(alphas)
        n = a.size
        if out is None:
            out = torch.empty((n, self.N, self.N), dtype=torch.complex64, device=self.device)
        _on_device(self.device, out=out)
        if out.dtype != torch.complex64 or not out.is_contiguous() or out.numel() < n * self.N * self.N:
            raise ValueError("out must be a contiguous complex64 tensor of n_alpha*N*N elements")
        L_ = lib()
        ws = _workspace(L_.fgfrft_update_workspace_bytes(self._h, n), self.device)
        check(L_.fgfrft_update(self._h, a.ctypes.data_as(P_double), n, _ptr(out), _ptr(ws), ws.numel(),
                               _stream(stream)), "fgfrft_update")
        _keep(stream, ws)
        return out

    def update_dev(self, alphas_dev: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
        """Update with the orders already on the device (float64 cuda tensor); capturable.

        Orders with |alpha| >= L give NaN planes (no host-side check is possible).
        """
        _on_device(self.device, alphas_dev=alphas_dev, out=out)
        if alphas_dev.dtype != torch.float64 or not alphas_dev.is_contiguous():
            raise ValueError("alphas_dev must be a contiguous float64 cuda tensor")
        n = alphas_dev.numel()
        if out.dtype != torch.complex64 or not out.is_contiguous() or out.numel() < n * self.N * self.N:
            raise ValueError("out must be a contiguous complex64 tensor of n_alpha*N*N elements")
        L_ = lib()
        ws, tmp = _caller_ws(ws, L_.fgfrft_update_workspace_bytes(self._h, n), self.device)
        check(L_.fgfrft_update_dev(self._h, _ptr(alphas_dev), n, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
              "fgfrft_update_dev")
        _keep(stream, tmp)
        return out

    def update_dev_static(self, alphas_dev: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """update_dev without a workspace: the library's fixed per-GPU tables (at most 4096 orders per
        call; calls that overlap on one GPU race on those tables)."""
        _on_device(self.device, alphas_dev=alphas_dev, out=out)
        if alphas_dev.dtype != torch.float64 or not alphas_dev.is_contiguous():
            raise ValueError("alphas_dev must be a contiguous float64 cuda tensor")
        n = alphas_dev.numel()
        if out.dtype != torch.complex64 or not out.is_contiguous() or out.numel() < n * self.N * self.N:
            raise ValueError("out must be a contiguous complex64 tensor of n_alpha*N*N elements")
        check(lib().fgfrft_update_dev_static(self._h, _ptr(alphas_dev), n, _ptr(out), _stream(stream)),
              "fgfrft_update_dev_static")
        return out

    def update_workspace_bytes(self, n_alpha: int) -> int:
        return int(lib().fgfrft_update_workspace_bytes(self._h, n_alpha))

    def apply(self, alphas, X: torch.Tensor, chunk: int = 0, stream=None, out: torch.Tensor | None = None,
              ws: torch.Tensor | None = None) -> torch.Tensor:
        """Y[a] = Q(alphas[a]) X[a] with X [n_alpha, N, B] or a shared [N, B] block.

        A real F with real signals takes the library's real-F route (the operator's real part R plus
        the rank-r imaginary part from P's basis).  out: complex64 [n_alpha, N, B]; ws: a caller
        workspace (contiguous uint8 cuda tensor) reused when large enough."""
        a = _alphas(alphas)
        n = a.size
        x_shared = X.dim() == 2
        B = X.shape[-1]
        xc = _check_signal(X, n, self.N, x_shared, self.device)
        if out is None:
            out = torch.empty((n, self.N, B), dtype=torch.complex64, device=self.device)
        _on_device(self.device, out=out)
        if out.dtype != torch.complex64 or not out.is_contiguous() or out.numel() != n * self.N * B:
            raise ValueError("out must be a contiguous complex64 tensor of n_alpha*N*B elements")
        L_ = lib()
        ws, tmp = _caller_ws(ws, L_.fgfrft_apply_workspace_bytes(self._h, n, B, xc, int(x_shared), chunk), self.device)
        check(L_.fgfrft_apply(self._h, a.ctypes.data_as(P_double), n, _ptr(X), xc, int(x_shared), B, _ptr(out), chunk,
                              _ptr(ws), ws.numel(), _stream(stream)), "fgfrft_apply")
        _keep(stream, tmp)
        return out

    def apply_workspace_bytes(self, n_alpha: int, B: int, x_complex: bool = False, x_shared: bool = False,
                              chunk: int = 0) -> int:
        return int(lib().fgfrft_apply_workspace_bytes(self._h, n_alpha, B, int(x_complex), int(x_shared), chunk))

    def apply_dev(self, alphas_dev: torch.Tensor, X: torch.Tensor, out: torch.Tensor,
                  ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """apply with the orders already on the device (float64 cuda tensor), all in one update
        launch; enqueues kernels only (capturable with a caller workspace).  Orders with
        |alpha| >= L give NaN outputs (no host-side check is possible)."""
        _on_device(self.device, alphas_dev=alphas_dev, out=out)
        if alphas_dev.dtype != torch.float64 or not alphas_dev.is_contiguous():
            raise ValueError("alphas_dev must be a contiguous float64 cuda tensor")
        n = alphas_dev.numel()
        x_shared = X.dim() == 2
        B = X.shape[-1]
        xc = _check_signal(X, n, self.N, x_shared, self.device)
        if out.dtype != torch.complex64 or not out.is_contiguous() or out.numel() != n * self.N * B:
            raise ValueError("out must be a contiguous complex64 tensor of n_alpha*N*B elements")
        L_ = lib()
        ws, tmp = _caller_ws(ws, L_.fgfrft_apply_dev_workspace_bytes(self._h, n, B, xc, int(x_shared)), self.device)
        check(L_.fgfrft_apply_dev(self._h, _ptr(alphas_dev), n, _ptr(X), xc, int(x_shared), B, _ptr(out), _ptr(ws),
                                  ws.numel(), _stream(stream)), "fgfrft_apply_dev")
        _keep(stream, tmp)
        return out

    def apply_dev_workspace_bytes(self, n_alpha: int, B: int, x_complex: bool = False, x_shared: bool = False) -> int:
        return int(lib().fgfrft_apply_dev_workspace_bytes(self._h, n_alpha, B, int(x_complex), int(x_shared)))

    def apply_batched(self, alphas, Xs, outs=None, ws: torch.Tensor | None = None, stream=None) -> list:
        """Grouped apply: request r gets Q(alphas[r]) Xs[r], each with its own order and signal count.

        alphas: host sequence of n orders; Xs: n contiguous cuda tensors [N, B_r] (all float32 or all
        complex64); outs: n complex64 [N, B_r] tensors or None.  One gather, one direct-route pass and
        one scatter per group of 64 requests, all on the device.
        """
        dev = self.device
        al = _alphas(alphas)
        n = al.size
        if len(Xs) != n:
            raise ValueError("one signal block per order")
        dts = {X.dtype for X in Xs}
        if dts == {torch.float32}:
            xc = 0
        elif dts == {torch.complex64}:
            xc = 1
        else:
            raise TypeError("signals must be all float32 or all complex64")
        for X in Xs:
            _on_device(dev, X=X)
            if X.dim() != 2 or X.shape[0] != self.N or not X.is_contiguous():
                raise ValueError(f"each signal block must be a contiguous cuda tensor of shape [{self.N}, B]")
        if outs is None:
            outs = [torch.empty((self.N, X.shape[1]), dtype=torch.complex64, device=dev) for X in Xs]
        if len(outs) != n:
            raise ValueError("one output per order")
        for X, Y in zip(Xs, outs):
            _on_device(dev, out=Y)
            if Y.shape != X.shape or Y.dtype != torch.complex64 or not Y.is_contiguous():
                raise ValueError("each output must be a contiguous complex64 tensor shaped like its signals")
        B = (ctypes.c_int * n)(*[int(X.shape[1]) for X in Xs])
        xp = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
        yp = (ctypes.c_void_p * n)(*[Y.data_ptr() for Y in outs])
        L_ = lib()
        ws, tmp = _caller_ws(ws, L_.fgfrft_apply_batched_workspace_bytes(self._h, n, B, xc), dev)
        check(L_.fgfrft_apply_batched(self._h, al.ctypes.data_as(P_double), n, B, xp, xc, yp, _ptr(ws), ws.numel(),
                                      _stream(stream)), "fgfrft_apply_batched")
        _keep(stream, tmp)
        return outs

    def apply_direct(self, alphas, col_order, X: torch.Tensor, ncols: int | None = None, out: torch.Tensor | None = None,
                     ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Y[:, c] = Q(alphas[col_order[c]]) X[:, c] straight from the resident stack (no operator formed).

        alphas: float64 cuda tensor (capturable) or host sequence; col_order: int32 cuda tensor or
        host sequence; X: cuda [N, ldx] float32 or complex64 (the first `ncols` columns are
        transformed); out: complex64 [N, ldy] with ldy >= ncols.  Columns with a bad order are NaN.
        """
        dev = self.device
        tmps = []
        if not isinstance(alphas, torch.Tensor) or not alphas.is_cuda:
            alphas = torch.from_numpy(_alphas(alphas)).to(dev)
            tmps.append(alphas)
        if not isinstance(col_order, torch.Tensor) or not col_order.is_cuda:
            col_order = torch.as_tensor(np.asarray(col_order, dtype=np.int32)).to(dev)
            tmps.append(col_order)
        _on_device(dev, alphas=alphas, col_order=col_order, X=X, out=out)
        if alphas.dtype != torch.float64 or not alphas.is_contiguous():
            raise ValueError("alphas must be a contiguous float64 tensor")
        if col_order.dtype != torch.int32 or not col_order.is_contiguous():
            raise ValueError("col_order must be a contiguous int32 tensor")
        if X.dim() != 2 or X.shape[0] != self.N or not X.is_cuda or not X.is_contiguous():
            raise ValueError(f"X must be a contiguous cuda tensor of shape [{self.N}, ldx]")
        if X.dtype == torch.float32:
            xc = 0
        elif X.dtype == torch.complex64:
            xc = 1
        else:
            raise TypeError("X must be float32 or complex64")
        ldx = X.shape[1]
        ncols = ldx if ncols is None else int(ncols)
        if col_order.numel() < ncols:
            raise ValueError("col_order must have at least ncols entries")
        if out is None:
            out = torch.empty((self.N, max(ncols, 1)), dtype=torch.complex64, device=dev)
        if out.dim() != 2 or out.shape[0] != self.N or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex64 tensor of shape [{self.N}, ldy]")
        L_ = lib()
        ws, tmp = _caller_ws(ws, L_.fgfrft_apply_direct_workspace_bytes(self._h, ncols, ldx), dev)
        tmps.append(tmp)
        check(L_.fgfrft_apply_direct(self._h, _ptr(alphas), alphas.numel(), _ptr(col_order), _ptr(X), xc, ncols, ldx,
                                     _ptr(out), out.shape[1], _ptr(ws), ws.numel(), _stream(stream)),
              "fgfrft_apply_direct")
        _keep(stream, *tmps)
        return out

    def direct_workspace_bytes(self, ncols: int, ldx: int) -> int:
        return int(lib().fgfrft_apply_direct_workspace_bytes(self._h, ncols, ldx))

    def grad(self, alphas, X: torch.Tensor, GY: torch.Tensor, want_dX: bool = True, stream=None):
        """(dl/dalpha as float64 numpy array, dl/dX or None) for GY = dl/dRe Y + j dl/dIm Y."""
        a = _alphas(alphas)
        n = a.size
        x_shared = X.dim() == 2
        B = X.shape[-1]
        xc = _check_signal(X, n, self.N, x_shared, self.device)
        _on_device(self.device, GY=GY)
        if GY.dtype != torch.complex64 or not GY.is_contiguous() or tuple(GY.shape) != (n, self.N, B):
            raise ValueError("GY must be contiguous complex64 [n_alpha, N, B]")
        dX = torch.empty_like(X) if want_dX else None
        dal = np.zeros(n, dtype=np.float64)
        L_ = lib()
        ws = _workspace(L_.fgfrft_grad_workspace_bytes(self._h, n, B, int(x_shared)), self.device)
        check(L_.fgfrft_grad(self._h, a.ctypes.data_as(P_double), n, _ptr(X), xc, int(x_shared), B, _ptr(GY),
                             dal.ctypes.data_as(P_double), _ptr(dX) if dX is not None else None, _ptr(ws),
                             ws.numel(), _stream(stream)), "fgfrft_grad")
        _keep(stream, ws)
        return dal, dX


def _check_signal(X: torch.Tensor, n: int, N: int, x_shared: bool, dev) -> int:
    _on_device(dev, X=X)
    if not X.is_contiguous():
        raise ValueError("X must be a contiguous cuda tensor")
    if X.dtype == torch.float32:
        xc = 0
    elif X.dtype == torch.complex64:
        xc = 1
    else:
        raise TypeError("X must be float32 or complex64")
    if x_shared:
        if X.shape[0] != N:
            raise ValueError("shared X must be [N, B]")
    elif X.dim() != 3 or X.shape[0] != n or X.shape[1] != N:
        raise ValueError("X must be [n_alpha, N, B] or [N, B]")
    return xc


def apply_operator(Q: torch.Tensor, X: torch.Tensor, adjoint: bool = False, y_real: bool = False,
                   out: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Y[a] = op(Q[a]) X[a] for a complex64 operator batch Q [n, N, N]."""
    if not Q.is_cuda:
        raise ValueError("Q must be a cuda tensor")
    if Q.dtype != torch.complex64 or not Q.is_contiguous() or Q.dim() != 3 or Q.shape[1] != Q.shape[2]:
        raise ValueError("Q must be contiguous complex64 [n, N, N]")
    n, N, _ = Q.shape
    x_shared = X.dim() == 2
    B = X.shape[-1]
    xc = _check_signal(X, n, N, x_shared, Q.device)
    _on_device(Q.device, out=out)
    ydt = torch.float32 if y_real else torch.complex64
    if out is None:
        Y = torch.empty((n, N, B), dtype=ydt, device=Q.device)
    else:
        if out.dtype != ydt or not out.is_contiguous() or tuple(out.shape) != (n, N, B):
            raise ValueError("out has the wrong dtype, shape or layout")
        Y = out
    L_ = lib()
    ws, tmp = _caller_ws(ws, L_.fgfrft_apply_operator_workspace_bytes(N, n, B, int(x_shared)), Q.device)
    check(L_.fgfrft_apply_operator(_ptr(Q), N, n, int(adjoint), _ptr(X), xc, int(x_shared), B, _ptr(Y), int(y_real),
                                   _ptr(ws), ws.numel(), _stream(stream)), "fgfrft_apply_operator")
    _keep(stream, tmp)
    return Y


def gfrft_exact(V: torch.Tensor, Vh: torch.Tensor, theta: torch.Tensor, alpha: float,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Exact GFRFT from a cached eigendecomposition: V diag(e^{j alpha theta}) V^H (complex128)."""
    for t, name in ((V, "V"), (Vh, "Vh")):
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
            raise ValueError(f"{name} must be a contiguous complex128 cuda matrix")
    N = V.shape[0]
    if tuple(V.shape) != (N, N) or tuple(Vh.shape) != (N, N):
        raise ValueError("V and Vh must be N x N")
    _on_device(V.device, Vh=Vh, theta=theta, out=out)
    if theta.dtype != torch.float64 or theta.numel() != N or not theta.is_contiguous():
        raise ValueError("theta must be a contiguous float64 cuda vector of length N")
    if out is None:
        out = torch.empty((N, N), dtype=torch.complex128, device=V.device)
    if out.dtype != torch.complex128 or not out.is_contiguous() or tuple(out.shape) != (N, N):
        raise ValueError("out must be a contiguous complex128 N x N tensor")
    L_ = lib()
    ws = _workspace(L_.fgfrft_gfrft_exact_workspace_bytes(N), V.device)
    check(L_.fgfrft_gfrft_exact(_ptr(V), _ptr(Vh), _ptr(theta), N, float(alpha), _ptr(out), _ptr(ws),
                                ws.numel(), _stream(stream)), "fgfrft_gfrft_exact")
    _keep(stream, ws)
    return out
