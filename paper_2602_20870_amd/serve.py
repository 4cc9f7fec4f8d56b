"""Continuous-batching server for FGFRFT requests over resident plans (one GPU).

A request is (graph id, order alpha, signal block X [N, B]).  The server keeps one
plan per graph resident in HBM (admitted only if its footprint fits the budget) and,
per plan, S slot sets: static device buffers for up to K orders (orders, signals,
operators, outputs, workspaces) plus pinned host staging.  Each scheduling step
  * admits arrived requests into the pending queue,
  * retires finished batches (event query), hands results to their futures and
    frees their slot set,
  * for every plan with pending requests and a free slot set, coalesces up to K of
    its requests into one batch and runs it on the slot set's stream (one stream per hardware
    queue; plans are grouped on them by size, so small plans do not queue behind large ones;
    batches on different queues overlap on the device), replayed from a captured hipGraph for the
    batch's size bucket, by one of two routes:
      - operator route: one fused operator-update launch for all the batch's orders
        followed by one apply launch (moves 16 N^2 bytes of operator per order);
      - direct route: the signals of the batch side by side, one column per signal
        with its own order, transformed straight from the resident stack (moves the
        (2L+1) N^2 stack elements once per 64 columns, no operator formed).
    The route is chosen per batch from the number of orders and of signal columns.
Requests that arrive while batches run wait only until a slot set of their plan is
free, not until the whole device drains.  Within one route a request's result does
not depend on the other requests of its batch (bitwise, tested); the two routes agree
to the parity bound.
"""
from __future__ import annotations

import collections
import gc
import os
import time
from concurrent.futures import Future

import numpy as np
import torch

from .ops import Plan, apply_operator

BUCKETS = (1, 2, 4, 8, 16, 32)
DIRECT_BLOCKS = 4          # the direct route takes batches of up to 4 x 64 signal columns
ROUTES = ("auto", "operator", "direct")


def prefer_direct(n_orders: int, n_blocks: int, L: int, real_route: bool = False) -> bool:
    """Route choice for one batch, in units of the operator route's stack stream S (its update
    reads the 2L resident matrices): the operator route costs S plus 16 N^2 bytes (write and read
    of one complex64 operator) per order, 4 / (2L+1) of S each, or 8 N^2 bytes (2 / (2L+1) of S) on
    the real-F route, which writes and reads only R = Re Q; the direct route costs about 0.85 S for
    the first 64-column block and about 0.6 S for each further one (measured at N = 4096, L = 32).
    Direct iff 0.6 (blocks - 1) < c n_orders / (2L+1) with c = 4 or 2, slightly conservative."""
    c = 2 if real_route else 4
    return n_blocks <= DIRECT_BLOCKS and 0.6 * (n_blocks - 1) * (2 * L + 1) < c * n_orders


def _distinct_queue_streams(n: int, device) -> list:
    """Up to n streams that run on different hardware queues.  Which queue a stream lands on is up
    to the runtime (and to what the process did before), so candidates are tested: a candidate is
    kept when a tiny command on it completes while a spin of about 10 ms on each stream kept so far
    is still running.  If fewer than n pass, the rest are filled with untested candidates."""
    cands = [torch.cuda.Stream(device=device) for _ in range(4 * n)]
    if not hasattr(torch.cuda, "_sleep"):      # no spin kernel in this torch build: untested streams
        return cands[:n]
    t = torch.zeros(1, device=device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(cands[0]):          # calibrate the spin: cycles per millisecond
        e0.record(cands[0])
        torch.cuda._sleep(1 << 20)
        e1.record(cands[0])
    e1.synchronize()
    per_ms = (1 << 20) / max(e0.elapsed_time(e1), 1e-3)
    cycles = int(min(max(10.0 * per_ms, 1 << 16), 32 << 20))   # at most 32x the calibration spin

    def apart(a, b) -> bool:
        ea, eb = torch.cuda.Event(), torch.cuda.Event()
        with torch.cuda.stream(a):
            torch.cuda._sleep(cycles)
            ea.record(a)
        with torch.cuda.stream(b):
            t.add_(1)
            eb.record(b)
        eb.synchronize()
        ok = not ea.query()
        ea.synchronize()
        return ok

    chosen = []
    for c in cands:
        if len(chosen) == n:
            break
        if all(apart(k, c) for k in chosen):
            chosen.append(c)
    rest = [c for c in cands if all(c is not k for k in chosen)]
    torch.cuda.synchronize(device)
    return chosen + rest[: n - len(chosen)]


class AdmissionError(RuntimeError):
    """A plan does not fit the server's HBM budget."""


def _direct_blocks(plan, route: str) -> range:
    """Direct-route block counts a slot set offers.  Only plans the matrix-core direct kernel takes
    (real F, N % 32 == 0) offer the route; the plain kernel of the other configurations is far slower
    than the operator route."""
    if route != "operator" and not plan.complex and plan.N % 32 == 0:
        return range(1, DIRECT_BLOCKS + 1)
    return range(0)


class _SlotSet:
    @staticmethod
    def device_bytes(plan, K: int, bmax: int, route: str) -> int:
        """Device bytes one slot set of `plan` allocates (the constructor checks its tensors add up to
        exactly this)."""
        from ._lib import lib
        N = plan.N
        b = K * 8 + K * N * bmax * 4 + K * N * bmax * 8      # orders, X, Y
        b += max(256, plan.apply_dev_workspace_bytes(K, bmax))  # the operators and their workspaces
        nbs = _direct_blocks(plan, route)
        b += sum(N * 64 * nb * 4 + 64 * nb * 4 + N * 64 * nb * 8 for nb in nbs)   # dX, dcols, dY
        b += max([256] + [plan.direct_workspace_bytes(64 * nb, 64 * nb) for nb in nbs])
        return b

    def __init__(self, plan: Plan, K: int, bmax: int, device, use_graphs: bool, route: str = "auto", stream=None):
        N = plan.N
        self.K, self.bmax, self.route = K, bmax, route
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.alphas = torch.zeros(K, dtype=torch.float64, device=device)
        self.X = torch.zeros((K, N, bmax), dtype=torch.float32, device=device)
        self.Y = torch.empty((K, N, bmax), dtype=torch.complex64, device=device)
        # operator route: fgfrft_apply_dev (the real-F route when the plan offers it: R = Re Q in the
        # workspace, half the bytes of a complex64 operator), one workspace for every bucket
        self.ows = torch.empty(max(256, plan.apply_dev_workspace_bytes(K, bmax)), dtype=torch.uint8, device=device)
        self.real_route = (not plan.complex and plan.r_minus1 <= 32 and N % 32 == 0 and bmax % 64 == 0)
        self.h_alphas = torch.zeros(K, dtype=torch.float64).pin_memory()
        self.h_X = torch.zeros((K, N, bmax), dtype=torch.float32).pin_memory()
        self.h_Y = torch.empty((K, N, bmax), dtype=torch.complex64).pin_memory()
        # direct route: per block count nb, signals [N, 64 nb] side by side, column -> order index
        self.dblocks = _direct_blocks(plan, route)
        self.dX = {nb: torch.zeros((N, 64 * nb), dtype=torch.float32, device=device) for nb in self.dblocks}
        self.dcols = {nb: torch.zeros(64 * nb, dtype=torch.int32, device=device) for nb in self.dblocks}
        self.dY = {nb: torch.empty((N, 64 * nb), dtype=torch.complex64, device=device) for nb in self.dblocks}
        self.dws = torch.empty(max([256] + [plan.direct_workspace_bytes(64 * nb, 64 * nb) for nb in self.dblocks]),
                               dtype=torch.uint8, device=device)
        self.h_dX = {nb: torch.zeros((N, 64 * nb), dtype=torch.float32).pin_memory() for nb in self.dblocks}
        self.h_dcols = {nb: torch.zeros(64 * nb, dtype=torch.int32).pin_memory() for nb in self.dblocks}
        self.h_dY = {nb: torch.empty((N, 64 * nb), dtype=torch.complex64).pin_memory() for nb in self.dblocks}
        # NumPy views of the pinned staging: the scheduling loop packs and unpacks with single-threaded
        # NumPy copies (torch's host copies fan out to its thread pool, whose wake-ups stall the loop)
        self.n_alphas, self.n_X, self.n_Y = self.h_alphas.numpy(), self.h_X.numpy(), self.h_Y.numpy()
        self.n_dX = {nb: t.numpy() for nb, t in self.h_dX.items()}
        self.n_dcols = {nb: t.numpy() for nb, t in self.h_dcols.items()}
        self.n_dY = {nb: t.numpy() for nb, t in self.h_dY.items()}
        self.event = torch.cuda.Event()   # recorded after each batch (one event reused)
        self.taken = None          # (route, bucket, column offsets) of the batch in flight
        self.plan = plan
        self.graphs = {}
        self.batch = None
        if self.nbytes() != _SlotSet.device_bytes(plan, K, bmax, route):
            raise AssertionError("slot-set byte count out of step with its allocation")
        if use_graphs:
            self._capture()

    def _run(self, key):
        route, k = key
        if route == "direct":
            self.plan.apply_direct(self.alphas, self.dcols[k], self.dX[k], out=self.dY[k], ws=self.dws)
        else:
            self.plan.apply_dev(self.alphas[:k], self.X[:k], out=self.Y[:k], ws=self.ows)

    def _keys(self):
        return [("operator", k) for k in BUCKETS if k <= self.K] + [("direct", nb) for nb in self.dblocks]

    def _capture(self):
        with torch.cuda.stream(self.stream):
            for key in self._keys():
                self._run(key)       # eager warm-up (kernel attributes, code objects)
        self.stream.synchronize()
        for key in self._keys():
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self._run(key)
            self.graphs[key] = g
        self.stream.synchronize()

    def nbytes(self) -> int:
        ts = [self.alphas, self.X, self.Y, self.ows, self.dws]
        ts += list(self.dX.values()) + list(self.dcols.values()) + list(self.dY.values())
        return sum(t.numel() * t.element_size() for t in ts)

    def choose(self, batch) -> tuple:
        ncols = sum(r.B for r in batch)
        nb = -(-ncols // 64)
        if self.dblocks and nb <= DIRECT_BLOCKS and (
                self.route == "direct" or prefer_direct(len(batch), nb, self.plan.L, self.real_route)):
            return ("direct", nb)
        k = next(b for b in BUCKETS if b >= len(batch)) if self.graphs else len(batch)
        return ("operator", k)

    def launch(self, batch):
        n = len(batch)
        t = time.perf_counter()
        for r in batch:
            r.t_launch, r.batch_size = t, n
        route, k = key = self.choose(batch)
        # padding orders get alpha = 0 (a valid order); padding rows and signal columns are left
        # as they are: every order's plane and every signal column is computed independently
        # (per-column scales), and padded outputs are never returned
        self.n_alphas[n:] = 0.0
        offs = []
        if route == "direct":
            hx, hc, off = self.n_dX[k], self.n_dcols[k], 0
            hc[:] = 0
            for i, r in enumerate(batch):
                self.n_alphas[i] = r.alpha
                hx[:, off: off + r.B] = r.X
                hc[off: off + r.B] = i
                offs.append(off)
                off += r.B
        else:
            for i, r in enumerate(batch):
                self.n_alphas[i] = r.alpha
                self.n_X[i, :, : r.B] = r.X
        with torch.cuda.stream(self.stream):
            self.alphas.copy_(self.h_alphas, non_blocking=True)
            if route == "direct":
                self.dcols[k].copy_(self.h_dcols[k], non_blocking=True)
                self.dX[k].copy_(self.h_dX[k], non_blocking=True)
            else:
                self.X[:k].copy_(self.h_X[:k], non_blocking=True)
            if self.graphs:
                self.graphs[key].replay()
            else:
                self._run(key)
            if route == "direct":
                self.h_dY[k].copy_(self.dY[k], non_blocking=True)
            else:
                self.h_Y[:n].copy_(self.Y[:n], non_blocking=True)
            self.event.record(self.stream)
        self.batch, self.taken = batch, (route, k, offs)

    def done(self) -> bool:
        return self.batch is not None and self.event.query()

    def retire(self, now: float):
        route, k, offs = self.taken
        for i, r in enumerate(self.batch):
            r.t_done, r.route = now, route
            if route == "direct":
                y = self.n_dY[k][:, offs[i]: offs[i] + r.B].copy()
            else:
                y = self.n_Y[i, :, : r.B].copy()
            r.future.set_result(y)
            r.future = None    # the result now belongs to the caller's future alone
        self.batch = self.taken = None


class _Request:
    __slots__ = ("gid", "alpha", "X", "B", "t_arrive", "t_launch", "t_done", "batch_size", "future", "route")

    def __init__(self, gid, alpha, X, t_arrive):
        self.gid, self.alpha = gid, float(alpha)
        self.X = np.asarray(X, dtype=np.float32)
        self.B = self.X.shape[1] if self.X.ndim == 2 else 0
        self.t_arrive, self.t_launch, self.t_done, self.batch_size = t_arrive, None, None, 0
        self.future, self.route = Future(), None


class Server:
    """Continuous-batching FGFRFT server over resident plans.

    hbm_budget: bytes of device memory the server may hold (plans + slot sets).
    K: orders per batch (one fused update launch); bmax: largest signal block;
    slot_sets: batches of one plan that may be in flight at once;
    route: "auto" (per batch, prefer_direct), "operator" or "direct" (when the batch's
    signals fit DIRECT_BLOCKS x 64 columns, else the operator route).  The direct route is
    offered for plans of real F with N % 32 == 0 (the matrix-core direct kernel).
    stacktype: storage of the plans' stacks, "fp16x2" (default: the FP32 stack's split operands,
    the same results bit for bit with no split work in the direct kernel) or "fp32".
    """

    def __init__(self, hbm_budget: int, K: int = 16, bmax: int = 64, slot_sets: int = 2, use_graphs: bool = True,
                 device: str = "cuda:0", route: str = "auto", stacktype: str = "fp16x2"):
        if route not in ROUTES:
            raise ValueError(f"route must be one of {ROUTES}")
        if stacktype not in ("fp32", "fp16x2"):
            raise ValueError("stacktype must be fp32 or fp16x2 (the same results bit for bit)")
        self.stacktype = stacktype
        self.budget, self.used = int(hbm_budget), 0
        self.K, self.bmax, self.S, self.route = K, bmax, slot_sets, route
        self.use_graphs = use_graphs
        self.device = torch.device(device)
        self.plans = {}
        self.slots = {}
        self.pending = collections.defaultdict(collections.deque)
        self.inflight = 0
        # one stream per hardware queue of the device (a queue runs its commands in order), chosen by
        # test on first admission
        self.n_queues = max(1, int(os.environ.get("GPU_MAX_HW_QUEUES", "4")))
        self.streams = []

    # ------------------------------------------------------------------ admission
    def footprint(self, N: int, L: int, complex_F: bool = False) -> int:
        """Device bytes of a plan before it exists: its resident stack and projector (exact) plus the
        operators, signal blocks and direct-route blocks of its S slot sets.  Their workspaces depend
        on the plan and are added at admission, once it exists; the FP64 scratch of the offline
        stage is released when planning ends and is not counted."""
        from ._lib import lib
        import ctypes
        pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        if lib().fgfrft_plan_bytes(N, L, 0 if complex_F else 1, 0, ctypes.byref(pb), ctypes.byref(sb)) != 0:
            raise ValueError(f"no plan for N={N}, L={L}: {lib().fgfrft_last_error().decode()}")
        per_set = self.K * N * N * 8 + self.K * N * self.bmax * (4 + 8)
        if self.route != "operator" and not complex_F and N % 32 == 0:   # direct-route blocks (1..4 x 64 columns)
            per_set += 10 * 64 * N * (4 + 8)
        return int(pb.value) + self.S * per_set

    def add_plan(self, gid, F: np.ndarray, L: int) -> None:
        """Make graph `gid` resident; raises AdmissionError if it does not fit the budget.  The check
        runs twice: on the footprint before anything is allocated, then on the exact bytes (stack,
        projector and every slot-set tensor) once the plan exists, before its slot sets are made."""
        F = np.asarray(F)
        cplx = np.iscomplexobj(F)
        N = F.shape[0]
        left = self.budget - self.used
        est = self.footprint(N, L, cplx)
        if est > left:
            raise AdmissionError(f"plan {gid} (N={N}, L={L}) needs {est / 1e9:.2f} GB; {left / 1e9:.2f} GB left")
        if not self.streams:
            self.streams = _distinct_queue_streams(self.n_queues, self.device)
        F = np.ascontiguousarray(F, dtype=np.complex128 if cplx else np.float64)
        plan = Plan(torch.from_numpy(F).to(self.device), L, stacktype=self.stacktype)
        need = plan.persistent.numel() + self.S * _SlotSet.device_bytes(plan, self.K, self.bmax, self.route)
        if need > left:
            del plan
            raise AdmissionError(f"plan {gid} (N={N}, L={L}) needs {need / 1e9:.2f} GB; {left / 1e9:.2f} GB left")
        sets = [_SlotSet(plan, self.K, self.bmax, self.device, self.use_graphs, self.route, self.streams[0])
                for _ in range(self.S)]
        self.plans[gid] = plan
        self.slots[gid] = sets
        self.used += need
        self._balance()

    def _balance(self):
        """Deal the slot sets to the hardware-queue streams by size class: sorted by the stack a
        launch streams (N^2 (2L+1)), the slot sets are cut into as many consecutive groups of equal
        count as there are streams, one group per stream, so plans of similar cost share a queue.  A
        queue runs its commands in order, so a small plan's batch that shares a queue with a large plan
        waits behind the large plan's launches (measured: N = 1024 requests at p50 2.0 ms behind
        N = 4096 batches for 0.1 ms of work of their own), while plans of similar size cost each other
        about their own service time.  (Giving each large plan a queue of its own and packing the small
        ones onto the rest measured worse: trace p50 1.5 against 1.1 ms.)  A slot set only launches
        after its previous batch has completed, so moving it to another stream needs no
        synchronisation."""
        units = [(p.N * p.N * (2 * p.L + 1), gid, j) for gid, p in self.plans.items()
                 for j in range(len(self.slots[gid]))]
        units.sort(key=lambda u: -u[0])
        nq = len(self.streams)
        for i, (_, gid, j) in enumerate(units):
            self.slots[gid][j].stream = self.streams[min(nq - 1, i * nq // len(units))]

    # ------------------------------------------------------------------ requests
    def submit(self, gid, alpha: float, X, t_arrive: float | None = None) -> Future:
        if gid not in self.plans:
            raise KeyError(f"graph {gid} is not resident")
        plan = self.plans[gid]
        if not abs(alpha) < plan.L:
            raise ValueError(f"order {alpha} outside (-L, L)")
        if np.iscomplexobj(X):
            raise TypeError("the server takes real signal blocks (float32)")
        r = _Request(gid, alpha, X, time.perf_counter() if t_arrive is None else t_arrive)
        if r.X.ndim != 2 or r.X.shape[0] != plan.N or not 1 <= r.B <= self.bmax:
            raise ValueError("X must be [N, B] with 1 <= B <= bmax")
        self.pending[gid].append(r)
        return r.future

    def step(self) -> int:
        """Retire finished batches and launch new ones; returns the number of batches launched."""
        now = time.perf_counter()
        for sets in self.slots.values():
            for s in sets:
                if s.done():
                    s.retire(now)
                    self.inflight -= 1
        launched = 0
        for gid, q in self.pending.items():
            while q:
                free = next((s for s in self.slots[gid] if s.batch is None), None)
                if free is None:
                    break
                batch = [q.popleft() for _ in range(min(self.K, len(q)))]
                free.launch(batch)
                self.inflight += 1
                launched += 1
        return launched

    def busy(self) -> bool:
        return self.inflight > 0 or any(self.pending.values())

    def drain(self):
        while self.busy():
            if not self.step():
                time.sleep(20e-6)


# ---------------------------------------------------------------------- workload driver
def poisson_trace(n: int, rate: float, gids, B_max: int, seed: int = 0):
    """Arrival times (s), graph ids (uniform), orders U[-2, 2], block sizes U{1..B_max}."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    g = rng.integers(0, len(gids), size=n)
    a = rng.uniform(-2.0, 2.0, size=n)
    b = rng.integers(1, B_max + 1, size=n)
    return t, [gids[i] for i in g], a, b


def run_trace(server: Server, trace, signals: dict, warmup: int = 0, keep_every: int = 1) -> dict:
    """Replay a trace in real time; latency = completion - arrival per request.

    The client keeps the result of every `keep_every`-th request (returned as `kept`:
    (trace index, future) pairs) and drops the others once they complete, as a client that
    consumes its results would: holding every result of a long trace (gigabytes of host
    arrays) makes each new result array fresh, page-faulted memory.  The cyclic garbage
    collector is paused during the replay: its collections over the trace's many request
    objects otherwise stall the scheduling loop for tens of milliseconds.  While batches are in
    flight the loop polls without sleeping (one host core busy)."""
    gc_was = gc.isenabled()
    gc.disable()
    try:
        return _run_trace(server, trace, signals, warmup, keep_every)
    finally:
        if gc_was:
            gc.enable()


def _run_trace(server: Server, trace, signals: dict, warmup: int, keep_every: int) -> dict:
    t_arr, gids, alphas, Bs = trace
    kept, reqs = [], []
    t0 = time.perf_counter()
    i, n = 0, len(t_arr)
    while i < n or server.busy():
        now = time.perf_counter() - t0
        while i < n and t_arr[i] <= now:
            X = signals[gids[i]][:, : Bs[i]]
            fut = server.submit(gids[i], alphas[i], X, t_arrive=t0 + t_arr[i])
            if i % keep_every == 0:
                kept.append((i, fut))
            reqs.append(server.pending[gids[i]][-1])
            i += 1
        if not server.step() and server.inflight == 0:
            # nothing running: sleep until the next arrival (at most 200 us); while batches run the
            # loop polls their events again at once, so a completion is retired without a sleep's delay
            nxt = t_arr[i] - (time.perf_counter() - t0) if i < n else 20e-6
            time.sleep(max(0.0, min(nxt, 200e-6)))
    wall = time.perf_counter() - t0
    rs = reqs[warmup:]
    direct_share = float(np.mean([r.route == "direct" for r in rs]))
    lat = np.array([r.t_done - r.t_arrive for r in rs])
    per_plan = {}
    for gid in sorted(set(r.gid for r in rs), key=str):
        lg = np.array([r.t_done - r.t_arrive for r in rs if r.gid == gid])
        per_plan[str(gid)] = dict(N=server.plans[gid].N, requests=len(lg), p50_ms=float(np.percentile(lg, 50) * 1e3),
                                  p99_ms=float(np.percentile(lg, 99) * 1e3))
    wait = np.array([r.t_launch - r.t_arrive for r in rs])
    service = np.array([r.t_done - r.t_launch for r in rs])
    return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), requests=len(lat), wall_s=wall,
                throughput_req_s=len(reqs) / wall,
                queue_wait_p50_ms=float(np.percentile(wait, 50) * 1e3),
                queue_wait_p99_ms=float(np.percentile(wait, 99) * 1e3),
                service_p50_ms=float(np.percentile(service, 50) * 1e3),
                service_p99_ms=float(np.percentile(service, 99) * 1e3),
                mean_batch=float(np.mean([r.batch_size for r in rs])), direct_share=direct_share, per_plan=per_plan,
                kept=kept)


def run_trace_one_launch(plans: dict, trace, signals: dict, warmup: int = 0, keep_every: int = 1, bmax: int = 64,
                         route: str = "auto", use_graphs: bool = True, device: str = "cuda:0") -> dict:
    """Baseline without coalescing or overlap: one launch per request, in arrival order, on the route
    the server picks for a batch of one (the direct route where the plan offers it), from buffers
    allocated once per plan (a slot set of one order, replayed from its captured graph), with only the
    result copy waited for.  Latency = completion - arrival.  `outputs`: index -> result of every
    `keep_every`-th request."""
    gc_was = gc.isenabled()
    gc.disable()
    try:
        dev = torch.device(device)
        stream = torch.cuda.Stream(device=dev)
        sets = {gid: _SlotSet(p, 1, bmax, dev, use_graphs, route, stream) for gid, p in plans.items()}
        t_arr, gids, alphas, Bs = trace
        t0 = time.perf_counter()
        lat, service, routes, outs = [], [], [], {}
        for i in range(len(t_arr)):
            now = time.perf_counter() - t0
            if t_arr[i] > now:
                time.sleep(t_arr[i] - now)
            r = _Request(gids[i], alphas[i], signals[gids[i]][:, : Bs[i]], t0 + t_arr[i])
            fut = r.future
            s = sets[gids[i]]
            s.launch([r])
            s.event.synchronize()
            s.retire(time.perf_counter())
            lat.append(r.t_done - r.t_arrive)
            service.append(r.t_done - r.t_launch)
            routes.append(r.route)
            if i % keep_every == 0:
                outs[i] = fut.result()
        wall = time.perf_counter() - t0
    finally:
        if gc_was:
            gc.enable()
    lat = np.array(lat[warmup:])
    service = np.array(service[warmup:])
    return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), requests=len(lat), wall_s=wall,
                throughput_req_s=len(t_arr) / wall, service_mean_ms=float(service.mean() * 1e3),
                service_p99_ms=float(np.percentile(service, 99) * 1e3),
                direct_share=float(np.mean([x == "direct" for x in routes[warmup:]])), outputs=outs)


def run_trace_per_request(plans: dict, trace, signals: dict, warmup: int = 0, keep_every: int = 1) -> dict:
    """Baseline: one update launch and one apply launch per request, in arrival order; keeps
    the results and pauses the garbage collector as run_trace does (`outputs`: index -> result)."""
    gc_was = gc.isenabled()
    gc.disable()
    try:
        return _run_trace_per_request(plans, trace, signals, warmup, keep_every)
    finally:
        if gc_was:
            gc.enable()


def _run_trace_per_request(plans: dict, trace, signals: dict, warmup: int, keep_every: int) -> dict:
    t_arr, gids, alphas, Bs = trace
    t0 = time.perf_counter()
    lat = []
    dev = next(iter(plans.values())).device
    outs = {}
    for i in range(len(t_arr)):
        now = time.perf_counter() - t0
        if t_arr[i] > now:
            time.sleep(t_arr[i] - now)
        p = plans[gids[i]]
        X = torch.from_numpy(np.ascontiguousarray(signals[gids[i]][:, : Bs[i]], dtype=np.float32)).to(dev)[None]
        Q = p.update([alphas[i]])
        Y = apply_operator(Q, X)
        y = Y[0].cpu().numpy()
        if i % keep_every == 0:
            outs[i] = y
        lat.append(time.perf_counter() - t0 - t_arr[i])
    wall = time.perf_counter() - t0
    lat = np.array(lat[warmup:])
    return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), requests=len(lat), wall_s=wall,
                throughput_req_s=len(t_arr) / wall, outputs=outs)
