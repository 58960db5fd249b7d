"""Serving many plain-optimiser solves of uneven hologram sizes on one GPU.

Each request is one hologram: its SLM size, its Gaussians (n = pixels / 5,
one colour), its target intensity, a wavelength and a propagation distance.
A solve is a fixed number of Adam steps of L_MSE (Alg. 1).

* Shape classes: requests of one (H, W) share the context layout (FFT plans,
  tile grid, buffer sizes), so they share *slots*.  A slot is one context of a
  class on one stream with its input and output buffers and its solve
  captured once as a HIP graph (binding.Solve over cgh_solve_*).
* Serving a request on a slot enqueues, on the slot's stream and without a
  host synchronisation: copies of the request's parameters and target into
  the slot, cgh_set_optics for the request's (lambda, z), one graph launch,
  and copies of the optimised parameters and loss log out.  Requests on one
  stream run in order; streams run concurrently.
* Scheduling: longest-processing-time-first assignment of the requests to the
  streams (balances the streams' total work), then each stream runs its
  queue shortest first (lowers the mean latency without changing the
  stream's total).  The cost of a request is the measured solve time of its
  class when known, else its pixel count.
* ``autotune`` times the batch at each candidate stream count and keeps the
  fastest.

All device work is the library's kernels; this module only owns buffers,
streams and the order of the calls.
"""
import time

import numpy as np
import torch

from . import binding, synth

WAVELENGTHS = (639e-9, 515e-9, 473e-9)
SIZES = ((512, 512), (768, 1024), (1024, 1024), (1080, 1920), (2048, 2048))
PITCH = 8e-6


class Request:
    """One hologram to solve; ``params`` and ``target`` are device tensors."""

    def __init__(self, index, H, W, n, params, target, wavelength, z):
        self.index, self.H, self.W, self.n = index, H, W, n
        self.params, self.target = params, target
        self.wavelength, self.z = wavelength, z
        self.out_params = None
        self.out_loss = None

    @property
    def pixels(self):
        return self.H * self.W


def make_requests(count, seed=300, sizes=SIZES, density=5, zrange=(2e-3, 10e-3), device="cuda"):
    """Seeded synthetic batch: size uniform over ``sizes``, n = H W // density
    Gaussians of one colour (the synthetic parameter distribution), wavelength
    uniform over the three colours, z uniform in ``zrange``.  Each size class
    has one synthetic target; a request uses it circularly shifted by a
    seeded random offset, so every target differs at the cost of one
    generation per class."""
    rng = np.random.default_rng(seed)
    base = {}
    out = []
    for i in range(count):
        k = int(rng.integers(len(sizes)))
        H, W = sizes[k]
        if k not in base:
            base[k] = synth.target(seed + 1 + k, 1, H, W)
        n = H * W // density
        p = binding.pack(synth.params(seed + 100 + i, n, H, W, 1), device=device)
        dy, dx = int(rng.integers(H)), int(rng.integers(W))
        T = torch.from_numpy(np.ascontiguousarray(np.roll(base[k], (dy, dx), axis=(-2, -1))))
        lam = WAVELENGTHS[int(rng.integers(len(WAVELENGTHS)))]
        z = float(rng.uniform(*zrange))
        out.append(Request(i, H, W, n, p, T.to(device), lam, z))
    return out


def plan(requests, streams, cost):
    """Longest-processing-time-first assignment of ``requests`` to ``streams``
    queues by ``cost(request)`` (ties: lower index first, then the lower
    stream), then each queue sorted shortest first.  Returns the queues."""
    load = [0.0] * streams
    queues = [[] for _ in range(streams)]
    for r in sorted(requests, key=lambda r: (-cost(r), r.index)):
        si = min(range(streams), key=lambda i: (load[i], i))
        load[si] += cost(r)
        queues[si].append(r)
    for q in queues:
        q.sort(key=lambda r: (cost(r), r.index))
    return queues


class Slot:
    """A context of one shape class on one stream, with its captured solve."""

    def __init__(self, H, W, n, steps, lr, stream, pitch, device):
        self.H, self.W, self.n = H, W, n
        self.stream = stream
        self.ctx = binding.Context(H, W, 1, pitch, [WAVELENGTHS[1]], [5e-3], max_gaussians=n)
        self.params = torch.zeros(binding.param_count(n, 1), dtype=torch.float32, device=device)
        self.target = torch.zeros((1, 1, H, W), dtype=torch.float32, device=device)
        self.solve = binding.Solve(self.ctx, self.params, n, self.target, steps, lr=lr,
                                   stream=stream)

    def enqueue(self, req):
        """Everything for one request on this slot's stream (no host wait)."""
        s = self.stream
        with torch.cuda.stream(s):
            self.params.copy_(req.params, non_blocking=True)
            self.target.view(-1).copy_(req.target.view(-1), non_blocking=True)
            self.ctx.set_optics([req.wavelength], [req.z], stream=s)
            self.solve.launch(s)
            req.out_params.copy_(self.params, non_blocking=True)
            req.out_loss.copy_(self.solve.loss_log, non_blocking=True)


class Server:
    """Slots over up to ``max_streams`` streams; ``run`` serves a batch."""

    def __init__(self, steps, lr=1e-3, max_streams=4, pitch=PITCH, device="cuda"):
        self.steps, self.lr, self.pitch, self.device = steps, lr, pitch, device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max_streams)]
        self.slots = {}
        self.class_cost = {}

    def slot(self, si, H, W, n):
        key = (si, H, W)
        if key not in self.slots:
            self.slots[key] = Slot(H, W, n, self.steps, self.lr, self.streams[si], self.pitch,
                                   self.device)
        s = self.slots[key]
        if s.n != n:
            raise ValueError(f"class {H}x{W} holds n = {s.n}, request has n = {n}")
        return s

    def cost(self, req):
        return self.class_cost.get((req.H, req.W), float(req.pixels))

    def plan(self, requests, streams):
        return plan(requests, streams, self.cost)

    def prepare(self, requests, streams):
        """Creates the slots and output buffers a run needs (not timed)."""
        for si, q in enumerate(self.plan(requests, streams)):
            for r in q:
                self.slot(si, r.H, r.W, r.n)
        for r in requests:
            if r.out_params is None:
                r.out_params = torch.empty_like(r.params)
                r.out_loss = torch.empty((self.steps, 2), dtype=torch.float64,
                                         device=self.device)
        torch.cuda.synchronize()

    def run(self, requests, streams=None):
        """Serves ``requests`` on the first ``streams`` streams.  Returns the
        batch wall time (host clock around the whole batch, s) and per request
        the solve latency (its own span on its stream, ms) and the turnaround
        (from the batch start to its completion, ms), from HIP events."""
        streams = len(self.streams) if streams is None else streams
        queues = self.plan(requests, streams)
        self.prepare(requests, streams)
        main = torch.cuda.current_stream(self.device)
        t0 = torch.cuda.Event(enable_timing=True)
        marks = {}
        host0 = time.perf_counter()
        t0.record(main)
        for si in range(streams):
            self.streams[si].wait_event(t0)
        # round-robin over the queues so that every stream gets work early
        depth = max((len(q) for q in queues), default=0)
        for k in range(depth):
            for si, q in enumerate(queues):
                if k >= len(q):
                    continue
                r = q[k]
                slot = self.slot(si, r.H, r.W, r.n)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(slot.stream)
                slot.enqueue(r)
                e1.record(slot.stream)
                marks[r.index] = (e0, e1, si)
        for si in range(streams):
            main.wait_stream(self.streams[si])
        torch.cuda.synchronize()
        wall = time.perf_counter() - host0
        # pair-list capacity: each slot reports an overflow in any step of any
        # solve it ran since its previous status read; raises CghError
        for key in {(si, r.H, r.W) for si, q in enumerate(queues) for r in q}:
            self.slots[key].ctx.read_status()
        latency = {i: e0.elapsed_time(e1) for i, (e0, e1, _) in marks.items()}
        turnaround = {i: t0.elapsed_time(e1) for i, (_, e1, _) in marks.items()}
        return {"wall_s": wall, "latency_ms": latency, "turnaround_ms": turnaround,
                "stream_of": {i: si for i, (_, _, si) in marks.items()}}

    def measure_class_costs(self, requests):
        """Solve time of one request per class, alone on stream 0 (ms); used
        as the scheduling cost of the class."""
        seen = {}
        for r in requests:
            seen.setdefault((r.H, r.W), r)
        for key, r in seen.items():
            res = self.run([r], streams=1)
            self.class_cost[key] = res["latency_ms"][r.index]
        return dict(self.class_cost)


def summary(requests, res):
    lat = np.array([res["latency_ms"][r.index] for r in requests])
    tat = np.array([res["turnaround_ms"][r.index] for r in requests])
    return {
        "holograms": len(requests),
        "wall_s": res["wall_s"],
        "holograms_per_s": len(requests) / res["wall_s"],
        "latency_p50_ms": float(np.percentile(lat, 50)),
        "latency_p99_ms": float(np.percentile(lat, 99)),
        "turnaround_p50_ms": float(np.percentile(tat, 50)),
        "turnaround_p99_ms": float(np.percentile(tat, 99)),
    }


def autotune(server, requests, candidates=(1, 2, 4)):
    """Runs the batch at each candidate stream count (a warm-up run: slots,
    graphs and caches; then a timed run) and returns (best count,
    {count: holograms/s}, {count: the timed run's result from ``run``})."""
    rates, runs = {}, {}
    for k in candidates:
        if k > len(server.streams):
            continue
        server.run(requests, streams=k)
        runs[k] = server.run(requests, streams=k)
        rates[k] = len(requests) / runs[k]["wall_s"]
    best = max(rates, key=lambda k: (rates[k], -k))
    return best, rates, runs


def solve_eager(ctx, params, n, target, steps, lr=1e-3):
    """The same solve by one call per kernel group from the host (no graph):
    rasterize, backward and Adam per step.  Returns the loss log [steps][2]."""
    dev = params.device
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
    grads = torch.empty_like(params)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    log = torch.zeros((steps, 2), dtype=torch.float64, device=dev)
    for t in range(1, steps + 1):
        ctx.rasterize(params, n, field)
        ctx.backward(params, n, field, target, loss=log[t - 1], grads=grads)
        binding.step(params, grads, m, v, t, lr)
    return log
