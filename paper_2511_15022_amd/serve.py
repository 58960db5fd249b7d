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

``BatchServer`` instead solves all requests of a size class together: one
batched context (cgh_config.batch = B) holds B holograms of the class, each
with its own Gaussians, target, wavelength and distance, so every kernel of
a step covers the whole class in one launch (the hologram index is part of
the grid) and small classes fill the chip.  A class with more than
``max_batch`` requests is cut into batches.  ``tune_tiles`` chooses the
rasterizer tile shape of each class by timing a short captured solve of the
class batch at every supported shape; ``autotune_batched`` then picks the
stream count.  Results equal the single-hologram solves bit for bit (the
same kernels over the same tile lists; tested).

``MixedServer`` serves each class in whichever of the two modes costs less
per hologram and step (measured: the tile probe of the class batch, the
solve of one request alone), with the class batches and the single requests
as jobs spread over shared streams longest first.

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

    def __init__(self, steps, lr=1e-3, max_streams=4, pitch=PITCH, device="cuda", streams=None):
        self.steps, self.lr, self.pitch, self.device = steps, lr, pitch, device
        self.streams = (list(streams) if streams is not None else
                        [torch.cuda.Stream(device=device) for _ in range(max_streams)])
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


# ---------------------------------------------------------------------------
# Batched serving: one context and one graph launch per batch of a size class
# ---------------------------------------------------------------------------
class BatchSlot:
    """A batched context of B holograms of one class on one stream, with its
    captured solve; ``enqueue`` loads up to B requests and launches it."""

    def __init__(self, H, W, n, B, steps, lr, stream, pitch, device, tile):
        self.H, self.W, self.n, self.B, self.tile = H, W, n, B, tile
        self.stream = stream
        self.per = binding.param_count(n, 1)
        self.ctx = binding.Context(H, W, 1, pitch, [WAVELENGTHS[1]], [5e-3], max_gaussians=n,
                                   batch=B, tile=tile, device=device)
        self.params = torch.zeros(B * self.per, dtype=torch.float32, device=device)
        self.target = torch.zeros((1, B, 1, H, W), dtype=torch.float32, device=device)
        self.solve = binding.Solve(self.ctx, self.params, n, self.target, steps, lr=lr,
                                   stream=stream)

    def enqueue(self, reqs):
        """Everything for one batch of requests on this slot's stream (no host
        wait).  Fewer than B requests leave the other holograms' inputs as
        they were; their results are not read."""
        s = self.stream
        with torch.cuda.stream(s):
            for b, r in enumerate(reqs):
                self.params[b * self.per:(b + 1) * self.per].copy_(r.params, non_blocking=True)
                self.target[0, b, 0].copy_(r.target.view(self.H, self.W), non_blocking=True)
                self.ctx.set_hologram_optics(b, [r.wavelength], [r.z], stream=s)
            self.solve.launch(s)
            for b, r in enumerate(reqs):
                r.out_params.copy_(self.params[b * self.per:(b + 1) * self.per],
                                   non_blocking=True)
                r.out_loss.copy_(self.solve.loss_log.view(-1, self.B, 2)[:, b], non_blocking=True)


def batches_of(requests, max_batch):
    """Requests grouped by size class (in order of first appearance), each
    class cut into batches of at most ``max_batch`` (in request order)."""
    classes = {}
    for r in requests:
        classes.setdefault((r.H, r.W), []).append(r)
    out = []
    for key, rs in classes.items():
        for i in range(0, len(rs), max_batch):
            out.append(rs[i:i + max_batch])
    return out


class BatchServer:
    """Serves a batch of requests as one batched solve per size-class batch,
    the batches spread over up to ``max_streams`` streams (longest first)."""

    def __init__(self, steps, lr=1e-3, max_streams=2, max_batch=binding.MAX_BATCH, pitch=PITCH,
                 device="cuda", streams=None):
        self.steps, self.lr, self.pitch, self.device = steps, lr, pitch, device
        self.max_batch = max_batch
        self.streams = (list(streams) if streams is not None else
                        [torch.cuda.Stream(device=device) for _ in range(max_streams)])
        self.slots = {}
        self.tiles = {}        # (H, W) -> tile shape (width, height)
        self.batch_ms = {}     # (H, W, B) -> measured solve time of a batch, ms

    def tile_of(self, H, W):
        return self.tiles.get((H, W), (16, 16))

    def slot(self, si, H, W, n, B):
        tile = self.tile_of(H, W)
        key = (si, H, W, B, tile)
        if key not in self.slots:
            self.slots[key] = BatchSlot(H, W, n, B, self.steps, self.lr, self.streams[si],
                                        self.pitch, self.device, tile)
        s = self.slots[key]
        if s.n != n:
            raise ValueError(f"class {H}x{W} holds n = {s.n}, request has n = {n}")
        return s

    def cost(self, batch):
        r = batch[0]
        return self.batch_ms.get((r.H, r.W, len(batch)), float(r.pixels * len(batch)))

    def prepare(self, requests, streams):
        for si, q in enumerate(plan_batches(batches_of(requests, self.max_batch), streams,
                                            self.cost)):
            for bt in q:
                self.slot(si, bt[0].H, bt[0].W, bt[0].n, len(bt))
        for r in requests:
            if r.out_params is None:
                r.out_params = torch.empty_like(r.params)
                r.out_loss = torch.empty((self.steps, 2), dtype=torch.float64,
                                         device=self.device)
        torch.cuda.synchronize()

    def run(self, requests, streams=None):
        """Serves ``requests``; returns the batch wall time (s) and per request
        the solve latency (its batch's span on its stream, ms) and turnaround
        (from the batch start, ms), from HIP events."""
        streams = len(self.streams) if streams is None else streams
        queues = plan_batches(batches_of(requests, self.max_batch), streams, self.cost)
        self.prepare(requests, streams)
        main = torch.cuda.current_stream(self.device)
        t0 = torch.cuda.Event(enable_timing=True)
        marks, spans = {}, []
        host0 = time.perf_counter()
        t0.record(main)
        for si in range(streams):
            self.streams[si].wait_event(t0)
        depth = max((len(q) for q in queues), default=0)
        for k in range(depth):
            for si, q in enumerate(queues):
                if k >= len(q):
                    continue
                bt = q[k]
                slot = self.slot(si, bt[0].H, bt[0].W, bt[0].n, len(bt))
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(slot.stream)
                slot.enqueue(bt)
                e1.record(slot.stream)
                spans.append((bt, e0, e1))
                for r in bt:
                    marks[r.index] = (e0, e1, si)
        for si in range(streams):
            main.wait_stream(self.streams[si])
        torch.cuda.synchronize()
        wall = time.perf_counter() - host0
        for slot in {self.slot(si, bt[0].H, bt[0].W, bt[0].n, len(bt))
                     for si, q in enumerate(queues) for bt in q}:
            slot.ctx.read_status()
        for bt, e0, e1 in spans:
            self.batch_ms[(bt[0].H, bt[0].W, len(bt))] = e0.elapsed_time(e1)
        latency = {i: e0.elapsed_time(e1) for i, (e0, e1, _) in marks.items()}
        turnaround = {i: t0.elapsed_time(e1) for i, (_, e1, _) in marks.items()}
        return {"wall_s": wall, "latency_ms": latency, "turnaround_ms": turnaround,
                "stream_of": {i: si for i, (_, _, si) in marks.items()},
                "batches": [(bt[0].H, bt[0].W, len(bt)) for _, q in enumerate(queues)
                            for bt in q]}

    def tune_tiles(self, requests, probe_steps=20, tiles=binding.TILE_SHAPES):
        """The project's tile-shape autotuner: for each size class, times a
        ``probe_steps``-step captured solve of the class's first batch at every
        tile shape (one warm-up launch, then one timed launch) and keeps the
        fastest shape.  Returns {(H, W): {tile: ms}}."""
        timings = {}
        for bt in batches_of(requests, self.max_batch):
            key = (bt[0].H, bt[0].W)
            if key in timings:
                continue
            timings[key] = {}
            for tile in tiles:
                ctx = binding.Context(key[0], key[1], 1, self.pitch, [WAVELENGTHS[1]], [5e-3],
                                      max_gaussians=bt[0].n, batch=len(bt), tile=tile,
                                      device=self.device)
                per = binding.param_count(bt[0].n, 1)
                P = torch.cat([r.params for r in bt])
                T = torch.stack([r.target.view(key) for r in bt]).view(1, len(bt), 1, *key)
                for b, r in enumerate(bt):
                    ctx.set_hologram_optics(b, [r.wavelength], [r.z])
                stream = self.streams[0]
                solve = binding.Solve(ctx, P.clone(), bt[0].n, T.contiguous(), probe_steps,
                                      lr=self.lr, stream=stream)
                solve.launch(stream)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                solve.launch(stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ctx.read_status()
                timings[key][tile] = e0.elapsed_time(e1)
                solve.close()
                ctx.close()
                del P, T, per
            self.tiles[key] = min(timings[key], key=lambda t: (timings[key][t], t != (16, 16)))
        torch.cuda.empty_cache()
        return timings


def plan_batches(batches, streams, cost):
    """Longest-processing-time-first assignment of batches to stream queues
    (as ``plan``), each queue then shortest first."""
    load = [0.0] * streams
    queues = [[] for _ in range(streams)]
    order = sorted(range(len(batches)), key=lambda i: (-cost(batches[i]), i))
    for i in order:
        si = min(range(streams), key=lambda k: (load[k], k))
        load[si] += cost(batches[i])
        queues[si].append(batches[i])
    for q in queues:
        q.sort(key=lambda bt: (cost(bt), bt[0].index))
    return queues


def autotune_batched(server, requests, candidates=(1, 2), probe_steps=20):
    """Tile shape per class (``BatchServer.tune_tiles``), then the stream
    count: each candidate gets a warm-up run and a timed run.  Returns
    (best stream count, {count: holograms/s}, {count: timed run}, tile timings)."""
    tile_ms = server.tune_tiles(requests, probe_steps=probe_steps)
    rates, runs = {}, {}
    for k in candidates:
        if k > len(server.streams):
            continue
        server.run(requests, streams=k)
        runs[k] = server.run(requests, streams=k)
        rates[k] = len(requests) / runs[k]["wall_s"]
    best = max(rates, key=lambda k: (rates[k], -k))
    return best, rates, runs, tile_ms


def mixed_jobs(requests, batched_classes, max_batch):
    """The jobs of a mixed run: each class in ``batched_classes`` as its class
    batches (as ``batches_of``), every other request on its own.  A job is a
    list of requests; a single request is a list of one with ``batched``
    False."""
    jobs = []
    for bt in batches_of(requests, max_batch):
        if (bt[0].H, bt[0].W) in batched_classes:
            jobs.append((True, bt))
        else:
            jobs.extend((False, [r]) for r in bt)
    return jobs


def plan_jobs(jobs, streams, cost):
    """``plan_batches`` for (batched, requests) jobs: longest first onto the
    least-loaded stream, then each queue shortest first; ties by the first
    request's index."""
    load = [0.0] * streams
    queues = [[] for _ in range(streams)]
    for i in sorted(range(len(jobs)), key=lambda i: (-cost(jobs[i]), jobs[i][1][0].index)):
        si = min(range(streams), key=lambda k: (load[k], k))
        load[si] += cost(jobs[i])
        queues[si].append(jobs[i])
    for q in queues:
        q.sort(key=lambda j: (cost(j), j[1][0].index))
    return queues


def choose_modes(batch_step_ms, single_step_ms):
    """The classes to batch: those whose measured time per hologram and step
    is lower in a batched context than alone.  ``batch_step_ms`` maps a class
    to (ms per step of its batch, batch size); ``single_step_ms`` to the ms per
    step of one hologram alone."""
    return {key for key, (ms, b) in batch_step_ms.items()
            if key in single_step_ms and ms / b < single_step_ms[key]}


class MixedServer:
    """Serves each size class in the mode that is faster per hologram for it
    (``choose_modes``): a batched context per class batch (``BatchServer``
    slots) or one single-hologram solve per request (``Server`` slots).  Both
    servers share the streams; the jobs (class batches and single requests)
    are spread over them longest first (``plan_batches``) by their measured
    cost, and each stream runs its queue shortest first."""

    def __init__(self, batch_server, single_server, batch_step_ms, single_step_ms):
        if batch_server.streams != single_server.streams:
            raise ValueError("the two servers must share their streams")
        self.b, self.s = batch_server, single_server
        self.batch_step_ms, self.single_step_ms = dict(batch_step_ms), dict(single_step_ms)
        self.batched = choose_modes(self.batch_step_ms, self.single_step_ms)
        self.streams = batch_server.streams
        self.steps, self.device = batch_server.steps, batch_server.device

    def cost(self, job):
        """Measured GPU time of a job alone: a class batch scaled from its
        class's probe batch, a single request from its class's solve."""
        batched, reqs = job
        key = (reqs[0].H, reqs[0].W)
        if batched:
            ms, b = self.batch_step_ms[key]
            return self.steps * ms * len(reqs) / b
        return self.steps * self.single_step_ms.get(key, float(reqs[0].pixels))

    def queues(self, requests, streams):
        return plan_jobs(mixed_jobs(requests, self.batched, self.b.max_batch), streams, self.cost)

    def slot(self, si, job):
        batched, reqs = job
        r = reqs[0]
        return self.b.slot(si, r.H, r.W, r.n, len(reqs)) if batched else self.s.slot(si, r.H, r.W, r.n)

    def run(self, requests, streams=None):
        """As ``BatchServer.run``: batch wall time and per-request latency
        (its job's span on its stream) and turnaround, from HIP events."""
        streams = len(self.streams) if streams is None else streams
        queues = self.queues(requests, streams)
        for si, q in enumerate(queues):
            for job in q:
                self.slot(si, job)
        for r in requests:
            if r.out_params is None:
                r.out_params = torch.empty_like(r.params)
                r.out_loss = torch.empty((self.steps, 2), dtype=torch.float64,
                                         device=self.device)
        torch.cuda.synchronize()
        main = torch.cuda.current_stream(self.device)
        t0 = torch.cuda.Event(enable_timing=True)
        marks = {}
        host0 = time.perf_counter()
        t0.record(main)
        for si in range(streams):
            self.streams[si].wait_event(t0)
        depth = max((len(q) for q in queues), default=0)
        for k in range(depth):
            for si, q in enumerate(queues):
                if k >= len(q):
                    continue
                job = q[k]
                slot = self.slot(si, job)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(slot.stream)
                slot.enqueue(job[1] if job[0] else job[1][0])
                e1.record(slot.stream)
                for r in job[1]:
                    marks[r.index] = (e0, e1, si)
        for si in range(streams):
            main.wait_stream(self.streams[si])
        torch.cuda.synchronize()
        wall = time.perf_counter() - host0
        for si, q in enumerate(queues):
            for job in q:
                self.slot(si, job).ctx.read_status()
        latency = {i: e0.elapsed_time(e1) for i, (e0, e1, _) in marks.items()}
        turnaround = {i: t0.elapsed_time(e1) for i, (_, e1, _) in marks.items()}
        return {"wall_s": wall, "latency_ms": latency, "turnaround_ms": turnaround,
                "stream_of": {i: si for i, (_, _, si) in marks.items()}}

