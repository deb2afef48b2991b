"""Continuous-batching alignment server over resident reference sets.

Requests (a particle stack against one resident refset) arrive at any time.
The server keeps a set of *active* requests and runs *steps*: every step
takes the next piece of every active request (up to a step budget of
particle rows, in admission order) and aligns all pieces in one
``mra_align_batch`` call, so a request that arrives while others are on the
GPU starts with the next step instead of waiting for them to finish.  Two
steps are kept in flight so the GPU does not idle while the host plans.

Admission is by HBM footprint: the library workspace is reserved once, and
a request is admitted when its images and results fit in the rest of the
budget next to the requests already active (first come, first admitted).
Requests whose particles are in host memory are copied to the device at
admission on a copy stream (the first step that uses them waits for the
copy on the device); their device images are freed when their last piece
completes.  Pieces never change results: every request's output equals
``mra_align`` on it alone, bit for bit.

A request that the executor refuses (its admission or a step with its
pieces raises, e.g. a refset that is not loaded or images of the wrong box)
completes with ``error`` set and its budget released; the other requests
of that step are launched again without it and go on unchanged.

The GPU side sits behind a small executor interface (``admit(req)``,
``launch(pieces) -> handle``, ``done(handle)``, ``wait(handle)``,
``release(req)``) so that the scheduler runs unchanged against a stand-in on
the CPU.

    python -m paper_2011_05755_amd.serve --requests 48 --rate 20
"""

from __future__ import annotations

import argparse
import dataclasses
import heapq
import json
import math
import sys
import time

RESULT_BYTES_PER_PARTICLE = 8 * 4   # ref, shift_x, shift_y, psi, mirror, cc, cc2, flat_index


@dataclasses.dataclass
class Request:
    refset_id: int
    N: int
    L: int
    shift_max: int            # the search range used for this request (>= 0)
    parts: object = None      # device tensor [N, L, L] (or a stand-in)
    out: object = None        # AlignResult of length N (or a stand-in)
    t_arrival: float = 0.0
    # filled in by the server
    rid: int = -1
    t_admit: float | None = None
    t_done: float | None = None
    next: int = 0             # first particle not yet scheduled
    inflight: int = 0         # pieces launched and not yet completed
    finished: int = 0         # particles completed
    error: str | None = None  # set when the request failed (its results are not valid)

    @property
    def S(self) -> int:
        return (2 * self.shift_max + 1) ** 2

    def footprint(self) -> int:
        return self.N * (self.L * self.L * 4 + RESULT_BYTES_PER_PARTICLE)

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrival


@dataclasses.dataclass
class Piece:
    req: Request
    n0: int
    n: int


class Server:
    """Scheduler state; ``poll(now)`` advances it (admit, retire, launch)."""

    def __init__(self, executor, hbm_budget: int, workspace_bytes: int = 0, step_rows: int = 1 << 17,
                 max_inflight: int = 2):
        if workspace_bytes >= hbm_budget:
            raise ValueError("the workspace reserve leaves no budget for requests")
        self.ex = executor
        self.budget = hbm_budget - workspace_bytes
        self.step_rows = step_rows
        self.max_inflight = max_inflight
        self.waiting: list[Request] = []     # arrived, not admitted (FIFO)
        self.active: list[Request] = []      # admitted, not finished (admission order)
        self.inflight: list[tuple[object, list[Piece]]] = []
        self.finished: list[Request] = []
        self.failed: list[Request] = []
        self.used = 0
        self.peak_used = 0
        self._next_id = 0
        self.steps = 0
        self.max_waiting = 0

    # ---- admission ----
    def submit(self, req: Request, now: float):
        req.rid = self._next_id
        self._next_id += 1
        req.t_arrival = now if req.t_arrival == 0.0 else req.t_arrival
        if req.footprint() > self.budget:
            raise ValueError(f"request {req.rid} needs {req.footprint()} B, more than the whole budget")
        self.waiting.append(req)
        self.max_waiting = max(self.max_waiting, len(self.waiting))

    def _admit(self, now: float):
        while self.waiting and self.used + self.waiting[0].footprint() <= self.budget:
            r = self.waiting.pop(0)
            r.t_admit = now
            self.used += r.footprint()
            self.peak_used = max(self.peak_used, self.used)
            self.active.append(r)
            try:
                self.ex.admit(r)
            except Exception as e:          # noqa: BLE001 - any refusal fails this request only
                self._fail(r, e, now)

    def _fail(self, r: Request, err: Exception, now: float):
        """End request r with an error: free its budget and device images;
        pieces of it still in flight are ignored when they complete."""
        if r.error is not None:
            return
        r.error = f"{type(err).__name__}: {err}"
        r.t_done = now
        if r in self.active:
            self.active.remove(r)
        self.used -= r.footprint()
        try:
            self.ex.release(r)
        finally:
            self.failed.append(r)

    def _launch(self, pieces: list[Piece], now: float):
        """Launch one step; if the executor refuses it, launch each request's
        pieces on their own so that only the offending requests fail."""
        try:
            self.inflight.append((self.ex.launch(pieces), pieces))
            return
        except Exception as e:              # noqa: BLE001
            by_req: dict[int, list[Piece]] = {}
            for p in pieces:
                by_req.setdefault(p.req.rid, []).append(p)
            if len(by_req) == 1:
                self._fail(pieces[0].req, e, now)
                return
        for ps in by_req.values():
            try:
                self.inflight.append((self.ex.launch(ps), ps))
            except Exception as e:          # noqa: BLE001
                self._fail(ps[0].req, e, now)

    # ---- steps ----
    def _plan_step(self) -> list[Piece]:
        """The next piece of every active request, in admission order, within
        the step's row budget (each request gets at least one particle while
        rows remain; the first request always gets one)."""
        pieces = []
        rows = 0
        todo = [r for r in self.active if r.next < r.N]
        if not todo:
            return pieces
        share = max(1, self.step_rows // len(todo))
        for r in todo:
            if rows >= self.step_rows and pieces:
                break
            n = min(r.N - r.next, max(1, share // r.S), max(1, (self.step_rows - rows) // r.S))
            pieces.append(Piece(r, r.next, n))
            r.next += n
            r.inflight += 1
            rows += n * r.S
        return pieces

    def _retire(self, now: float):
        keep = []
        for h, pieces in self.inflight:
            if self.ex.done(h):
                for p in pieces:
                    if p.req.error is not None:
                        continue
                    p.req.inflight -= 1
                    p.req.finished += p.n
                    if p.req.finished == p.req.N:
                        p.req.t_done = now
                        self.used -= p.req.footprint()
                        self.ex.release(p.req)
                        self.active.remove(p.req)
                        self.finished.append(p.req)
            else:
                keep.append((h, pieces))
        self.inflight = keep

    def poll(self, now: float) -> bool:
        """One scheduling round.  Returns True if anything is left to do."""
        self._retire(now)
        self._admit(now)
        while len(self.inflight) < self.max_inflight:
            pieces = self._plan_step()
            if not pieces:
                break
            self._launch(pieces, now)
            self.steps += 1
        return bool(self.waiting or self.active or self.inflight)

    def wait_one(self):
        if self.inflight:
            self.ex.wait(self.inflight[0][0])


def percentile(xs: list[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not xs:
        return math.nan
    s = sorted(xs)
    k = max(0, min(len(s) - 1, math.ceil(q / 100.0 * len(s)) - 1))
    return s[k]


def run_trace(server: Server, arrivals: list[tuple[float, Request]], clock=time.perf_counter,
              sleep=time.sleep, warmup: int = 0, progress=None) -> dict:
    """Feed `arrivals` ((offset s, request), sorted) to the server on the
    clock, run until every request is finished; return latency statistics
    over the requests after the first `warmup` arrivals.  `progress(n_done)`
    is called as requests finish."""
    t0 = clock()
    heap = [(t, i, r) for i, (t, r) in enumerate(arrivals)]
    heapq.heapify(heap)
    busy = True
    while heap or busy:
        now = clock() - t0
        while heap and heap[0][0] <= now:
            t, _, r = heapq.heappop(heap)
            r.t_arrival = t
            server.submit(r, t)
        done_before = len(server.finished)
        busy = server.poll(now)
        if progress and len(server.finished) != done_before:
            progress(len(server.finished))
        if server.inflight:
            server.wait_one()      # block on the oldest step; the next is already queued
        elif heap:
            sleep(max(0.0, min(heap[0][0] - (clock() - t0), 0.05)))
    t_end = clock() - t0
    measured = [r for r in server.finished if r.rid >= warmup]
    lat = [r.latency for r in measured]
    parts = sum(r.N for r in measured)
    first = min((r.t_arrival for r in measured), default=0.0)
    t_last = max((r.t_done for r in measured), default=t_end)
    return dict(requests=len(measured), warmup_requests=len(server.finished) - len(measured),
                failed_requests=len(server.failed), particles=parts, steps=server.steps,
                p50_s=percentile(lat, 50), p99_s=percentile(lat, 99), max_s=max(lat) if lat else math.nan,
                mean_s=sum(lat) / len(lat) if lat else math.nan,
                makespan_s=t_last - first, particles_per_s=parts / max(t_last - first, 1e-9),
                max_waiting=server.max_waiting, peak_admitted_gib=server.peak_used / 2**30)


# ---------------------------------------------------------------------------
# GPU executor over libmra


class AlignExecutor:
    """Runs a step as one mra_align_batch call on the context's stream and
    marks it with an event.  Requests whose particles are in (pinned) host
    memory are copied to the device at admission on a copy stream."""

    def __init__(self, ctx):
        import torch
        self.ctx = ctx
        self.torch = torch
        self.dev = torch.device("cuda", ctx.device)
        self.copy_stream = torch.cuda.Stream(self.dev)

    def admit(self, r: Request):
        t = self.torch
        r.dev_parts, r.ready = r.parts, None
        if not r.parts.is_cuda:
            with t.cuda.stream(self.ctx.stream):
                r.dev_parts = t.empty(r.parts.shape, dtype=r.parts.dtype, device=self.dev)
            with t.cuda.stream(self.copy_stream):
                r.dev_parts.copy_(r.parts, non_blocking=True)
                r.dev_parts.record_stream(self.copy_stream)
                r.ready = t.cuda.Event()
                r.ready.record(self.copy_stream)

    def launch(self, pieces: list[Piece]):
        stacks = []
        for p in pieces:
            r = p.req
            if r.ready is not None:            # first use: wait for the copy on the device
                self.ctx.stream.wait_event(r.ready)
                r.ready = None
            stacks.append((r.refset_id, r.dev_parts[p.n0:p.n0 + p.n], r.shift_max, r.out.narrow(p.n0, p.n)))
        self.ctx.align_batch(stacks)
        ev = self.torch.cuda.Event()
        ev.record(self.ctx.stream)
        return ev

    def done(self, ev) -> bool:
        return ev.query()

    def wait(self, ev):
        ev.synchronize()

    def release(self, r: Request):
        r.dev_parts = None        # device images of a host request go back to the allocator


def make_refsets(ctx, n_sets: int, seed: int, precision: str, specs=None):
    """Resident refsets drawn from the uneven-stack size distribution."""
    import torch

    from . import synth
    specs = specs or synth.uneven_stack_specs(n_sets, seed=seed)
    dev = torch.device("cuda", ctx.device)
    sets = []
    for i, sp in enumerate(specs[:n_sets]):
        blobs = synth.make_blobs(sp["K"], sp["L"], seed=(seed, 100 + i), rho_max=sp["rho_max"])
        refs = synth.render_refs(blobs).to(dev)
        ctx.load_refs(i, refs, r_min=sp["r_min"], r_max=sp["r_max"], shift_max=sp["shift_max"],
                      precision=precision)
        sets.append(dict(id=i, blobs=blobs, refs=refs, **sp))
    return sets


def make_requests(sets, n_req: int, rate: float, seed: int, device, n_scale: float = 1.0,
                  host: bool = False, pool: bool = False):
    """Poisson arrivals at `rate`/s; each request draws its refset uniformly
    and its size from the uneven-stack distribution (N uniform 2k..50k,
    scaled by n_scale; shift range of its refset).  host: particles in pinned
    host memory (copied at admission), else resident on the device.  pool:
    every refset gets one stack of the largest size and a request takes a
    random contiguous slice of it (for long traces that could not hold a
    stack per request)."""
    import numpy as np

    from . import mra, synth
    rng = np.random.default_rng(seed)
    n_max = max(1, int(round(50000 * n_scale)))
    pools = {}
    if pool:
        for s in sets:
            p, _ = synth.make_particles(s["blobs"], n_max, s["shift_max"], s["snr"], seed=(seed, 500 + s["id"]),
                                        device=device)
            pools[s["id"]] = p.cpu().pin_memory() if host else p
    t = 0.0
    out = []
    for j in range(n_req):
        t += rng.exponential(1.0 / rate)
        s = sets[int(rng.integers(len(sets)))]
        N = max(1, int(round(int(rng.integers(2000, 50001)) * n_scale)))
        if pool:
            o = int(rng.integers(0, n_max - N + 1))
            parts = pools[s["id"]][o:o + N]
        else:
            parts, _ = synth.make_particles(s["blobs"], N, s["shift_max"], s["snr"], seed=(seed, 1000 + j),
                                            device=device)
            if host:
                parts = parts.cpu().pin_memory()
        r = Request(refset_id=s["id"], N=N, L=s["L"], shift_max=s["shift_max"], parts=parts,
                    out=mra.AlignResult.empty(N, device))
        out.append((t, r))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="continuous-batching alignment server on one GPU")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--rate", type=float, default=20.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--refsets", type=int, default=8)
    ap.add_argument("--precision", default="bf16", choices=("fp32", "bf16", "fp16"))
    ap.add_argument("--budget-gib", type=float, default=96.0, help="HBM budget for admitted requests")
    ap.add_argument("--step-rows", type=int, default=1 << 18)
    ap.add_argument("--n-scale", type=float, default=1.0, help="scale of the request sizes")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--check", type=int, default=4, help="requests re-run alone and compared bit for bit")
    ap.add_argument("--host-inputs", action="store_true", help="particles in pinned host memory")
    ap.add_argument("--warmup-requests", type=int, default=0, help="first arrivals left out of the statistics")
    ap.add_argument("--pool", action="store_true", help="requests slice one pre-generated stack per refset")
    ap.add_argument("--workspace-gib", type=float, default=8.0, help="library workspace cap (reserved)")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import mra
    dev = torch.device("cuda", 0)
    ws = int(args.workspace_gib * 2**30)
    ctx = mra.Context(0, workspace_cap=ws)
    sets = make_refsets(ctx, args.refsets, args.seed, args.precision)
    n_all = args.requests + args.warmup_requests
    arrivals = make_requests(sets, n_all, args.rate, args.seed, dev, args.n_scale, host=args.host_inputs,
                             pool=args.pool)
    torch.cuda.synchronize()
    server = Server(AlignExecutor(ctx), hbm_budget=int(args.budget_gib * 2**30), workspace_bytes=ws,
                    step_rows=args.step_rows)
    t_start = time.perf_counter()

    def progress(n):
        if n % 25 == 0 or n == n_all:
            print(f"[serve] {n}/{n_all} requests done, {time.perf_counter() - t_start:.1f} s, "
                  f"waiting {len(server.waiting)}, active {len(server.active)}", file=sys.stderr, flush=True)

    stats = run_trace(server, arrivals, warmup=args.warmup_requests, progress=progress)
    torch.cuda.synchronize()
    same = 0
    for _, r in arrivals[:args.check]:
        alone = ctx.align(r.refset_id, r.parts.to(dev))
        a, b = alone.to_numpy(), r.out.to_numpy()
        same += all(np.array_equal(a[k], b[k]) for k in a)
    offered = sum(r.N for _, r in arrivals) / max(arrivals[-1][0], 1e-9)
    line = dict(workload=f"serving: {args.warmup_requests} warm-up + {args.requests} measured requests, Poisson "
                         f"{args.rate}/s, {args.refsets} resident refsets, {args.precision}"
                         + (", host inputs" if args.host_inputs else "") + (", pooled stacks" if args.pool else ""),
                offered_particles_per_s=round(offered, 1),
                same_alone_and_in_mix=f"{same}/{min(args.check, len(arrivals))}",
                **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()})
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
