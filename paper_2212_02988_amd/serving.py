"""Continuous-batching serving loop for many concurrent agent streams.

Each agent stream is one PRISM filter whose voxel map and filter state stay
resident in HBM for the stream's lifetime.  Frames arrive at their own pace
(a stream's frames in order).  The loop

* admits a stream only when its device footprint (map + filter state + input
  slots, all sized by the library's size queries) fits the HBM budget, keeps
  the others queued in arrival order, and admits queued streams as soon as
  finished ones release their memory;
* batches continuously: on every tick, the admitted streams that have a
  pending frame and a free input slot form one batch per HIP stream (agents
  are spread over a small pool of HIP streams at admission), and one library
  call (prism_filter_step_batch) stages their frames into their slots and runs
  the whole step for all of them with one kernel launch per stage, ragged over
  their different image and map sizes (batch_graphs=True: the stages replayed
  from a HIP graph recorded per member set and slots); frames arriving while a
  batch runs join the next one.  (batched=False submits each stream's step on its own,
  as a HIP graph recorded per slot.)  Completions come from the library's
  per-slot events (prism_filter_poll on one member per batch);
* allows up to ``depth`` steps of one agent in flight (they are ordered on its
  HIP stream; each slot is reused only after the step that read it finished),
  and records per-frame latency from arrival to host-visible completion.

Results are independent of the mix: every kernel of a step reads and writes
only its own agent's buffers and every reduction has a fixed order, so an
agent's state and map are bitwise the same alone and among others.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional, Tuple

import numpy as np
import torch

from . import prism as P


@dataclasses.dataclass
class StreamSpec:
    stream_id: int
    grid: P.Grid
    cam: P.Camera
    params: P.FilterParams
    x0: np.ndarray                   # (t, q, v, w), 13 values; (t, q, v, w, b), 16 with MODE_ACCEL_BIAS
    P0: np.ndarray                   # 12 x 12; 15 x 15 with MODE_ACCEL_BIAS
    n_frames: int                    # the stream closes after this many frames


@dataclasses.dataclass
class _Frame:
    arrival: float                   # host clock (perf_counter) of arrival
    depth: object                    # [H, W] float32: device tensor or host array
    rgb: object                      # [H, W, 3]
    u: object                        # [6] float64 or None (first frame)
    index: int
    ready: object = None             # torch.cuda.Event after which device frames are complete


def footprint_bytes(spec: StreamSpec, depth: int = 2, staged: bool = False) -> int:
    """Device bytes an admitted stream holds: map, filter state and `depth`
    input slots (depth f32, rgb f32, control f64), each rounded to the
    allocator's 512-byte granule."""
    r = lambda b: (b + 511) // 512 * 512
    cfg = P.filter_cfg(spec.grid, spec.cam, spec.params)
    npix = spec.cam.width * spec.cam.height
    slot = r(4 * npix) + r(12 * npix) + r(48)
    return r(P.map_bytes(spec.grid)) + r(P.filter_bytes(cfg)) + depth * slot


class _Agent:
    """One admitted stream: its filter, `depth` device input slots registered
    with the library (plus pinned host slots when frames come from the host),
    and the frames waiting or in flight."""

    def __init__(self, spec: StreamSpec, hip_stream: torch.cuda.Stream, depth: int, staged: bool,
                 use_graph: bool):
        self.spec = spec
        self.stream = hip_stream
        self.depth = depth
        self.staged = staged
        self.flags = (P.SUBMIT_FROM_HOST if staged else 0) | (0 if use_graph else P.SUBMIT_EAGER)
        H, W = spec.cam.height, spec.cam.width
        with torch.cuda.stream(hip_stream):
            self.filter = P.Filter(spec.grid, spec.cam, spec.params)
            self.filter.map.init(stream=hip_stream)
            self.filter.reset(spec.x0, spec.P0, stream=hip_stream)
            slots = [(torch.empty((H, W), dtype=torch.float32, device="cuda"),
                      torch.empty((H, W, 3), dtype=torch.float32, device="cuda"),
                      torch.zeros(6, dtype=torch.float64, device="cuda")) for _ in range(depth)]
            self.filter.set_slots(slots)
            self.host = None
            if staged:
                self.host = [(torch.empty((H, W), dtype=torch.float32).pin_memory(),
                              torch.empty((H, W, 3), dtype=torch.float32).pin_memory(),
                              torch.zeros(6, dtype=torch.float64).pin_memory()) for _ in range(depth)]
        self.pending: Deque[_Frame] = collections.deque()
        self.in_flight: Deque[_Frame] = collections.deque()
        self.launched = 0
        self.done = 0

    def ready(self) -> bool:
        return bool(self.pending) and self.launched - self.done < self.depth

    def source(self):
        """The next frame's buffers as the library reads them (staged: copied
        into this step's pinned host slot first)."""
        fr = self.pending[0]
        if not self.staged:
            if fr.ready is not None:
                self.stream.wait_event(fr.ready)     # the frame's producer, on another stream
            return fr.depth, fr.rgb, fr.u
        hd, hc, hu = self.host[self.launched % self.depth]
        hd.numpy()[...] = fr.depth
        hc.numpy()[...] = fr.rgb
        if fr.u is not None:
            hu.numpy()[...] = fr.u
        return hd, hc, None if fr.u is None else hu

    def launched_one(self):
        self.in_flight.append(self.pending.popleft())
        self.launched += 1

    def launch(self):
        """Submit the next frame on its own (one step graph per slot)."""
        if self.filter.submit(*self.source(), stream=self.stream, flags=self.flags) is None:
            return False
        self.launched_one()
        return True

    def complete_one(self) -> _Frame:
        self.done += 1
        return self.in_flight.popleft()

    def finished(self) -> bool:
        return self.done >= self.spec.n_frames


class ServingLoop:
    """Admission, continuous launching and completion tracking of agent
    streams on one GPU.

    hbm_budget: bytes the streams may hold together (None: the free device
    memory less `reserve`).  staged=False: frames are device tensors already in
    HBM (copied device-to-device into a slot); staged=True: host arrays copied
    through pinned buffers.  keep_final=True reads back each stream's final
    state and dense map when it retires (for tests)."""

    def __init__(self, hbm_budget: Optional[int] = None, n_hip_streams: int = 4, depth: int = 2,
                 staged: bool = False, use_graphs: bool = True, reserve: int = 2 << 30, keep_final: bool = False,
                 batched: bool = True, batch_graphs: bool = True):
        free, _ = torch.cuda.mem_get_info()
        cap = max(0, free - reserve)
        self.budget = cap if hbm_budget is None else min(int(hbm_budget), cap)
        self.pool = [torch.cuda.Stream() for _ in range(n_hip_streams)]
        self.depth = depth
        self.staged = staged
        self.use_graphs = use_graphs
        self.batched = batched
        self.batch_graphs = batch_graphs   # batched steps replayed from graphs recorded per member set
        self.keep_final = keep_final
        self.batches = 0
        # launched batches per HIP stream, oldest first: (agents, probe agent,
        # the probe's submission count that marks the batch complete).  A
        # batch's steps end together on its stream, so one event tells.
        self.inflight: Dict[int, Deque[tuple]] = collections.defaultdict(collections.deque)
        self.queue: Deque[StreamSpec] = collections.deque()
        self.agents: Dict[int, _Agent] = {}
        self.held = 0
        self.waiting: Dict[int, Deque[_Frame]] = collections.defaultdict(collections.deque)
        self.latencies: List[float] = []
        self.per_stream_latency: Dict[int, List[float]] = collections.defaultdict(list)
        self.admit_time: Dict[int, float] = {}
        self.completed = 0
        self.max_concurrent = 0
        self.max_held_bytes = 0
        self.final: Dict[int, dict] = {}
        self.totals: Dict[int, dict] = {}
        self._rr = 0
        self.host_submit_s = 0.0          # host time inside step submissions
        self.host_poll_s = 0.0            # host time inside completion polls

    # ---- admission -------------------------------------------------------
    def open_stream(self, spec: StreamSpec):
        need = footprint_bytes(spec, self.depth, self.staged)
        if need > self.budget:
            raise P.PrismError(f"stream {spec.stream_id} needs {need} bytes, more than the budget {self.budget}")
        self.queue.append(spec)
        self._admit()

    def _admit(self):
        while self.queue:
            spec = self.queue[0]
            need = footprint_bytes(spec, self.depth, self.staged)
            if self.held + need > self.budget:
                return
            self.queue.popleft()
            hs = self.pool[self._rr % len(self.pool)]
            self._rr += 1
            ag = _Agent(spec, hs, self.depth, self.staged, self.use_graphs)
            self.agents[spec.stream_id] = ag
            self.held += need
            self.max_held_bytes = max(self.max_held_bytes, self.held)
            self.admit_time[spec.stream_id] = time.perf_counter()
            self.max_concurrent = max(self.max_concurrent, len(self.agents))
            ag.pending.extend(self.waiting.pop(spec.stream_id, ()))

    def _retire(self, ag: _Agent):
        sid = ag.spec.stream_id
        # totals for throughput accounting (one small read of the state)
        st0 = ag.filter.state()
        self.totals[sid] = dict(steps=int(st0.step), n_updated_total=int(st0.n_updated_total))
        if ag.spec.grid.capacity > 0:
            used, dropped = (int(v) for v in ag.filter.map.pool_usage(stream=ag.stream).cpu())
            self.totals[sid].update(pool_used=used, pool_dropped=dropped, pool_capacity=int(ag.spec.grid.capacity))
        if self.keep_final:
            st = ag.filter.state()
            mean, var = ag.filter.map.to_dense(stream=ag.stream)
            torch.cuda.synchronize()
            self.final[sid] = dict(state=st, mean=mean.cpu(), var=var.cpu())
        ag.stream.synchronize()
        del self.agents[sid]
        self.held -= footprint_bytes(ag.spec, self.depth, self.staged)
        ag.filter = None
        ag.host = None
        self._admit()

    # ---- frames ----------------------------------------------------------
    def push_frame(self, stream_id: int, arrival: float, depth, rgb, u, index: int, ready=None):
        """Queue a frame.  Device frames (staged=False) are read by the
        library on the agent's HIP stream, which does not otherwise wait for
        the stream that wrote them: pass `ready`, a torch.cuda.Event recorded
        on the producing stream after the frame's tensors were written, or
        push only frames that are already complete (e.g. synchronized)."""
        fr = _Frame(arrival, depth, rgb, u, index, ready)
        ag = self.agents.get(stream_id)
        if ag is None:
            self.waiting[stream_id].append(fr)       # queued on the host until the stream is admitted
        else:
            ag.pending.append(fr)

    # ---- progress --------------------------------------------------------
    def poll(self) -> int:
        """Retire finished batches (oldest first on each HIP stream); returns
        how many steps completed."""
        n = 0
        retire = []
        for q in self.inflight.values():
            while q:
                ags, probe, need = q[0]
                t0 = time.perf_counter()
                c = probe.filter.poll()
                self.host_poll_s += time.perf_counter() - t0
                if c < need:
                    break
                q.popleft()
                now = time.perf_counter()
                for ag in ags:
                    fr = ag.complete_one()
                    lat = now - fr.arrival
                    self.latencies.append(lat)
                    self.per_stream_latency[ag.spec.stream_id].append(lat)
                    if ag.finished():
                        retire.append(ag)
                self.completed += len(ags)
                n += len(ags)
        for ag in retire:
            self._retire(ag)
        return n

    def tick(self) -> int:
        """Launch every step that can start now; returns how many.  Batched:
        the ready agents of each HIP stream form one batch (one launch per
        stage for all of them); otherwise each agent submits on its own."""
        n = 0
        progress = True
        while progress:
            progress = False
            if self.batched:
                groups: Dict[int, List[_Agent]] = collections.defaultdict(list)
                for ag in self.agents.values():
                    if ag.ready():
                        groups[id(ag.stream)].append(ag)
                for ags in groups.values():
                    t0 = time.perf_counter()
                    fl = (ags[0].flags & P.SUBMIT_FROM_HOST) | (P.SUBMIT_GRAPH if self.batch_graphs else 0)
                    ok = P.filter_step_batch([ag.filter for ag in ags], [ag.source() for ag in ags],
                                             stream=ags[0].stream, flags=fl)
                    self.host_submit_s += time.perf_counter() - t0
                    if ok:
                        for ag in ags:
                            ag.launched_one()
                        self.inflight[id(ags[0].stream)].append((ags, ags[-1], ags[-1].launched))
                        n += len(ags)
                        self.batches += 1
                        progress = True
            else:
                for ag in self.agents.values():
                    if ag.ready():
                        t0 = time.perf_counter()
                        ok = ag.launch()
                        self.host_submit_s += time.perf_counter() - t0
                        if ok:
                            self.inflight[id(ag.stream)].append(([ag], ag, ag.launched))
                            self.batches += 1
                            n += 1
                            progress = True
        return n

    def busy(self) -> bool:
        return bool(self.queue) or bool(self.agents) or bool(self.waiting)

    def idle_device(self) -> bool:
        return not any(self.inflight.values())

    def run_until_idle(self, timeout: float = 600.0):
        t0 = time.perf_counter()
        while self.busy():
            self.poll()
            self.tick()
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("serving loop did not drain")
        torch.cuda.synchronize()

    def stats(self) -> Dict[str, float]:
        lat = np.array(self.latencies) * 1e3
        pct = (lambda q: float(np.percentile(lat, q))) if len(lat) else (lambda q: float("nan"))
        return {"completed": self.completed, "p50_ms": pct(50), "p99_ms": pct(99),
                "max_ms": float(lat.max()) if len(lat) else float("nan"),
                "max_concurrent": self.max_concurrent, "max_held_bytes": self.max_held_bytes,
                "budget_bytes": self.budget}


def run_schedule(loop: ServingLoop, specs: List[StreamSpec], schedule: List[tuple],
                 frame_source: Callable[[int, int], tuple], realtime: bool = True,
                 timeout: float = 900.0) -> float:
    """Open every stream, then feed frames at their arrival times (schedule:
    (t_seconds, stream_id, index) sorted by t) while keeping the loop going.
    realtime=False delivers every frame at time 0 (backlog: throughput).
    Returns the wall time from start to the last completion."""
    t0 = time.perf_counter()
    for sp in specs:
        loop.open_stream(sp)
    i = 0
    while i < len(schedule) or loop.busy():
        now = time.perf_counter() - t0
        while i < len(schedule) and (not realtime or schedule[i][0] <= now):
            ta, sid, idx = schedule[i]
            src = frame_source(sid, idx)     # (depth, rgb, u) or (depth, rgb, u, ready event)
            loop.push_frame(sid, t0 + (ta if realtime else 0.0), src[0], src[1], src[2], idx,
                            ready=src[3] if len(src) > 3 else None)
            i += 1
        loop.poll()
        loop.tick()
        if time.perf_counter() - t0 > timeout:
            raise TimeoutError("serving run did not finish")
        if realtime and i < len(schedule) and not any(a.in_flight for a in loop.agents.values()):
            wait = schedule[i][0] - (time.perf_counter() - t0)
            if wait > 2e-4:
                time.sleep(min(wait, 1e-3))
    torch.cuda.synchronize()
    return time.perf_counter() - t0
