"""Streaming correlator: several input streams share one GPU (Sec. II).

Frames arrive from the network side in pinned host memory (the ring
buffers of Sec. II-A).  The server

* admits a frame to the device only while the HBM it needs fits a fixed
  budget (frame buffers in flight plus every open stream's resident
  accumulators), so a burst waits in host memory instead of failing;
* copies admitted frames host-to-device on a copy stream;
* launches, whenever the GPU has room, ONE persistent batched launch over
  the oldest ready frame of every stream (continuous batching: frames that
  arrive while a batch runs join the next one);
* keeps each stream's integration resident on the device, adding frame
  after frame (Sec. II-B), and at the end of an integration normalises it
  for lost samples (Sec. II-C) and copies it out, while the stream's next
  integration proceeds in a second accumulator;
* with aligned streams, bounds every integration by the frames' sequence
  numbers (window k holds frames k L .. k L + L - 1), so the integrations
  of different streams cover the same time and :class:`Combiner` can join
  them, ordered by stream id, into one output over all their channels
  (Sec. II-C: the eight streams of a host are combined; Sec. II-D: the
  sequence number aligns frames in time).

Every compute step runs in the library's kernels (xengine); this module
only schedules them and owns the memory accounting.  Frame latency is
measured from arrival in pinned memory to the completion of the
accumulation that consumed the frame, on the GPU's clock.
"""

from __future__ import annotations

import collections
import dataclasses
import queue
import sys
import threading
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np

from . import xengine


@dataclasses.dataclass
class StreamConfig:
    stream_id: int
    N: int
    F: int
    T: int                       # samples per frame
    B: int                       # samples per loss-mask block
    frames_per_integration: int
    # integrations bounded by sequence number: window k = frames with
    # seq // frames_per_integration == k (a window may hold fewer frames
    # when some never arrived); False: every frames_per_integration
    # frames in arrival order
    aligned: bool = False


@dataclasses.dataclass
class Frame:
    stream_id: int
    seq: int                     # sequence number of the frame in its stream
    packed: "object"             # pinned uint8 [T][F][N] host tensor (or in HBM)
    mask: "object"               # pinned uint8 [F][nblk] host tensor or None
    t_arrival: float             # time.perf_counter() at arrival
    # set by the server
    slices: int = 0              # time slices the frame is copied and integrated in
    copied: int = 0              # slices whose copy has been issued
    launched: int = 0            # slices launched
    ev_copy_start: "object" = None
    ev_copied: "object" = None   # copy of the last slice done
    t_copy_issue: float = 0.0    # host time the first slice's copy was issued
    done: int = 0                # slices whose batch has finished
    t_done: float = 0.0


@dataclasses.dataclass
class _Slice:
    frame: Frame
    t0: int
    t1: int
    packed: "object"             # device uint8 [t1 - t0][F][N]
    mask: "object"               # device uint8 [F][ceil((t1 - t0) / B)] or None
    ev_copied: "object"          # None: nothing to wait for
    slot: int = -1               # pool slot, released when the batch is done


@dataclasses.dataclass
class IntegrationResult:
    stream_id: int
    index: int                   # integration number of the stream
    frames: int
    vis: np.ndarray              # int32 [F][P][2]
    count: np.ndarray            # int64 [F]
    out: np.ndarray              # float32 [F][P][2]
    t_ready: float
    seq_first: int = -1          # sequence numbers of the first and last frame
    seq_last: int = -1
    window: int = -1             # aligned streams: the sequence-number window


class _Stream:
    def __init__(self, cfg: StreamConfig, device, slice_samples: int,
                 pinned_results: bool = True):
        import torch
        self.cfg = cfg
        N, F = cfg.N, cfg.F
        P = N * (N + 1) // 2
        self.acc = [xengine.new_accumulators(N, F, device) for _ in range(2)]
        self.out = [torch.empty((F, P, 2), dtype=torch.float32, device=device)
                    for _ in range(2)]
        self.host = [(torch.empty((F, P, 2), dtype=torch.int32, pin_memory=pinned_results),
                      torch.empty((F,), dtype=torch.int64, pin_memory=pinned_results),
                      torch.empty((F, P, 2), dtype=torch.float32, pin_memory=pinned_results))
                     for _ in range(2)]
        self.ev_d2h = [None, None]   # copy-out of buffer k finished
        self.host_busy = [False, False]  # host copy k not yet taken
        self.host_free = [threading.Event(), threading.Event()]
        for e in self.host_free:
            e.set()
        self.cur = 0
        self.frames_in = 0           # frames launched into the current integration
        self.seq_first = -1          # ... and the sequence numbers they span
        self.seq_last = -1
        self.window = -1             # aligned: window of the current integration
        self.index = 0
        self.slice_samples = slice_samples
        self.pending: Deque[_Slice] = collections.deque()  # copied or copying, not launched
        self.waiting: Deque[Frame] = collections.deque()   # arrived, slices left to copy
        self.resident_bytes = self.resident_bytes_for(cfg)

    @staticmethod
    def resident_bytes_for(cfg: StreamConfig) -> int:
        P = cfg.N * (cfg.N + 1) // 2
        return 2 * (2 * cfg.F * P * 8 + cfg.F * 8)


class SlotPool:
    """Device frame buffers carved once, at start-up, out of the HBM budget
    (the counterpart of the ring buffers of Sec. II-A): ``n`` slots of
    ``slot_bytes`` for a time slice of packed samples, each with a small
    region for the slice's loss mask and a pinned host staging area for
    that mask.  Nothing is allocated or freed in steady state."""

    MASK_BYTES = 4096

    def __init__(self, torch, device, n: int, slot_bytes: int):
        self.n = n
        self.slot_bytes = slot_bytes
        self.data = torch.empty(n * slot_bytes, dtype=torch.uint8, device=device)
        self.masks = torch.empty(n * self.MASK_BYTES, dtype=torch.uint8, device=device)
        self.host_masks = torch.empty(n * self.MASK_BYTES, dtype=torch.uint8, pin_memory=True)
        self.free: List[int] = list(range(n - 1, -1, -1))

    @property
    def bytes(self) -> int:
        return self.n * (self.slot_bytes + self.MASK_BYTES)

    def take(self) -> int:
        return self.free.pop() if self.free else -1

    def give(self, k: int) -> None:
        self.free.append(k)

    def packed(self, k: int, shape):
        n = shape[0] * shape[1] * shape[2]
        return self.data[k * self.slot_bytes:k * self.slot_bytes + n].view(shape)

    def mask(self, k: int, shape, host: bool = False):
        n = shape[0] * shape[1]
        buf = self.host_masks if host else self.masks
        return buf[k * self.MASK_BYTES:k * self.MASK_BYTES + n].view(shape)


def slice_samples_for(cfg: StreamConfig, slot_bytes: int, want: Optional[int] = None) -> int:
    """Samples per time slice of a stream's frames: at most ``want`` (default:
    the whole frame) and what fits one slot, a multiple of the loss-mask
    block so that every slice's mask is whole blocks of the frame's."""
    per_sample = cfg.F * cfg.N
    fit = slot_bytes // per_sample // cfg.B * cfg.B
    if fit < 1:
        raise ValueError(f"stream {cfg.stream_id}: one {cfg.B}-sample mask block "
                         f"({cfg.B * per_sample} B) does not fit a {slot_bytes} B slot")
    s = min(cfg.T, fit)
    if want is not None:
        s = min(s, max(cfg.B, want // cfg.B * cfg.B))
    if cfg.F * ((s + cfg.B - 1) // cfg.B) > SlotPool.MASK_BYTES:
        raise ValueError(f"stream {cfg.stream_id}: a slice's loss mask exceeds "
                         f"{SlotPool.MASK_BYTES} B; use shorter slices")
    return s


class StreamServer:
    """Admission, batching and integration of frames from many streams.

    Host frames are copied in time slices of at most ``slice_samples``
    samples (default: whole frames, as far as a slot holds them) into slots
    of a device pool carved out of ``hbm_budget`` at start-up
    (``pool_bytes``, default half the budget; the rest holds the streams'
    resident accumulators).  A slice is accumulated as soon as its copy has
    landed: one batched launch takes the oldest landed slice of every
    stream, so a frame's compute overlaps the copy of its later slices and
    a large frame does not hold the GPU until it has crossed the host link
    whole.  Copies are issued oldest frame first, as slots free up."""

    def __init__(self, hbm_budget: int, device: int = 0, max_inflight: int = 2,
                 handle: Optional[xengine.Handle] = None,
                 on_result: Optional[Callable[[IntegrationResult], None]] = None,
                 slot_bytes: int = 32 << 20, pool_bytes: Optional[int] = None,
                 slice_samples: Optional[int] = None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.budget = int(hbm_budget)
        self.max_inflight = max_inflight
        self.h = handle or xengine.default_handle(device)
        self.copy_stream = torch.cuda.Stream(self.device)
        self.compute_stream = torch.cuda.Stream(self.device)
        self.d2h_stream = torch.cuda.Stream(self.device)
        pool_bytes = self.budget // 2 if pool_bytes is None else int(pool_bytes)
        n_slots = pool_bytes // (slot_bytes + SlotPool.MASK_BYTES)
        if n_slots < 1:
            raise MemoryError(f"a {pool_bytes} B pool holds no {slot_bytes} B slot")
        self.pool = SlotPool(torch, self.device, n_slots, slot_bytes)
        self.used = self.pool.bytes
        self.slice_want = slice_samples
        self.streams: Dict[int, _Stream] = {}
        self.arrivals: "queue.Queue[Frame]" = queue.Queue()
        self.inflight: Deque[tuple] = collections.deque()   # (event, slices)
        # finished integrations are handed to a delivery thread, which waits
        # for their copy-out and copies them out of the pinned buffers, so
        # that the scheduling loop never copies a result (tens of MB)
        self._out_q: "queue.Queue" = queue.Queue()
        self._out_pending = 0
        self._out_lock = threading.Lock()
        self._deliver_error: Optional[BaseException] = None
        self._deliverer = threading.Thread(target=self._deliver, daemon=True)
        self._deliverer.start()
        self.results: Dict[int, List[IntegrationResult]] = collections.defaultdict(list)
        self.on_result = on_result
        self.latencies: List[float] = []
        self.breakdown: List[tuple] = []   # per frame: (wait, copy, finish) seconds
        self.done_frames: List[tuple] = []  # per frame: (stream, seq, arrival time)
        self.bytes_done = 0
        self.samples_done = 0
        self.frames_done = 0
        self.batches = 0
        self.batch_sizes: List[int] = []
        self.max_used = self.used
        self.admission_waits = 0
        # host clock <-> GPU clock: an event recorded and waited for now,
        # re-anchored every 20 ms while serving (the two clocks drift apart
        # by parts per thousand over seconds)
        ev_ref = torch.cuda.Event(enable_timing=True)
        ev_ref.record(self.compute_stream)
        ev_ref.synchronize()
        self._ref = (ev_ref, time.perf_counter())   # one attribute: replaced whole
        self._anchor = None          # anchor event in flight
        self._anchor_period = 0.02

    # -- streams ----------------------------------------------------------

    def open(self, cfg: StreamConfig) -> None:
        if cfg.stream_id in self.streams:
            raise ValueError(f"stream {cfg.stream_id} already open")
        need = _Stream.resident_bytes_for(cfg)
        if need > self.budget - self.used:
            raise MemoryError(
                f"stream {cfg.stream_id}: accumulators ({need} B) do not fit the HBM "
                f"budget ({self.budget - self.used} B free beside the frame pool)")
        s_len = slice_samples_for(cfg, self.pool.slot_bytes, self.slice_want)
        self.used += need
        self.max_used = max(self.max_used, self.used)
        with self.torch.cuda.stream(self.compute_stream):
            self.streams[cfg.stream_id] = _Stream(cfg, self.device, s_len)

    def close(self, stream_id: int) -> None:
        """Forget a stream whose frames have all been integrated."""
        self._take_arrivals()
        s = self.streams[stream_id]
        if s.pending or s.waiting or s.frames_in:
            raise RuntimeError(f"stream {stream_id} still has frames")
        self.sync()
        self.used -= s.resident_bytes
        del self.streams[stream_id]

    def abort(self, stream_id: int) -> int:
        """A stream that died mid-integration: drop its queued frames and its
        open integration, return their slots, and close it; the other
        streams go on untouched.  Returns the frames dropped, those
        submitted but not yet scheduled included."""
        self._take_arrivals()
        self.sync_launched(stream_id)
        s = self.streams[stream_id]
        dropped = len({id(f) for f in s.waiting} | {id(sl.frame) for sl in s.pending})
        for sl in s.pending:
            if sl.slot >= 0:
                if sl.ev_copied is not None:
                    sl.ev_copied.synchronize()
                self.pool.give(sl.slot)
        s.pending.clear()
        s.waiting.clear()
        s.frames_in = 0
        self._drain_deliveries()
        self.used -= s.resident_bytes
        del self.streams[stream_id]
        return dropped

    def sync_launched(self, stream_id: int) -> None:
        """Wait until every batch launched so far has completed."""
        while self.inflight:
            self.inflight[0][0].synchronize()
            self._complete()

    def _drain_deliveries(self) -> None:
        while self._out_pending > 0:
            time.sleep(50e-6)
        self._raise_delivery_error()

    def _raise_delivery_error(self) -> None:
        err = self._deliver_error
        if err is not None:
            self._deliver_error = None
            raise RuntimeError("delivering an integration result failed") from err

    # -- checkpoint / resume ------------------------------------------------

    def checkpoint(self, path: str) -> None:
        """Write every stream's open integration (sums, counts, samples and
        the integration's bookkeeping) to an .npz file, after serving
        everything submitted so far.  A server with the same streams open
        continues from it with :meth:`resume`."""
        import json
        self.sync()
        arrays, meta = {}, {}
        for sid, s in self.streams.items():
            vis, cnt = s.acc[s.cur]
            snap = xengine.snapshot(vis, cnt, self.compute_stream)
            arrays[f"vis_{sid}"] = snap["vis"]
            arrays[f"count_{sid}"] = snap["count"]
            meta[str(sid)] = {"cfg": dataclasses.asdict(s.cfg), "samples": snap["samples"],
                              "frames_in": s.frames_in, "seq_first": s.seq_first,
                              "seq_last": s.seq_last, "window": s.window, "index": s.index}
        np.savez(path, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **arrays)

    def resume(self, path: str) -> None:
        """Load a checkpoint into the open streams of the same ids and shapes;
        their next frames continue the saved integrations."""
        import json
        self.sync()
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(z["meta"].tobytes().decode())
            for sid_text, m in meta.items():
                sid = int(sid_text)
                s = self.streams.get(sid)
                if s is None or dataclasses.asdict(s.cfg) != m["cfg"]:
                    raise ValueError(f"stream {sid} is not open with the checkpoint's shape")
                vis, cnt = s.acc[s.cur]
                xengine.restore({"vis": z[f"vis_{sid}"], "count": z[f"count_{sid}"],
                                 "samples": m["samples"]}, vis, cnt, self.compute_stream)
                s.frames_in = m["frames_in"]
                s.seq_first, s.seq_last = m["seq_first"], m["seq_last"]
                s.window, s.index = m["window"], m["index"]

    # -- input --------------------------------------------------------------

    def submit(self, frame: Frame) -> None:
        """Hand over a frame in pinned host memory (thread-safe)."""
        if frame.t_arrival <= 0:
            frame.t_arrival = time.perf_counter()
        self.arrivals.put(frame)

    # -- scheduling ---------------------------------------------------------

    def _gpu_time(self, ev) -> float:
        ev_ref, t_ref = self._ref
        return t_ref + ev_ref.elapsed_time(ev) / 1e3

    def _reanchor(self) -> None:
        """Move the clock anchor to a fresh event on a stream with no
        queued work, taking the host time when the host sees it done."""
        now = time.perf_counter()
        if self._anchor is None:
            if now - self._ref[1] >= self._anchor_period:
                ev = self.torch.cuda.Event(enable_timing=True)
                ev.record(self.d2h_stream)
                self._anchor = ev
        elif self._anchor.query():
            self._ref = (self._anchor, now)
            self._anchor = None

    def clock_offset(self) -> float:
        """Host time minus the GPU-clock time of an event recorded and
        waited for now: the error of the current anchor (seconds)."""
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.d2h_stream)
        ev.synchronize()
        return time.perf_counter() - self._gpu_time(ev)

    def _take_arrivals(self) -> None:
        """Move the frames handed over by :meth:`submit` to their streams'
        queues."""
        while True:
            try:
                fr = self.arrivals.get_nowait()
            except queue.Empty:
                return
            s = self.streams.get(fr.stream_id)
            if s is None:
                raise KeyError(f"frame for unopened stream {fr.stream_id}")
            fr.slices = -(-s.cfg.T // s.slice_samples)
            s.waiting.append(fr)

    def _admit(self) -> None:
        torch = self.torch
        self._take_arrivals()
        # slices of the oldest frame first, across streams, while slots last
        while True:
            head = [(s.waiting[0].t_arrival, sid) for sid, s in self.streams.items()
                    if s.waiting]
            if not head:
                return
            _, sid = min(head)
            s = self.streams[sid]
            fr = s.waiting[0]
            cfg = s.cfg
            if fr.packed.is_cuda:
                # already in HBM: the whole frame as one slice, nothing to copy
                s.waiting.popleft()
                fr.slices = fr.copied = 1
                s.pending.append(_Slice(fr, 0, cfg.T, fr.packed, fr.mask, None))
                continue
            k = self.pool.take()
            if k < 0:
                self.admission_waits += 1
                return          # no slot: wait for a batch to finish
            j = fr.copied
            t0 = j * s.slice_samples
            t1 = min(cfg.T, t0 + s.slice_samples)
            dp = self.pool.packed(k, (t1 - t0, cfg.F, cfg.N))
            dm = None
            if fr.mask is not None:
                b0, b1 = t0 // cfg.B, -(-t1 // cfg.B)
                hm = self.pool.mask(k, (cfg.F, b1 - b0), host=True)
                hm.copy_(fr.mask[:, b0:b1])     # host to pinned host, a few KB
                dm = self.pool.mask(k, (cfg.F, b1 - b0))
            with torch.cuda.stream(self.copy_stream):
                if j == 0:
                    fr.ev_copy_start = torch.cuda.Event(enable_timing=True)
                    fr.ev_copy_start.record(self.copy_stream)
                    fr.t_copy_issue = time.perf_counter()
                dp.copy_(fr.packed[t0:t1], non_blocking=True)
                if dm is not None:
                    dm.copy_(hm, non_blocking=True)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.copy_stream)
            fr.copied += 1
            if fr.copied == fr.slices:
                fr.ev_copied = ev
                s.waiting.popleft()
            s.pending.append(_Slice(fr, t0, t1, dp, dm, ev, k))

    def _launch(self) -> bool:
        torch = self.torch
        if len(self.inflight) >= self.max_inflight:
            return False
        batch = []
        for sid, s in self.streams.items():
            if s.pending and (s.pending[0].ev_copied is None or s.pending[0].ev_copied.query()):
                batch.append((s, s.pending.popleft()))
        if not batch:
            return False
        cs = self.compute_stream
        items = []
        for s, sl in batch:
            fr = sl.frame
            if s.cfg.aligned and fr.launched == 0:
                w = fr.seq // s.cfg.frames_per_integration
                if s.frames_in and w != s.window:
                    # a frame of a later window: the current one is over,
                    # short of the frames that never came
                    self._finish(s)
                s.window = w
            if sl.ev_copied is not None:
                cs.wait_event(sl.ev_copied)
            vis, cnt = s.acc[s.cur]
            items.append((sl.packed, sl.mask, s.cfg.B, vis, cnt))
        xengine.accumulate_batch(items, handle=self.h, stream=cs)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(cs)
        self.inflight.append((ev, [sl for _, sl in batch]))
        self.batches += 1
        self.batch_sizes.append(len(batch))
        # frames whose last slice this batch takes, and the integrations they
        # complete
        for s, sl in batch:
            fr = sl.frame
            fr.launched += 1
            if fr.launched < fr.slices:
                continue
            if s.frames_in == 0:
                s.seq_first = fr.seq
            s.seq_last = fr.seq
            s.frames_in += 1
            L = s.cfg.frames_per_integration
            if s.cfg.aligned:
                if (fr.seq + 1) % L == 0:      # the window's last frame
                    self._finish(s)
            elif s.frames_in >= L:
                self._finish(s)
        return True

    def _finish(self, s: _Stream) -> None:
        """End stream s's integration: normalise it, copy it out, and switch
        the stream to its other accumulator (all on the compute stream)."""
        torch = self.torch
        cs = self.compute_stream
        k = s.cur
        vis, cnt = s.acc[k]
        xengine.normalize(vis, cnt, s.out[k], handle=self.h, stream=cs)
        ev_norm = torch.cuda.Event()
        ev_norm.record(cs)
        # the host copy of buffer k (two integrations ago) must have been
        # taken: its copy-out is long done, collect it
        if s.host_busy[k]:
            s.host_free[k].wait()      # delivered long ago, in practice
        s.host_busy[k] = True
        s.host_free[k].clear()
        hv, hc, ho = s.host[k]
        self.d2h_stream.wait_event(ev_norm)
        with torch.cuda.stream(self.d2h_stream):
            hv.copy_(vis, non_blocking=True)
            hc.copy_(cnt, non_blocking=True)
            ho.copy_(s.out[k], non_blocking=True)
            ev_d2h = torch.cuda.Event(enable_timing=True)
            ev_d2h.record(self.d2h_stream)
        s.ev_d2h[k] = ev_d2h
        with self._out_lock:
            self._out_pending += 1
        self._out_q.put((ev_d2h, s, k, s.index, s.frames_in,
                         (s.seq_first, s.seq_last, s.window if s.cfg.aligned else -1)))
        s.index += 1
        s.frames_in = 0
        s.cur ^= 1
        nk = s.cur
        # the other accumulator starts from zero once its last copy-out has
        # read it
        if s.ev_d2h[nk] is not None:
            cs.wait_event(s.ev_d2h[nk])
        with torch.cuda.stream(cs):
            s.acc[nk][0].zero_()
            s.acc[nk][1].zero_()
            xengine.reset_integration(s.acc[nk][0])

    def flush(self, stream_id: int) -> None:
        """End the stream's open integration now (e.g. the last, partial
        window of an aligned stream); its result arrives as usual."""
        s = self.streams[stream_id]
        self.sync()
        if s.frames_in:
            self._finish(s)
            self.sync()

    def _complete(self) -> int:
        n = 0
        while self.inflight and self.inflight[0][0].query():
            ev, slices = self.inflight.popleft()
            t_done = self._gpu_time(ev)
            for sl in slices:
                if sl.slot >= 0:
                    self.pool.give(sl.slot)
                fr = sl.frame
                cfg = self.streams[fr.stream_id].cfg
                self.bytes_done += (sl.t1 - sl.t0) * cfg.F * cfg.N
                self.samples_done += (sl.t1 - sl.t0) * cfg.F * cfg.N
                fr.done += 1
                if fr.done < fr.slices:
                    continue
                fr.t_done = t_done
                self.latencies.append(t_done - fr.t_arrival)
                if fr.ev_copy_start is not None:
                    t_start = self._gpu_time(fr.ev_copy_start)
                    t_copied = self._gpu_time(fr.ev_copied)
                else:
                    t_start = t_copied = fr.t_arrival
                # waiting before the bytes move, the copy, and the rest
                self.breakdown.append((t_start - fr.t_arrival, t_copied - t_start,
                                       t_done - t_copied))
                self.done_frames.append((fr.stream_id, fr.seq, fr.t_arrival))
                self.frames_done += 1
                fr.packed = fr.mask = None
            n += 1
        return n

    def _deliver(self) -> None:
        """Delivery thread: per finished integration, wait for its copy-out,
        copy it from the pinned buffers (torch copies release the
        interpreter lock), free the buffers and hand the result over.
        An exception (a failing callback, say) is kept for the scheduling
        thread to raise; the buffers are freed and the result counted as
        delivered either way, so nothing waits for it forever."""
        while True:
            ev, s, k, index, frames, (q0, q1, win) = self._out_q.get()
            freed = False
            try:
                ev.synchronize()
                hv, hc, ho = (t.clone() for t in s.host[k])
                res = IntegrationResult(s.cfg.stream_id, index, frames, hv.numpy(), hc.numpy(),
                                        ho.numpy(), self._gpu_time(ev), q0, q1, win)
                # free buffer k before the callback, which may take long; the
                # scheduling thread may then reuse it at once
                s.host_busy[k] = False
                s.host_free[k].set()
                freed = True
                self.results[s.cfg.stream_id].append(res)
                if self.on_result is not None:
                    self.on_result(res)
            except BaseException as e:    # raised again by the scheduling thread
                if self._deliver_error is None:
                    self._deliver_error = e
            finally:
                if not freed:
                    s.host_busy[k] = False
                    s.host_free[k].set()
                with self._out_lock:
                    self._out_pending -= 1

    def step(self) -> bool:
        """One scheduling pass; True if anything happened.  Raises
        RuntimeError if a result could not be delivered."""
        self._raise_delivery_error()
        self._reanchor()
        done = self._complete()
        self._admit()
        launched = False
        while self._launch():
            launched = True
        return bool(done) or launched

    def busy(self) -> bool:
        return (not self.arrivals.empty() or bool(self.inflight) or self._out_pending > 0 or
                any(s.pending or s.waiting for s in self.streams.values()))

    def sync(self) -> None:
        """Run until every submitted frame and finished integration is out."""
        while self.busy():
            if not self.step():
                time.sleep(20e-6)
        self._raise_delivery_error()

    def serve(self, stop: threading.Event, idle_sleep: float = 20e-6) -> None:
        """Scheduling loop until `stop` is set and nothing is left."""
        while not (stop.is_set() and not self.busy()):
            if not self.step():
                time.sleep(idle_sleep)

    # -- reporting ----------------------------------------------------------

    def stats(self, wall_s: float) -> dict:
        lat = np.array(self.latencies) * 1e3
        bd = np.array(self.breakdown).reshape(-1, 3) * 1e3
        parts = {}
        if bd.size:
            slow = bd[lat >= np.percentile(lat, 99)]
            for k, name in enumerate(("wait", "copy", "finish")):
                parts[name] = {"p50_ms": float(np.percentile(bd[:, k], 50)),
                               "p99_ms": float(np.percentile(bd[:, k], 99)),
                               "mean_in_slowest_1pct_ms": float(slow[:, k].mean())}
        return {
            "latency_breakdown": parts,
            "frames": self.frames_done,
            "batches": self.batches,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "max_ms": float(lat.max()) if lat.size else None,
            "gbps": 8.0 * self.samples_done / wall_s / 1e9 if wall_s > 0 else 0.0,
            "hbm_budget": self.budget,
            "hbm_peak_used": self.max_used,
            "admission_waits": self.admission_waits,
        }


# ---------------------------------------------------------------------------
# combining streams
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class CombinedIntegration:
    """The integrations of several streams of one correlator over the same
    sequence-number window, joined channel-wise in stream-id order."""
    window: int
    stream_ids: List[int]        # in channel order
    channel_offsets: List[int]   # first channel of each stream
    frames: List[int]            # frames each stream integrated
    seq_first: int               # first and last frame sequence number seen
    seq_last: int
    vis: np.ndarray              # int32 [sum F][P][2]
    count: np.ndarray            # int64 [sum F]
    out: np.ndarray              # float32 [sum F][P][2]

    def save(self, path: str) -> None:
        """Dump to a .npz file: the three arrays plus the window, the stream
        ids with their channel offsets and frame counts, and the sequence
        range."""
        np.savez(path, vis=self.vis, count=self.count, out=self.out,
                 window=np.int64(self.window), stream_ids=np.asarray(self.stream_ids),
                 channel_offsets=np.asarray(self.channel_offsets),
                 frames=np.asarray(self.frames),
                 seq=np.asarray([self.seq_first, self.seq_last], dtype=np.int64))


class Combiner:
    """Joins the aligned integrations of the streams of one correlator (the
    same N, each stream its own channels), as the post-processing stage
    combines the streams of a host: results are held per sequence-number
    window until every stream has delivered that window, then concatenated
    along the channel axis in increasing stream id.  Use ``add`` as the
    server's ``on_result`` callback."""

    def __init__(self, stream_ids, on_combined: Optional[Callable] = None):
        self.ids = sorted(int(x) for x in stream_ids)
        if len(set(self.ids)) != len(self.ids) or not self.ids:
            raise ValueError("stream ids must be distinct and not empty")
        self.on_combined = on_combined
        self.held: Dict[int, Dict[int, IntegrationResult]] = {}
        self.combined: List[CombinedIntegration] = []

    def add(self, res: IntegrationResult) -> Optional[CombinedIntegration]:
        if res.stream_id not in self.ids:
            raise KeyError(f"stream {res.stream_id} is not combined here")
        if res.window < 0:
            raise ValueError("combining needs sequence-aligned streams (StreamConfig.aligned)")
        parts = self.held.setdefault(res.window, {})
        if res.stream_id in parts:
            raise ValueError(f"stream {res.stream_id} delivered window {res.window} twice")
        parts[res.stream_id] = res
        if len(parts) < len(self.ids):
            return None
        del self.held[res.window]
        c = self._join(res.window, [parts[i] for i in self.ids])
        self.combined.append(c)
        if self.on_combined is not None:
            self.on_combined(c)
        return c

    def incomplete(self) -> Dict[int, List[int]]:
        """Windows still waiting, with the streams that have not delivered."""
        return {w: [i for i in self.ids if i not in parts] for w, parts in self.held.items()}

    @staticmethod
    def _join(window: int, parts: List[IntegrationResult]) -> CombinedIntegration:
        P = parts[0].vis.shape[1]
        if any(r.vis.shape[1] != P for r in parts):
            raise ValueError("combined streams must have the same number of inputs")
        offsets, off = [], 0
        for r in parts:
            offsets.append(off)
            off += r.vis.shape[0]
        return CombinedIntegration(
            window=window, stream_ids=[r.stream_id for r in parts], channel_offsets=offsets,
            frames=[r.frames for r in parts],
            seq_first=min(r.seq_first for r in parts), seq_last=max(r.seq_last for r in parts),
            vis=np.concatenate([r.vis for r in parts]),
            count=np.concatenate([r.count for r in parts]),
            out=np.concatenate([r.out for r in parts]))


# ---------------------------------------------------------------------------
# offered load
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class LoadResult:
    server: StreamServer
    stats: dict
    frames: Dict[int, list]          # per stream: the distinct frames (synth.Frame)
    sequence: Dict[int, List[int]]   # per stream: pool index of each frame, in order


def _frame_pool(specs, distinct: int, B: int):
    """``distinct`` frames per stream: one generated, the others derived
    from it (synth.stream_frame_variant), which costs a copy rather than
    a fresh draw of Gaussian noise."""
    from . import synth
    out = {}
    for s in specs:
        base = synth.stream_frame(s, 0, B)
        out[s.stream_id] = [base] + [synth.stream_frame_variant(s, base, k)
                                     for k in range(1, distinct)]
    return out


def run_load(specs, frames_per_stream: Optional[int] = None, integrations: int = 1,
             speed: float = 1.0, hbm_budget: int = 2 << 30, distinct: int = 2,
             duration: Optional[float] = None,
             B: int = 256, device: int = 0, max_inflight: int = 2,
             device_resident: bool = False, seed: int = 0, pool=None,
             handle: Optional[xengine.Handle] = None, slot_bytes: int = 32 << 20,
             pool_bytes: Optional[int] = None,
             slice_samples: Optional[int] = None) -> LoadResult:
    """Offer each stream's frames with Poisson arrivals at ``speed`` times
    its rate (``speed`` = inf: all at once) and serve them.

    Each stream sends ``frames_per_stream`` frames (default: ``integrations``
    whole integrations; with ``duration``: as many as its rate offers in that
    many seconds, at the arrival times of a Poisson process given that
    count, i.e. sorted uniform times over the duration, so that the realised
    rate matches the offered one), cycling through ``distinct`` frames.
    ``device_resident``: the frames are already in HBM (no host link), to
    measure the serving loop's own sustained rate.  ``slot_bytes``,
    ``pool_bytes`` and ``slice_samples`` configure the server's frame pool
    and time slices."""
    import torch
    pool = pool or _frame_pool(specs, distinct, B)
    dev = torch.device("cuda", device)
    tens = {}
    for s in specs:
        lst = []
        for fr in pool[s.stream_id]:
            p = torch.from_numpy(fr.packed)
            m = torch.from_numpy(fr.mask)
            if device_resident:
                lst.append((p.to(dev), m.to(dev)))
            else:
                lst.append((p.pin_memory(), m.pin_memory()))
        tens[s.stream_id] = lst
    torch.cuda.synchronize(dev)
    rng = np.random.default_rng(seed)
    arrivals = []
    sequence = {}
    for s in specs:
        rate = s.frame_rate * speed
        if duration is not None and np.isfinite(rate):
            n = max(1, int(round(rate * duration)))
            t = np.sort(rng.uniform(0.0, duration, n))
        else:
            n = frames_per_stream or integrations * s.frames_per_integration
            gaps = (rng.exponential(1.0 / rate, n) if np.isfinite(rate) else np.zeros(n))
            t = np.cumsum(gaps)
        k_pool = len(tens[s.stream_id])
        sequence[s.stream_id] = [k % k_pool for k in range(n)]
        arrivals += [(float(t[k]), s.stream_id, k) for k in range(n)]
    arrivals.sort()
    server = StreamServer(hbm_budget, device, max_inflight, handle, slot_bytes=slot_bytes,
                          pool_bytes=pool_bytes, slice_samples=slice_samples)
    for s in specs:
        server.open(StreamConfig(s.stream_id, s.N, s.F, s.T, B, s.frames_per_integration))
    stop = threading.Event()

    late = []

    def produce():
        # a frame's arrival is its scheduled Poisson time, so that time the
        # producer spends behind schedule counts as queueing delay
        t0 = time.perf_counter()
        for t_off, sid, k in arrivals:
            due = t0 + t_off
            delay = due - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            p, m = tens[sid][sequence[sid][k]]
            late.append(max(0.0, time.perf_counter() - due))
            server.submit(Frame(sid, k, p, m, due))
        stop.set()

    prod = threading.Thread(target=produce, daemon=True)
    # the producer and the scheduling loop share the interpreter: hand the
    # lock over every 100 us rather than every 5 ms, so that a frame is not
    # handed over milliseconds late while the loop polls its events
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    t_start = time.perf_counter()
    try:
        prod.start()
        server.serve(stop)
        prod.join()
    finally:
        sys.setswitchinterval(switch)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t_start
    st = server.stats(wall)
    st["wall_s"] = wall
    st["clock_offset_ms"] = server.clock_offset() * 1e3
    st["offered_gbps"] = (sum(s.rate_bps for s in specs) * speed / 1e9
                          if np.isfinite(speed) else None)
    # what the draw actually offered: its bytes over the span of the
    # arrivals (the duration when given)
    span = duration if duration is not None else (arrivals[-1][0] if arrivals else 0.0)
    bits = sum(8.0 * s.N * s.F * s.T * len(sequence[s.stream_id]) for s in specs)
    st["offered_realized_gbps"] = bits / span / 1e9 if span > 0 else None
    st["arrival_span_s"] = span
    st["device_resident"] = device_resident
    if late:
        lt = np.array(late) * 1e3
        st["submit_late_p50_ms"] = float(np.percentile(lt, 50))
        st["submit_late_p99_ms"] = float(np.percentile(lt, 99))
    return LoadResult(server, st, pool, sequence)


def run_plain(specs, pool, frames_per_stream: int, B: int = 256, device: int = 0,
              handle: Optional[xengine.Handle] = None) -> dict:
    """The same frames, device-resident, one plain xe_accumulate launch per
    frame in arrival order: the baseline the batched server must beat."""
    import torch
    dev = torch.device("cuda", device)
    h = handle or xengine.default_handle(device)
    acc = {s.stream_id: xengine.new_accumulators(s.N, s.F, dev) for s in specs}
    tens = {s.stream_id: [(torch.from_numpy(f.packed).to(dev), torch.from_numpy(f.mask).to(dev))
                          for f in pool[s.stream_id]] for s in specs}
    order = [(k, s.stream_id) for k in range(frames_per_stream) for s in specs]
    samples = sum(s.N * s.F * s.T for s in specs) * frames_per_stream

    def once():
        for k, sid in order:
            p, m = tens[sid][k % len(tens[sid])]
            vis, cnt = acc[sid]
            xengine.accumulate(p, m, B, vis, cnt, handle=h)

    once()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    once()
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    return {"frames": len(order), "wall_s": wall, "gbps": 8.0 * samples / wall / 1e9}
