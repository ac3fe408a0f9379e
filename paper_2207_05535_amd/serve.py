"""Continuous-batching request loop over the native server (``pa_server_*``).

A request is one PA run (a descriptor).  The loop replays an arrival trace
in real time: arrived requests wait in FIFO order and are admitted while a
slot is free and their footprint fits in the server's device arena; every
tick enqueues one temperature step for all resident runs (one set of shared
launches); runs that reach their last temperature have their records copied
to pinned host memory and their slot and memory released at once, so the
next waiting request can be admitted on the following tick while the others
keep running.  Completion is observed through an event recorded after the
tick, so the host stays at most ``max_inflight`` ticks ahead of the device.

Only argument marshalling and bookkeeping happen here; admission,
allocation, work lists and every kernel live in ``libpa.so``.
"""
from __future__ import annotations

import collections
import math
import time

import numpy as np

from . import (PA_OBS_DTYPE, PA_Q_TWO_POP, pa_server_admit, pa_server_create, pa_server_destroy,
               pa_server_footprint, pa_server_info, pa_server_read_obs, pa_server_release,
               pa_server_step)


class Server:
    """A pa_server over a torch-allocated device arena and torch's current
    stream (or the one given)."""

    def __init__(self, arena_bytes, max_slots=16, repr_="msc", tuning_cache=None, device="cuda",
                 stream=None):
        import torch
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.arena.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        self.repr = repr_
        self.max_slots = max_slots
        self.h = pa_server_create(repr_, ptr, arena_bytes, max_slots, tuning_cache, self.stream.cuda_stream)
        self._fin = np.zeros(max_slots, np.int32)

    def footprint(self, desc):
        return pa_server_footprint(desc, self.repr)

    def admit(self, desc):
        return pa_server_admit(self.h, desc)

    def step(self):
        return pa_server_step(self.h, self._fin)

    def read_obs(self, slot, desc, sync=True):
        """Records of a resident run as [K][n_pop]; with sync=False returns
        (pinned tensor, view) and the caller must wait for the stream."""
        import torch
        npop = 2 if desc["overlap"] == PA_Q_TWO_POP else 1
        n = len(desc["beta"]) * npop
        buf = torch.empty(n * PA_OBS_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
        pa_server_read_obs(self.h, slot, buf.data_ptr(), sync)
        view = buf.numpy().view(PA_OBS_DTYPE).reshape(len(desc["beta"]), npop)
        return view if sync else (buf, view)

    def release(self, slot):
        pa_server_release(self.h, slot)

    def info(self):
        return pa_server_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            pa_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_flips(obs, desc):
    """Attempted flips of a finished run: sum over steps i >= 1 of theta R_i N
    (both populations for two-population runs); none at theta = infinity,
    where energies are drawn instead of sweeping."""
    N = desc["L"] ** 2
    return int(obs["R_i"][1:].sum()) * max(desc["theta"], 0) * N


def replay(server, trace, time_scale=1.0, max_inflight=2, clock=time.perf_counter, progress=None):
    """Replays [(t_arrival_s, desc)] against ``server``; arrival times are
    multiplied by ``time_scale`` (0: everything arrives at once).  Returns
    (records, summary): per request its arrival, admission and finish times
    (s from the start), latency, flips and records; the summary holds the
    latency percentiles, achieved flips/ns over the whole replay and over
    the device-busy ticks, and the peak residency."""
    import torch
    n = len(trace)
    order = sorted(range(n), key=lambda q: trace[q][0])
    arrivals = collections.deque(order)
    waiting = collections.deque()
    active = {}                       # slot -> request
    inflight = collections.deque()    # (start event, end event, [(request, pinned buf, view)])
    rec = [dict(arrival=trace[q][0] * time_scale, admit=None, finish=None) for q in range(n)]
    busy_s = 0.0
    peak = 0
    done = 0
    stream = server.stream
    t0 = clock()

    def retire(block):
        nonlocal done, busy_s
        while inflight and (block or len(inflight) > max_inflight or inflight[0][1].query()):
            ev0, ev1, batch = inflight.popleft()
            ev1.synchronize()
            busy_s += ev0.elapsed_time(ev1) / 1e3
            t = clock() - t0
            for q, buf, view in batch:
                rec[q]["finish"] = t
                rec[q]["obs"] = view.copy()
                del buf
                done += 1
                if progress:
                    progress(done, n, t)
            block = False

    while done < n:
        now = clock() - t0
        while arrivals and rec[arrivals[0]]["arrival"] <= now:
            waiting.append(arrivals.popleft())
        while waiting:
            q = waiting[0]
            slot = server.admit(trace[q][1])
            if slot is None:
                break
            waiting.popleft()
            active[slot] = q
            rec[q]["admit"] = clock() - t0
        peak = max(peak, len(active))
        if active:
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            fin = server.step()
            batch = []
            for slot in fin:
                q = active.pop(slot)
                buf, view = server.read_obs(slot, trace[q][1], sync=False)
                server.release(slot)
                batch.append((q, buf, view))
            ev1.record(stream)
            inflight.append((ev0, ev1, batch))
            retire(False)
        elif inflight:
            retire(True)
        elif arrivals:
            time.sleep(max(0.0, rec[arrivals[0]]["arrival"] - (clock() - t0)))
        elif waiting:
            raise RuntimeError("a waiting request can never be admitted (footprint exceeds the arena)")
    for q in range(n):
        d = trace[q][1]
        rec[q]["latency"] = rec[q]["finish"] - rec[q]["arrival"]
        rec[q]["flips"] = run_flips(rec[q]["obs"], d)
        rec[q]["L"] = d["L"]
    lat = sorted(r["latency"] for r in rec)
    flips = sum(r["flips"] for r in rec)
    span = max(r["finish"] for r in rec) - min(r["arrival"] for r in rec)

    def pct(p):
        k = (len(lat) - 1) * p
        f = math.floor(k)
        c = min(f + 1, len(lat) - 1)
        return lat[f] + (lat[c] - lat[f]) * (k - f)

    summary = dict(requests=n, p50_s=pct(0.5), p99_s=pct(0.99), mean_s=sum(lat) / n, max_s=lat[-1],
                   flips=flips, span_s=span, flips_per_ns=flips / span / 1e9,
                   busy_s=busy_s, busy_flips_per_ns=flips / busy_s / 1e9 if busy_s > 0 else None,
                   peak_resident=peak)
    return rec, summary
