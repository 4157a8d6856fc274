"""Serving loop: continuous batching of lattice jobs on one GPU.

Thin binding of the su3_server_* entry points of the C ABI plus the loop
that feeds a timed job stream into the server.  The server (native, in the
library) admits jobs by HBM footprint inside one caller-owned arena, runs
batched sweeps of every admitted job (one per su3_server_step, up to a given
number per su3_server_run) and retires finished jobs; the feeding loop only
submits arrivals, runs the server and records times.
"""
import ctypes as C
import time

import numpy as np

from . import su3hb as _hb


class su3_job(C.Structure):
    _fields_ = [("params", _hb.su3_params), ("beta", C.c_double), ("nsweeps", C.c_int32), ("hot", C.c_int32)]


class su3_job_result(C.Structure):
    _fields_ = [("state", C.c_int32), ("sweeps_done", C.c_int32), ("plaquette", C.c_double * 3),
                ("kp_attempts", C.c_uint64), ("kp_accepts", C.c_uint64), ("bad_links", C.c_int64)]


QUEUED, ACTIVE, DONE = 0, 1, 2

_lib = _hb.lib()
_st, _vp = C.c_int, C.c_void_p
for _name, _res, _args in (
        ("su3_server_create", _st, [_vp, C.c_size_t, C.c_int32, _vp, C.POINTER(_vp)]),
        ("su3_server_submit", _st, [_vp, C.POINTER(su3_job), C.POINTER(C.c_int64)]),
        ("su3_server_step", _st, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        ("su3_server_run", _st, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        ("su3_server_poll", _st, [_vp, C.c_int64, C.POINTER(su3_job_result)]),
        ("su3_server_release", _st, [_vp, C.c_int64]),
        ("su3_server_get_links", _st, [_vp, C.c_int64, C.POINTER(C.c_double), C.c_size_t]),
        ("su3_server_stats", _st, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_uint64)]),
        ("su3_server_destroy", _st, [_vp])):
    _f = getattr(_lib, _name)
    _f.restype, _f.argtypes = _res, _args


def make_job(L, beta, nsweeps, seed, precision=32, nlat=1, flip_mask=None, nhit=1, hot=1):
    j = su3_job()
    j.params = _hb.make_params(L, nlat=nlat, flip_mask=flip_mask, precision=precision, nhit=nhit, seed=seed)
    j.beta, j.nsweeps, j.hot = float(beta), int(nsweeps), int(hot)
    return j


class Server:
    """A job server over a torch-allocated device arena of `arena_bytes`."""

    def __init__(self, arena_bytes, max_active=256, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the job server needs a GPU")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p(0)
        _hb._check(_lib.su3_server_create(C.c_void_p(self.arena.data_ptr()), int(arena_bytes), int(max_active),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)), "su3_server_create")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            _lib.su3_server_destroy(h)
            self.h = None

    def submit(self, job):
        jid = C.c_int64(0)
        _hb._check(_lib.su3_server_submit(self.h, C.byref(job), C.byref(jid)), "su3_server_submit")
        return jid.value

    def step(self):
        a, q, f = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _hb._check(_lib.su3_server_step(self.h, C.byref(a), C.byref(q), C.byref(f)), "su3_server_step")
        return a.value, q.value, f.value

    def run(self, max_sweeps):
        """su3_server_run: up to max_sweeps sweeps of every admitted job, one synchronisation."""
        a, q, f = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _hb._check(_lib.su3_server_run(self.h, int(max_sweeps), C.byref(a), C.byref(q), C.byref(f)),
                   "su3_server_run")
        return a.value, q.value, f.value

    def poll(self, jid):
        r = su3_job_result()
        _hb._check(_lib.su3_server_poll(self.h, int(jid), C.byref(r)), "su3_server_poll")
        return {"state": r.state, "sweeps_done": r.sweeps_done, "plaquette": list(r.plaquette),
                "kp_attempts": r.kp_attempts, "kp_accepts": r.kp_accepts, "bad_links": r.bad_links}

    def release(self, jid):
        """su3_server_release: drop a finished job's record."""
        _hb._check(_lib.su3_server_release(self.h, int(jid)), "su3_server_release")

    def get_links(self, jid, n_doubles):
        """su3_server_get_links: an active job's links, canonical FP64 layout, shape (n_doubles // 18, 18)."""
        out = np.empty(int(n_doubles), dtype=np.float64)
        _hb._check(_lib.su3_server_get_links(self.h, int(jid), out.ctypes.data_as(C.POINTER(C.c_double)),
                                             out.size), "su3_server_get_links")
        return out.reshape(-1, 18)

    def stats(self):
        u, p, s = C.c_size_t(0), C.c_size_t(0), C.c_uint64(0)
        _hb._check(_lib.su3_server_stats(self.h, C.byref(u), C.byref(p), C.byref(s)), "su3_server_stats")
        return {"arena_used": u.value, "arena_peak": p.value, "steps": s.value}


def _volume(L):
    return int(np.prod(L)) if isinstance(L, (tuple, list)) else int(L) ** 4


def run_stream(jobs, arena_bytes=4 << 30, max_active=256, realtime=True, sweeps_per_call=8):
    """Feed `jobs` (dicts from workloads.serving_stream) into a server.

    realtime: a job is submitted once the wall clock passes its arrival time;
    otherwise everything is submitted at once.  Each server call runs up to
    `sweeps_per_call` sweeps (su3_server_run), so the per-call launch and
    synchronisation cost is shared by several sweeps.  Returns (records,
    summary): per job its arrival, completion and latency (seconds since the
    stream started) and final plaquette/counters."""
    srv = Server(arena_bytes, max_active)
    order = sorted(jobs, key=lambda j: j["arrival"])
    ids, recs, pending = {}, {}, set()
    nxt, done = 0, 0
    t0 = time.perf_counter()
    while done < len(order):
        now = time.perf_counter() - t0
        while nxt < len(order) and (not realtime or order[nxt]["arrival"] <= now):
            j = order[nxt]
            jid = srv.submit(make_job(j["L"], j["beta"], j["nsweeps"], j["seed"], j["precision"], j.get("nlat", 1),
                                      j.get("flip_mask"), j.get("nhit", 1), j.get("hot", 1)))
            ids[jid] = j
            pending.add(jid)
            recs[j["id"]] = {"arrival": j["arrival"] if realtime else 0.0, "submitted": now}
            nxt += 1
        active, queued, finished = srv.run(sweeps_per_call)
        if finished:
            t = time.perf_counter() - t0
            for jid in sorted(pending):
                res = srv.poll(jid)
                if res["state"] == DONE:
                    r = recs[ids[jid]["id"]]
                    r.update(res)
                    r["done"] = t
                    r["latency"] = t - r["arrival"]
                    srv.release(jid)  # the server keeps no record of it from here on
                    pending.discard(jid)
                    done += 1
        if active == 0 and queued == 0 and nxt < len(order):
            time.sleep(max(0.0, order[nxt]["arrival"] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    lat = np.array([recs[j["id"]]["latency"] for j in order])
    updates = sum(4 * _volume(j["L"]) * j.get("nlat", 1) * j["nsweeps"] for j in order)
    st = srv.stats()
    summary = {"jobs": len(order), "wall_s": wall, "p50_latency_s": float(np.percentile(lat, 50)),
               "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
               "max_latency_s": float(lat.max()), "link_updates": int(updates),
               "throughput_updates_per_s": updates / wall, "arena_bytes": int(arena_bytes),
               "arena_peak_bytes": st["arena_peak"], "max_active": max_active, "steps": st["steps"],
               "sweeps_per_call": sweeps_per_call}
    return recs, summary


def run_stream_benchmark(n_jobs=256, rate=20.0, seed=0, arena_bytes=4 << 30, max_active=256):
    """The mixed stream of the serving workload: 256 jobs, L in {8..24},
    beta in [5.5, 6.2], 50-500 sweeps, Poisson arrivals at 20 jobs/s, FP32."""
    from .workloads import serving_stream

    jobs = serving_stream(n_jobs=n_jobs, rate=rate, seed=seed, precision=32)
    _, summary = run_stream(jobs, arena_bytes=arena_bytes, max_active=max_active, realtime=True)
    summary["workload"] = (f"{n_jobs} jobs, L uniform in (8,10,12,16,20,24), beta uniform in [5.5,6.2], "
                           f"50-500 sweeps, Poisson arrivals at {rate}/s, FP32 links, hot start")
    return summary
