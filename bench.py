#!/usr/bin/env python3
"""Throughput of the checkerboard SU(3) heat-bath sweep on one MI355X.

Workload (default): a 32^4 periodic lattice, beta = 5.7, FP64 links, hot
(Haar-random) start from Philox seed 1, 1-hit heat bath.  One step = one sweep
(8 checkerboard passes, 4 * 32^4 link updates) followed by one plaquette
measurement (su3_sweep_measure: the plaquette of every sweep is reduced on the
GPU and copied back once at the end).  `value` is link updates per second over the timed steps, with
the lattice already resident in HBM.  The start configuration is created
before the timed region, as the paper excludes it from its timings (Sec. 2).

Also reported on the same JSON line:
  roofline      the heat-bath pass kernel against HBM bandwidth, timed with
                HIP events on the library's stream around one pass launch per
                sweep, rotating through the eight passes of a sweep
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
  fp32          the FP32-link tier on the same workload and its plaquette
                deviation from the FP64 chain
  serving       the mixed job stream through the job server: p50/p99 latency
                (arrival to completion) and throughput
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
REAL_BYTES = {64: 8, 32: 4}
# Algorithmic bytes of one link update in a pass: the pass reads every link of
# the lattice once (8 link reads per updated link) and writes the updated
# link, 9 link transfers of an SU(3) matrix of 18 reals (the paper's storage).
# The roofline fraction is taken against this figure.  This library stores a
# link as its rows 0 and 1 (12 reals, row 2 rebuilt), so the bytes it must
# move are 9 x 12 reals; that figure is reported beside it as "stored".
LINK_REALS, STORED_REALS, TRANSFERS_PER_UPDATE = 18, 12, 9


# device warm-up before each of the other configurations' timed sweeps (milliseconds)
CONFIG_WARMUP_MS = 50.0


def bytes_per_update(precision):
    """Algorithmic bytes per link update: 9 transfers of an 18-real link."""
    return TRANSFERS_PER_UPDATE * LINK_REALS * REAL_BYTES[precision]


def stored_bytes_per_update(precision):
    """Bytes per link update with 12-real storage: 9 transfers of rows 0 and 1."""
    return TRANSFERS_PER_UPDATE * STORED_REALS * REAL_BYTES[precision]


PROFILE_DIR = os.path.join(ROOT, "profiles")
# what the pass kernel's counters depend on: its code, its launch shape, the
# pass order the host picks and the compiler flags
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0904_1179_amd", "csrc", f)
                  for f in ("kernels.hip", "device.h", "geom.h", "launch.h", "layout.cpp", "api.hip")] + \
                 [os.path.join(ROOT, "paper_0904_1179_amd", "build.py")]


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank lines removed, so
    that stored counter figures stay valid across comment-only edits."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        text = re.sub(r"/\*.*?\*/", "", open(p).read(), flags=re.S)
        for line in text.splitlines():
            code = re.sub(r"//.*", "", line).strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def stored_traffic(name):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current kernel source."""
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_gpu(L, precision, steps, warmup, beta, seed=1, device_warmup_ms=0.0):
    import torch

    from paper_0904_1179_amd import Lattice

    lat = Lattice(L, nlat=1, precision=precision, seed=seed)
    lat.start(hot=True)
    warmed_ms = device_warmup(device_warmup_ms, L, precision, beta)
    if warmup > 0:
        lat.sweep_measure(warmup, beta)
    torch.cuda.synchronize()
    lat.profile(True)
    lat.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plaq = [float(p) for p in lat.sweep_measure(steps, beta)[:, 0]]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pass_ms, passes = lat.profile_read()
    lat.profile(False)
    # the last fused measurement against the full plaquette kernel (after the timed region)
    full = float(lat.plaquette()[0])
    V = L ** 4
    return {"seconds": t1 - t0, "updates": 4 * V * steps, "pass_ms": pass_ms / max(passes, 1), "passes": passes,
            "plaquette": plaq, "plaquette_full_kernel": full, "lattice": lat, "device_warmup_ms": warmed_ms}


def repeat_rates(lat, beta, repeats=10, sweeps=10):
    """Spread of the sweep rate: `repeats` fresh hot starts of the same
    lattice, each followed by `sweeps` sweeps timed with HIP events on the
    lattice's stream (su3_sweep, no measurement)."""
    import numpy as np
    import torch

    rates = []
    for _ in range(repeats):
        lat.start(hot=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.sweep(sweeps, beta)
        e1.record(lat.stream)
        e1.synchronize()
        rates.append(4 * lat.V * lat.nlat * sweeps / (e0.elapsed_time(e1) * 1e-3))
    r = np.sort(np.array(rates))
    return {"repeats": repeats, "sweeps_each": sweeps, "median": float(np.median(r)),
            "p10": float(np.percentile(r, 10)), "p90": float(np.percentile(r, 90)), "unit": "link updates/s",
            "timing": "HIP events around su3_sweep on the lattice's stream, each from a fresh hot start"}


def device_warmup(ms, L, precision, beta, nlat=1, flip_mask=None, measure=False, betas=None):
    """Keep the GPU busy for `ms` milliseconds with the workload's own pass
    kernels, on a scratch lattice of the same shape and precision (hot start,
    discarded afterwards; the timed lattice's chain is not touched): sweeps,
    sweeps with the plaquette (measure) or sweeps with two couplings (betas).  On a
    GPU that was idle, or that ran other kernels, the passes of the first
    ~25 ms of sustained load run up to 30 % slower (they start at full speed,
    slow down after ~2 ms and recover over ~20 ms; a second lattice allocated
    later runs at full speed from its first sweep, so the effect follows the
    device's load history, not the allocation; a warm-up with the copy kernel
    left the timed steps ~3 % slower than one with the pass kernels).  It is
    not part of the workload and not in the timed region."""
    import torch

    from paper_0904_1179_amd import Lattice

    if ms <= 0:
        return 0.0
    lat = Lattice(L, nlat=nlat, precision=precision, seed=0x5eed, flip_mask=flip_mask)
    lat.start(hot=True)

    def run(n):
        if betas is not None:
            lat.sweep_betas(n, *betas)
        elif measure:
            lat.sweep_measure(n, beta)
        else:
            lat.sweep(n, beta)

    run(1)
    torch.cuda.synchronize()  # start the clock after the first sweep: lazy start-up costs are not GPU load
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < ms * 1e-3:
        run(4)
        torch.cuda.synchronize()
    del lat
    return (time.perf_counter() - t0) * 1e3


def copy_probe_gbs(nbytes=1 << 30, reps=10):
    import torch

    from paper_0904_1179_amd import su3_stream_copy

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    su3_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        su3_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize()
    return 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def fp32_deviation(L, beta, sweeps=2, seed=1):
    """Plaquette of the FP32 tier against the FP64 chain from the same start, per sweep."""
    from paper_0904_1179_amd import Lattice

    a = Lattice(L, precision=64, seed=seed)
    b = Lattice(L, precision=32, seed=seed)
    a.start(hot=True)
    b.start(hot=True)
    out = []
    for _ in range(sweeps):
        a.sweep(1, beta)
        b.sweep(1, beta)
        pa, pb = a.plaquette()[0], b.plaquette()[0]
        out.append(abs(pb - pa) / abs(pa))
    return out


def chain_deviation(p32, p64, bound=1e-5):
    """Per-sweep plaquette relative error of an FP32 chain against the FP64
    chain from the same start: the values, their maximum before the first
    sweep above `bound` (the onset of decorrelation, after which the two
    chains are independent samples) and that onset (1-based; null if none)."""
    import numpy as np

    p32, p64 = np.asarray(p32, dtype=float), np.asarray(p64, dtype=float)
    rel = np.abs(p32 - p64) / np.abs(p64)
    over = np.nonzero(rel > bound)[0]
    onset = int(over[0]) if over.size else None
    before = rel[:onset] if onset is not None else rel
    return {"rel_err_per_sweep": [float(f"{x:.3e}") for x in rel],
            "max_rel_err_before_onset": float(before.max()) if before.size else None,
            "onset_sweep": None if onset is None else onset + 1, "bound": bound}


def config_rate(L, nlat, precision, beta, sweeps, seed=1, flip_mask=None, hot=True, untimed=1, every=True,
                warmup_ms=CONFIG_WARMUP_MS):
    """Link updates/s of `sweeps` sweeps on one more workload configuration,
    after the start, a device warm-up with the same kernels on a scratch
    lattice (these timed regions last only milliseconds) and `untimed`
    untimed sweeps, with the plaquette after every sweep (every=True) or once
    after the last (outside the timed region); also the algorithmic bytes per
    second of the passes and the plaquettes (all sweeps with every=True, kept
    for the FP32 comparison)."""
    import torch

    from paper_0904_1179_amd import Lattice

    lat = Lattice(L, nlat=nlat, precision=precision, seed=seed, flip_mask=flip_mask)
    lat.start(hot=hot)
    device_warmup(warmup_ms, L, precision, beta, nlat=nlat, flip_mask=flip_mask, measure=every)
    if untimed:
        lat.sweep(untimed, beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if every:
        plaq = lat.sweep_measure(sweeps, beta)
    else:
        lat.sweep(sweeps, beta)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    if not every:
        plaq = [lat.plaquette()]
    updates = 4 * lat.V * nlat * sweeps
    del lat
    torch.cuda.empty_cache()
    return {"value": updates / t, "unit": "link updates/s", "sweeps": sweeps, "seconds": t,
            "algorithmic_gbs": round(updates / t * bytes_per_update(precision) / 1e9, 1),
            "stored_gbs": round(updates / t * stored_bytes_per_update(precision) / 1e9, 1),
            "plaquette_last": [float(x) for x in plaq[-1]],
            "_plaquette_series": [float(x[0]) for x in plaq]}


def two_coupling_rate(L, beta0, beta1, sweeps, seed=1, warmup_ms=CONFIG_WARMUP_MS):
    """Double-layered torus (flip mask 0x7) with per-layer couplings: link
    updates/s of `sweeps` sweeps (a device warm-up with the same kernels on a
    scratch lattice and one untimed sweep first), then the per-layer
    plaquettes and Polyakov loops."""
    import torch

    from paper_0904_1179_amd import Lattice

    lat = Lattice(L, nlat=2, precision=64, seed=seed, flip_mask=0x7)
    lat.start(hot=True)
    device_warmup(warmup_ms, L, 64, beta0, nlat=2, flip_mask=0x7, betas=(beta0, beta1))
    lat.sweep_betas(1, beta0, beta1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep_betas(sweeps, beta0, beta1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    poly = lat.polyakov()
    out = {"value": 4 * lat.V * 2 * sweeps / t, "unit": "link updates/s", "sweeps": sweeps, "seconds": t,
           "beta": [beta0, beta1], "plaquette_per_layer": [float(x) for x in lat.plaquette()[1:]],
           "polyakov_per_layer": [[float(z.real), float(z.imag)] for z in poly[1:]]}
    del lat
    torch.cuda.empty_cache()
    return out


def host_cpu():
    """Host CPU model (lscpu, else /proc/cpuinfo), core counts and the OpenMP thread count."""
    import subprocess

    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            model = "unknown"
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or nproc
    return {"model": model, "nproc": nproc, "cpu_count": os.cpu_count(), "omp_threads": threads}


def oracle_rate(L, nlat, beta, sweeps, threads, hot=True, flip_mask=None, seed=1, min_seconds=None):
    """The FP64 oracle on the host: `sweeps` sweeps (or, with min_seconds,
    sweeps one at a time until that much wall time has passed) after the
    start, which is excluded from the time as the paper excludes it."""
    from oracle import su3ref

    lat = su3ref.Oracle(L, nlat=nlat, flip_mask=flip_mask, seed=seed)
    lat.start(hot)
    done = 0
    t0 = time.perf_counter()
    if min_seconds is None:
        lat.sweep(sweeps, beta, nthreads=threads)
        done = sweeps
    else:
        while done < sweeps:
            lat.sweep(1, beta, nthreads=threads)
            done += 1
            if time.perf_counter() - t0 >= min_seconds:
                break
    t = time.perf_counter() - t0
    V = (L ** 4) if isinstance(L, int) else int(__import__("numpy").prod(L))
    ups = 4 * V * nlat * done
    return {"value": ups / t, "unit": "link updates/s", "threads": threads, "sweeps": done, "seconds": round(t, 3),
            "us_per_update_core": t * threads / ups * 1e6, "plaquette_last": [float(x) for x in lat.plaquette()]}


def cpu_baseline(L, beta, seed=1, min_seconds=1.5, max_sweeps=64, configs=True):
    """The FP64 oracle, as it stands, on the host cores: the headline lattice
    (sweeps one at a time until min_seconds of wall time have passed, all
    cores) and, with configs, the other workload configurations: 8^4 cold 32
    sweeps (all cores and one core), the 2 x 16^4 double-layered torus 32
    sweeps and 64^4 at beta 6.0 10 sweeps (all cores)."""
    cpu = host_cpu()
    threads = cpu["omp_threads"]
    head = oracle_rate(L, 1, beta, max_sweeps, threads, seed=seed, min_seconds=min_seconds)
    one = oracle_rate(16, 1, beta, 1, 1, seed=seed)
    out = {"value": head["value"], "unit": "link updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{head['sweeps']} sweeps of the {L}^4 hot-start lattice ({head['sweeps'] * 4 * L ** 4} link "
                     f"updates) at beta={beta}, OpenMP over the links of each pass; start excluded",
           "seconds": head["seconds"], "cpu_seconds_approx": head["seconds"] * threads,
           "host_cpu": cpu["model"], "nproc": cpu["nproc"], "cpu_count": cpu["cpu_count"],
           "single_core": {"value": one["value"], "us_per_update": one["us_per_update_core"],
                           "sample": "1 sweep of a 16^4 hot-start lattice, 1 thread"}}
    if configs:
        out["configs"] = {
            "8^4_fp64_cold_beta5.7_32sweeps": oracle_rate(8, 1, 5.7, 32, threads, hot=False, seed=seed),
            "8^4_fp64_cold_beta5.7_32sweeps_1core": oracle_rate(8, 1, 5.7, 32, 1, hot=False, seed=seed),
            "dlt_2x16^4_fp64_beta5.7_32sweeps": oracle_rate(16, 2, 5.7, 32, threads, flip_mask=0x7, seed=seed),
            "64^4_fp64_beta6.0_10sweeps": oracle_rate(64, 1, 6.0, 10, threads, seed=seed)}
    return out


def served_fp32_deviation(jobs, recs, count=8):
    """FP32 error of served jobs: for `count` jobs of the stream, the final
    plaquette of the served FP32 chain against the same job run alone in
    FP64 (same seed, start, beta and sweeps).  The jobs run 50-500 sweeps, past
    the onset of decorrelation of FP32 and FP64 chains (an accept/reject
    decision taken differently), so the deviation is a thermal fluctuation of
    order (6 V)^-1/2, reported with that scale."""
    import numpy as np

    from paper_0904_1179_amd import Lattice

    out = []
    for j in sorted(jobs, key=lambda j: j["id"])[:count]:
        lat = Lattice(j["L"], precision=64, seed=j["seed"])
        lat.start(j.get("hot", 1))
        lat.sweep(j["nsweeps"], j["beta"])
        p64 = float(lat.plaquette()[0])
        p32 = float(recs[j["id"]]["plaquette"][0])
        V = j["L"] ** 4
        out.append({"job": j["id"], "L": j["L"], "sweeps": j["nsweeps"], "fp32": p32, "fp64": p64,
                    "rel_err": abs(p32 - p64) / abs(p64), "fluctuation_scale": float((6 * V) ** -0.5)})
        del lat
    return {"jobs": out, "max_rel_err": max(o["rel_err"] for o in out),
            "note": "final plaquette of the served FP32 job vs the same job alone in FP64; chains this long have "
                    "decorrelated, so compare with fluctuation_scale"}


def startup_trace(L, beta, blocks=20, per_block=10, seed=1):
    """Sweep time from the first sweep of the process: lattice A from a hot
    start, `blocks` blocks of `per_block` sweeps each timed with HIP events on
    its stream, then a second lattice B allocated and started the same way;
    the GPU's clocks, power and temperature are sampled meanwhile (amdsmi)."""
    import threading

    import torch

    from paper_0904_1179_amd import Lattice

    samples, stop = [], threading.Event()
    smi = None
    try:
        import amdsmi

        amdsmi.amdsmi_init()
        smi = amdsmi.amdsmi_get_processor_handles()[0]
    except Exception as e:  # noqa: BLE001 -- the trace still runs without clock samples
        samples.append({"error": repr(e)})

    def sample():
        # current clocks as the driver reads them (the metrics table is refreshed too rarely for
        # the ~30 ms scale of the effect)
        import amdsmi

        kinds = {"gfx_mhz": amdsmi.AmdSmiClkType.GFX, "mem_mhz": amdsmi.AmdSmiClkType.MEM,
                 "fabric_mhz": amdsmi.AmdSmiClkType.DF, "soc_mhz": amdsmi.AmdSmiClkType.SOC}
        while not stop.is_set():
            t = time.perf_counter()
            rec = {"t": t}
            for k, ct in kinds.items():
                try:
                    rec[k] = amdsmi.amdsmi_get_clock_info(smi, ct)["clk"]
                except Exception as e:  # noqa: BLE001 -- a clock domain may not be readable
                    rec.setdefault("errors", []).append(f"{k}: {e!r}")
            samples.append(rec)
            time.sleep(0.001)

    th = None
    if smi is not None:
        th = threading.Thread(target=sample, daemon=True)
        th.start()
        time.sleep(0.2)  # the idle clocks before the first sweep

    def run(lat):
        out = []
        for _ in range(blocks):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ta = time.perf_counter()
            e0.record(lat.stream)
            lat.sweep(per_block, beta)
            e1.record(lat.stream)
            e1.synchronize()
            out.append((ta, time.perf_counter(), e0.elapsed_time(e1) / per_block))
        return out

    t_begin = time.perf_counter()
    a = Lattice(L, seed=seed)
    a.start(True)
    torch.cuda.synchronize()
    ra = run(a)
    b = Lattice(L, seed=seed + 1)
    b.start(True)
    torch.cuda.synchronize()
    rb = run(b)
    stop.set()
    if th is not None:
        th.join()

    def clocks(t0, t1):
        sel = [s for s in samples if "t" in s and t0 <= s["t"] <= t1]
        keys = set().union(*[s.keys() for s in sel]) - {"t", "errors"} if sel else set()
        out = {}
        for k in keys:
            vals = [s[k] for s in sel if isinstance(s.get(k), (int, float))]
            if vals:
                out[k] = round(sum(vals) / len(vals), 1)
        return out

    def rows(r):
        return [{"ms_per_sweep": round(ms, 4), "t_s": round(ta - t_begin, 3), **clocks(ta, tb)} for ta, tb, ms in r]

    return {"lattice": f"{L}^4 FP64 hot start, beta={beta}, su3_sweep in blocks of {per_block} sweeps",
            "idle_before": clocks(0.0, t_begin), "A_first_lattice": rows(ra), "B_second_lattice": rows(rb),
            "samples": len(samples), "sample_errors": sorted({e for s in samples for e in s.get("errors", [])})[:4]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1, help="must be 1: one lattice on one GPU")
    ap.add_argument("--steps", type=int, default=50, help="timed steps (sweep + fused plaquette)")
    ap.add_argument("--warmup", type=int, default=100, help="untimed steps before the timed region")
    ap.add_argument("--L", type=int, default=32, help="extent of the L^4 periodic lattice")
    ap.add_argument("--beta", type=float, default=5.7)
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32))
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--no-cpu-configs", action="store_true",
                    help="time the CPU oracle on the headline lattice only (not 8^4, 2x16^4, 64^4)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-link run")
    ap.add_argument("--no-copy-probe", action="store_true", help="skip the 1 GiB copy bandwidth probe")
    ap.add_argument("--no-serving", action="store_true", help="skip the mixed job stream")
    ap.add_argument("--no-configs", action="store_true", help="skip the other configurations (8^4, 16^4, 2x16^4 DLT, 64^4)")
    ap.add_argument("--device-warmup-ms", type=float, default=100.0,
                    help="busy the GPU this long with the pass kernels on a scratch lattice before the timed "
                         "lattice's warm-up steps (power ramp)")
    ap.add_argument("--startup-trace", action="store_true",
                    help="only trace the sweep time from the process's first sweep (two lattices, clocks sampled)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py: the benchmark runs one lattice on one GPU; --gpus above 1 is not supported "
                  "(independent chains or a halo-exchange decomposition would be needed)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    L, beta, prec = args.L, args.beta, args.precision
    if args.startup_trace:
        print(json.dumps(startup_trace(L, beta)), flush=True)
        return
    main_run = run_gpu(L, prec, args.steps, args.warmup, beta, device_warmup_ms=args.device_warmup_ms)
    warmed_ms = main_run["device_warmup_ms"]
    ups = main_run["updates"] / main_run["seconds"]
    pass_s = main_run["pass_ms"] * 1e-3
    links_per_pass = L ** 4 // 2
    alg_bytes = bytes_per_update(prec) * links_per_pass
    stored_bytes = stored_bytes_per_update(prec) * links_per_pass
    achieved = alg_bytes / pass_s / 1e9
    traffic = stored_traffic(f"k_update_{L}x4_fp{prec}_traffic.txt")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"k_update<mu, {'double' if prec == 64 else 'float'}>",
                "algorithmic_bytes_per_update": bytes_per_update(prec), "algorithmic_bytes_per_launch": alg_bytes,
                "stored_bytes_per_update": stored_bytes_per_update(prec), "stored_bytes_per_launch": stored_bytes,
                "achieved_stored_gbs": round(stored_bytes / pass_s / 1e9, 1),
                "frac_stored": round(stored_bytes / pass_s / 1e9 / HBM_PEAK_GBS, 4),
                "launch_us": round(main_run["pass_ms"] * 1e3, 2), "launches_timed": main_run["passes"]}
    if not args.no_copy_probe:
        roofline["copy_probe_gbs"] = round(copy_probe_gbs(), 1)
        # the pass's HBM traffic rate against what a plain copy reaches
        if traffic is not None:
            roofline["traffic_gbs_over_copy_probe"] = round(traffic / pass_s / 1e9 / roofline["copy_probe_gbs"], 3)
    spread = repeat_rates(main_run["lattice"], beta)
    del main_run["lattice"]

    out = {"metric": "SU(3) link updates/sec at 32^4 (FP64 checkerboard heat-bath sweep + plaquette)",
           "value": ups, "unit": "link updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": main_run["seconds"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prec == 64 else "f32",
           "data": "synthetic (Haar-random hot start from Philox seed 1)",
           "config": {"workload": f"{L}^4 periodic lattice, beta={beta}, hot start, 1-hit heat bath, "
                                  f"step = 1 sweep + 1 plaquette", "L": L, "nlat": 1, "beta": beta,
                      "precision": prec, "parallelism": "single GPU"},
           "us_per_update_gpu": main_run["seconds"] / main_run["updates"] * 1e6,
           "plaquette_last": main_run["plaquette"][-1],
           "plaquette_last_full_kernel": main_run["plaquette_full_kernel"],
           "sweep_rate_spread": spread,
           "device_warmup_ms": round(warmed_ms, 1),
           "roofline": roofline}

    if not args.no_fp32 and prec == 64:
        r32 = run_gpu(L, 32, args.steps, args.warmup, beta, device_warmup_ms=args.device_warmup_ms)
        del r32["lattice"]
        v32 = r32["updates"] / r32["seconds"]
        pass32 = r32["pass_ms"] * 1e-3
        out["fp32"] = {"value": v32, "unit": "link updates/s", "speedup_vs_fp64": v32 / ups,
                       "launch_us": round(r32["pass_ms"] * 1e3, 2),
                       "achieved_gbs": round(bytes_per_update(32) * links_per_pass / pass32 / 1e9, 1),
                       "achieved_stored_gbs": round(stored_bytes_per_update(32) * links_per_pass / pass32 / 1e9, 1),
                       "plaquette_rel_err_vs_fp64_first_sweeps": fp32_deviation(L, beta),
                       "timed_steps_vs_fp64_chain": chain_deviation(r32["plaquette"], main_run["plaquette"]),
                       "note": "FP32 links, products and heat-bath scalars; FP64 reunitarisation and sums. Errors: "
                               "per-sweep plaquette of the FP32 chain against the FP64 chain from the same start"}

    if not args.no_configs and prec == 64:
        # the other timed workload configurations: 8^4 from a cold start, 32 sweeps (launch-bound: reported
        # only); 16^4 in both precisions (the lattice fits in the 256 MB Infinity Cache: not an HBM figure);
        # a double-layered 2 x 16^4 torus (flip mask 0x7) at beta 5.7, with the per-layer plaquette after every
        # sweep and, separately, only after the last; 64^4 at beta 6.0 in both precisions
        # (10 sweeps each after one untimed sweep); the double-layered torus with per-layer couplings
        # 5.5 / 6.2 (32 sweeps) with its Polyakov loops
        cfg = {
            "8^4_fp64_cold_beta5.7": config_rate(8, 1, 64, 5.7, 32, hot=False, untimed=0),
            "16^4_fp64_beta5.7": config_rate(16, 1, 64, 5.7, 32),
            "16^4_fp32_beta5.7": config_rate(16, 1, 32, 5.7, 32),
            "dlt_2x16^4_fp64_beta5.7": config_rate(16, 2, 64, 5.7, 32, flip_mask=0x7),
            "dlt_2x16^4_fp64_beta5.7_plaquette_at_end": config_rate(16, 2, 64, 5.7, 32, flip_mask=0x7, every=False),
            "64^4_fp64_beta6.0": config_rate(64, 1, 64, 6.0, 10),
            "64^4_fp32_beta6.0": config_rate(64, 1, 32, 6.0, 10),
            "dlt_2x16^4_fp64_beta5.5|6.2": two_coupling_rate(16, 5.5, 6.2, 32)}
        # each FP32 figure with its error against the FP64 chain of the same configuration (same seed,
        # start and sweeps: the FP64 runs above)
        for k32, k64 in (("16^4_fp32_beta5.7", "16^4_fp64_beta5.7"), ("64^4_fp32_beta6.0", "64^4_fp64_beta6.0")):
            cfg[k32]["vs_fp64_chain"] = chain_deviation(cfg[k32]["_plaquette_series"], cfg[k64]["_plaquette_series"])
        for v in cfg.values():
            v.pop("_plaquette_series", None)
        out["configs"] = cfg

    if not args.no_serving:
        from paper_0904_1179_amd.serve import run_stream, run_stream_benchmark
        from paper_0904_1179_amd.workloads import serving_stream

        serving = run_stream_benchmark()
        # saturation: the same 256 jobs all submitted at t = 0 (what the server sustains, not the offered load)
        jobs = serving_stream(n_jobs=256, rate=20.0, seed=0, precision=32)
        recs, sat = run_stream(jobs, arena_bytes=4 << 30, max_active=256, realtime=False)
        serving["saturation"] = {k: sat[k] for k in ("wall_s", "throughput_updates_per_s", "p50_latency_s",
                                                     "p99_latency_s", "steps", "arena_peak_bytes")}
        serving["saturation"]["workload"] = "the same 256 jobs, all submitted at t = 0"
        serving["fp32_vs_fp64"] = served_fp32_deviation(jobs, recs)
        out["serving"] = serving

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, beta, configs=not args.no_cpu_configs)

    # the paper's own figures (CPU wall clock, FP64), as context only
    out["paper_context"] = {
        "one_e5405_core_updates_per_s": 4 * 16 ** 4 * 32 / 48.7,  # Table 1: non-MPI, 16^4, 32 sweeps, 48.7 s
        "cray_xt4_1296_cores_updates_per_s": 4 * 48 ** 4 * 256 / 28.2,  # Table 3: 48^4 PBC, 256 sweeps, 28.2 s
        "note": "Berg & Wu, Tables 1 and 3: 2 GHz Intel E5405 (g77) and 2.3 GHz Opteron Cray XT4 (PGI), FP64"}

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
