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
# the lattice once (8 reads per updated link) and writes the updated link.
# A link is stored and moved as its rows 0 and 1 (12 reals; row 2 is rebuilt).
READ_REALS, WRITE_REALS, READS_PER_UPDATE = 12, 12, 8


def bytes_per_update(precision):
    return (READS_PER_UPDATE * READ_REALS + WRITE_REALS) * REAL_BYTES[precision]
PROFILE_DIR = os.path.join(ROOT, "profiles")
# what the pass kernel's counters depend on: its code, its launch shape and the
# pass order the host picks
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0904_1179_amd", "csrc", f)
                  for f in ("kernels.hip", "device.h", "launch.h", "api.hip")]


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


def run_gpu(L, precision, steps, warmup, beta, seed=1):
    import torch

    from paper_0904_1179_amd import Lattice

    lat = Lattice(L, nlat=1, precision=precision, seed=seed)
    lat.start(hot=True)
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
            "plaquette": plaq, "plaquette_full_kernel": full, "lattice": lat}


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


def config_rate(L, nlat, precision, beta, sweeps, seed=1, flip_mask=None, hot=True, untimed=1, every=True):
    """Link updates/s of `sweeps` sweeps on one more workload configuration,
    after the start and `untimed` untimed sweeps, with the plaquette after
    every sweep (every=True) or once after the last (outside the timed
    region); also the algorithmic bytes per second of the passes and the last
    plaquettes."""
    import torch

    from paper_0904_1179_amd import Lattice

    lat = Lattice(L, nlat=nlat, precision=precision, seed=seed, flip_mask=flip_mask)
    lat.start(hot=hot)
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
            "plaquette_last": [float(x) for x in plaq[-1]]}


def two_coupling_rate(L, beta0, beta1, sweeps, seed=1):
    """Double-layered torus (flip mask 0x7) with per-layer couplings: link
    updates/s of `sweeps` sweeps (one untimed sweep first), then the per-layer
    plaquettes and Polyakov loops."""
    import torch

    from paper_0904_1179_amd import Lattice

    lat = Lattice(L, nlat=2, precision=64, seed=seed, flip_mask=0x7)
    lat.start(hot=True)
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


def cpu_baseline(L, beta, seed=1, min_seconds=1.5, max_sweeps=64):
    """The FP64 oracle, as it stands, on the host cores: sweeps of the same
    lattice, one at a time, until min_seconds of wall time have passed."""
    from oracle import su3ref

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    lat = su3ref.Oracle(L, nlat=1, seed=seed)
    lat.start(True)
    sweeps = 0
    t0 = time.perf_counter()
    while sweeps < max_sweeps:
        lat.sweep(1, beta, nthreads=threads)
        sweeps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    t = time.perf_counter() - t0
    one = su3ref.Oracle(16, nlat=1, seed=seed)
    one.start(True)
    t1 = time.perf_counter()
    one.sweep(1, beta, nthreads=1)
    t_one = time.perf_counter() - t1
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": sweeps * 4 * L ** 4 / t, "unit": "link updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} sweeps of the {L}^4 hot-start lattice ({sweeps * 4 * L ** 4} link updates) at "
                      f"beta={beta}, OpenMP over the links of each pass; start excluded",
            "seconds": t, "cpu_seconds_approx": t * threads, "host_cpu": cpu,
            "single_core": {"value": 4 * 16 ** 4 / t_one, "us_per_update": t_one / (4 * 16 ** 4) * 1e6,
                            "sample": "1 sweep of a 16^4 hot-start lattice, 1 thread"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1, help="must be 1: one lattice on one GPU")
    ap.add_argument("--steps", type=int, default=50, help="timed steps (sweep + fused plaquette)")
    # the first ~60 sweeps of a process run up to 15% slower while the GPU warms
    # up (a second lattice in the same process runs at full speed at once)
    ap.add_argument("--warmup", type=int, default=100, help="untimed steps before the timed region")
    ap.add_argument("--L", type=int, default=32, help="extent of the L^4 periodic lattice")
    ap.add_argument("--beta", type=float, default=5.7)
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32))
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-link run")
    ap.add_argument("--no-copy-probe", action="store_true", help="skip the 1 GiB copy bandwidth probe")
    ap.add_argument("--no-serving", action="store_true", help="skip the mixed job stream")
    ap.add_argument("--no-configs", action="store_true", help="skip the other configurations (8^4, 16^4, 2x16^4 DLT, 64^4)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py: this build runs one lattice on one GPU; --gpus above 1 is not supported "
                  "(independent chains or a halo-exchange decomposition would be needed)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    L, beta, prec = args.L, args.beta, args.precision
    main_run = run_gpu(L, prec, args.steps, args.warmup, beta)
    ups = main_run["updates"] / main_run["seconds"]
    pass_s = main_run["pass_ms"] * 1e-3
    links_per_pass = L ** 4 // 2
    alg_bytes = bytes_per_update(prec) * links_per_pass
    achieved = alg_bytes / pass_s / 1e9
    traffic = stored_traffic(f"k_update_{L}x4_fp{prec}_traffic.txt")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"k_update<mu, {'double' if prec == 64 else 'float'}>",
                "algorithmic_bytes_per_launch": alg_bytes, "algorithmic_bytes_per_update": bytes_per_update(prec),
                "updates_per_s_vs_18_real_roofline": round(links_per_pass / pass_s / (HBM_PEAK_GBS * 1e9 / (9 * 18 * REAL_BYTES[prec])), 4), "launch_us": round(main_run["pass_ms"] * 1e3, 2),
                "launches_timed": main_run["passes"]}
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
           "roofline": roofline}

    if not args.no_fp32 and prec == 64:
        r32 = run_gpu(L, 32, args.steps, args.warmup, beta)
        del r32["lattice"]
        v32 = r32["updates"] / r32["seconds"]
        alg32 = bytes_per_update(32) * links_per_pass
        out["fp32"] = {"value": v32, "unit": "link updates/s", "speedup_vs_fp64": v32 / ups,
                       "launch_us": round(r32["pass_ms"] * 1e3, 2),
                       "achieved_gbs": round(alg32 / (r32["pass_ms"] * 1e-3) / 1e9, 1),
                       "plaquette_rel_err_vs_fp64_per_sweep": fp32_deviation(L, beta),
                       "note": "FP32 links and products; FP64 heat-bath scalars, reunitarisation and sums"}

    if not args.no_configs and prec == 64:
        # the other timed workload configurations: 8^4 from a cold start, 32 sweeps (launch-bound: reported
        # only); 16^4 in both precisions (the lattice fits in the 256 MB Infinity Cache: not an HBM figure);
        # a double-layered 2 x 16^4 torus (flip mask 0x7) at beta 5.7, with the per-layer plaquette after every
        # sweep and, separately, only after the last; 64^4 at beta 6.0 in both precisions
        # (10 sweeps each after one untimed sweep); the double-layered torus with per-layer couplings
        # 5.5 / 6.2 (32 sweeps) with its Polyakov loops
        out["configs"] = {
            "8^4_fp64_cold_beta5.7": config_rate(8, 1, 64, 5.7, 32, hot=False, untimed=0),
            "16^4_fp64_beta5.7": config_rate(16, 1, 64, 5.7, 32),
            "16^4_fp32_beta5.7": config_rate(16, 1, 32, 5.7, 32),
            "dlt_2x16^4_fp64_beta5.7": config_rate(16, 2, 64, 5.7, 32, flip_mask=0x7),
            "dlt_2x16^4_fp64_beta5.7_plaquette_at_end": config_rate(16, 2, 64, 5.7, 32, flip_mask=0x7, every=False),
            "64^4_fp64_beta6.0": config_rate(64, 1, 64, 6.0, 10),
            "64^4_fp32_beta6.0": config_rate(64, 1, 32, 6.0, 10),
            "dlt_2x16^4_fp64_beta5.5|6.2": two_coupling_rate(16, 5.5, 6.2, 32)}

    if not args.no_serving:
        from paper_0904_1179_amd.serve import run_stream_benchmark

        out["serving"] = run_stream_benchmark()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, beta)

    # the paper's own figures (CPU wall clock, FP64), as context only
    out["paper_context"] = {
        "one_e5405_core_updates_per_s": 4 * 16 ** 4 * 32 / 48.7,  # Table 1: non-MPI, 16^4, 32 sweeps, 48.7 s
        "cray_xt4_1296_cores_updates_per_s": 4 * 48 ** 4 * 256 / 28.2,  # Table 3: 48^4 PBC, 256 sweeps, 28.2 s
        "note": "Berg & Wu, Tables 1 and 3: 2 GHz Intel E5405 (g77) and 2.3 GHz Opteron Cray XT4 (PGI), FP64"}

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
