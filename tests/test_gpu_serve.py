"""GPU tests of the job server (continuous batching).

Each job's result in the mix must equal the same job run alone through the
single-lattice path: the server gives every link the same per-link arithmetic
and the same keyed random numbers, so the final plaquette is compared bit for
bit and the heat-bath counters exactly.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0904_1179_amd as hb_

    return hb_


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


MIX = [
    # (L, nlat, precision, beta, nsweeps, seed, hot, nhit)
    (8, 1, 32, 5.7, 6, 11, 1, 1),
    ((6, 4, 10, 2), 1, 32, 5.9, 3, 12, 1, 1),
    (4, 1, 64, 6.1, 9, 13, 0, 1),
    (10, 1, 32, 5.5, 4, 14, 1, 1),
    ((4, 4, 4, 6), 2, 64, 5.7, 5, 15, 1, 1),
    (6, 1, 64, 5.8, 7, 16, 1, 2),
    (12, 1, 32, 6.2, 2, 17, 1, 1),
    (8, 2, 32, 5.7, 3, 18, 0, 1),
]


def _alone(hb, L, nlat, prec, beta, nsw, seed, hot, nhit):
    lat = hb.Lattice(L, nlat=nlat, precision=prec, seed=seed, nhit=nhit)
    lat.start(hot)
    lat.sweep(nsw, beta)
    return lat.plaquette(), lat.counters()[1:]


@pytest.mark.parametrize("sweeps_per_call", [1, 8])
def test_each_result_identical_alone_and_in_the_mix(hb, sweeps_per_call):
    from paper_0904_1179_amd import serve

    jobs = [{"id": k, "arrival": 0.0, "L": L, "nlat": nlat, "precision": prec, "beta": beta, "nsweeps": nsw,
             "seed": seed, "hot": hot, "nhit": nhit} for k, (L, nlat, prec, beta, nsw, seed, hot, nhit) in
            enumerate(MIX)]
    # an arena that holds only a few of these lattices at a time: admission waits on memory
    p12 = hb.make_params(12, precision=32)
    nl, ns = hb.su3_footprint(p12)
    arena = 3 * (nl + ns) + (1 << 20)
    recs, summary = serve.run_stream(jobs, arena_bytes=arena, max_active=4, realtime=False,
                                     sweeps_per_call=sweeps_per_call)
    _say(f"mix: {summary['steps']} steps, arena peak {summary['arena_peak_bytes']} of {arena}")
    assert summary["arena_peak_bytes"] <= arena
    for k, spec in enumerate(MIX):
        r = recs[k]
        p_alone, cnt_alone = _alone(hb, *spec)
        nlat = spec[1]
        assert np.array_equal(np.array(r["plaquette"][:1 + nlat]), p_alone), (spec, r["plaquette"], p_alone)
        assert (r["kp_attempts"], r["kp_accepts"]) == cnt_alone
        assert r["sweeps_done"] == spec[4]


def test_admission_limited_by_footprint_and_slots(hb):
    from paper_0904_1179_amd import serve

    p = hb.make_params(8, precision=32)
    nl, ns = hb.su3_footprint(p)
    one = (nl + 255) // 256 * 256 + (ns + 255) // 256 * 256
    srv = serve.Server(arena_bytes=2 * one + (1 << 16), max_active=8)
    ids = [srv.submit(serve.make_job(8, 5.7, 3, seed=100 + k)) for k in range(6)]
    active, queued, _ = srv.step()
    assert active == 2 and queued == 4  # two footprints fit
    seen_done = 0
    for _ in range(50):
        active, queued, fin = srv.step()
        assert active <= 2
        seen_done += fin
        if active == 0 and queued == 0:
            break
    assert seen_done == 6
    assert all(srv.poll(i)["state"] == serve.DONE for i in ids)
    assert srv.stats()["arena_peak"] <= 2 * one
    # a job whose footprint exceeds the arena can never be admitted
    with pytest.raises(hb.SU3Error) as e:
        srv.submit(serve.make_job(16, 5.7, 1, seed=1))
    assert e.value.status == -2
    # slots: max_active bounds the batch even when memory is plentiful
    srv2 = serve.Server(arena_bytes=64 << 20, max_active=3)
    for k in range(5):
        srv2.submit(serve.make_job(4, 5.7, 2, seed=k + 1))
    assert srv2.step()[:2] == (3, 2)


def test_invalid_jobs_rejected(hb):
    from paper_0904_1179_amd import serve

    srv = serve.Server(arena_bytes=16 << 20, max_active=2)
    for bad in (serve.make_job(5, 5.7, 1, 1), serve.make_job(4, -1.0, 1, 1), serve.make_job(4, 5.7, 0, 1)):
        with pytest.raises(hb.SU3Error) as e:
            srv.submit(bad)
        assert e.value.status == -1
    with pytest.raises(hb.SU3Error) as e:
        srv.run(0)
    assert e.value.status == -1


def test_short_realtime_stream(hb):
    from paper_0904_1179_amd import serve
    from paper_0904_1179_amd.workloads import serving_stream

    jobs = serving_stream(n_jobs=24, rate=80.0, seed=3, precision=32, sizes=(4, 6, 8, 10), sweep_range=(5, 40))
    recs, s = serve.run_stream(jobs, arena_bytes=256 << 20, max_active=16, realtime=True)
    _say(f"short stream: p50 {s['p50_latency_s'] * 1e3:.1f} ms, p99 {s['p99_latency_s'] * 1e3:.1f} ms, "
         f"{s['throughput_updates_per_s']:.3e} updates/s, {s['steps']} steps")
    assert len(recs) == 24 and all("latency" in r and r["latency"] > 0 for r in recs.values())
    assert 0 < s["p50_latency_s"] <= s["p99_latency_s"] <= s["max_latency_s"]
    # a mid-stream spot check: job 5's result equals the job run alone
    j = jobs[5]
    p_alone, cnt = _alone(hb, j["L"], 1, 32, j["beta"], j["nsweeps"], j["seed"], 1, 1)
    assert recs[5]["plaquette"][0] == p_alone[0]
