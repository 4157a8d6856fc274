"""Seeded synthetic inputs of the benchmark workloads (no method arithmetic).

The paper's workloads are symmetric L^4 periodic lattices and two-layer DLT
lattices at beta = 5.7 (Tables 1-3); there is no dataset.  The mixed job
stream stands in for a serving load: lattice sizes, couplings and sweep
counts drawn uniformly, Poisson arrivals.
"""
import numpy as np

SERVING_SIZES = (8, 10, 12, 16, 20, 24)


def serving_stream(n_jobs=256, rate=20.0, seed=0, precision=32, sizes=SERVING_SIZES, beta_range=(5.5, 6.2),
                   sweep_range=(50, 500)):
    """Jobs with L uniform in `sizes` (L^4 periodic), beta uniform in
    `beta_range`, sweep count uniform in `sweep_range` (inclusive), Philox
    seed 1 + j, hot start; exponential inter-arrival gaps of mean 1/rate,
    first arrival at t = 0.  Returns a list of dicts sorted by arrival."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrivals = np.concatenate([[0.0], np.cumsum(gaps[1:])])
    L = rng.choice(np.asarray(sizes), size=n_jobs)
    beta = rng.uniform(beta_range[0], beta_range[1], size=n_jobs)
    sweeps = rng.integers(sweep_range[0], sweep_range[1] + 1, size=n_jobs)
    return [{"id": j, "arrival": float(arrivals[j]), "L": int(L[j]), "nlat": 1, "beta": float(beta[j]),
             "nsweeps": int(sweeps[j]), "seed": 1 + j, "precision": precision, "hot": 1, "nhit": 1}
            for j in range(n_jobs)]
