"""Oracle values of single links after the first sweep, computed one by one.

In the first sweep the link U_mu(x) is updated exactly once, in pass
q = 2*mu + parity(x) + 1 (passes mu = 0..3 x parity even, odd), from its own
start value and the values its 18 staple links hold after pass q-1.  Each of
those is either still its start value or was itself updated in an earlier
pass, so any link's value after the sweep follows from a finite set of start
links.  This lets the oracle check sampled links of lattices far too large
for a full oracle sweep.  Uses only the oracle's primitives.
"""
import numpy as np

from oracle import su3ref


class FirstSweepCone:
    def __init__(self, L, nlat=1, flip_mask=None, seed=1, beta=5.7, nhit=1, hot=True):
        self.geo = su3ref.Geometry(L, nlat=nlat, flip_mask=flip_mask)
        self.seed, self.beta, self.nhit, self.hot = seed, beta, nhit, hot
        self.memo = {}

    def start_value(self, lid):
        if self.hot:
            return su3ref.hot_link(self.seed, lid)
        return np.eye(3, dtype=complex)

    def pass_of(self, lid):
        site, mu = divmod(int(lid), 4)
        return 2 * mu + self.geo.parity(site) + 1

    def value(self, lid, stage=8):
        """Value of link lid after pass `stage` (0 = start, 8 = end of sweep 1)."""
        lid = int(lid)
        q = self.pass_of(lid)
        if q > stage:
            return self.start_value(lid)
        if lid not in self.memo:
            site, mu = divmod(lid, 4)
            nb = [self.value(l, q - 1) for l in self.geo.staple_lids(site, mu)]
            A = su3ref.staple_from_links(nb)
            U, _, _ = su3ref.heatbath_link(self.start_value(lid), A, self.beta, self.seed, lid, 0, self.nhit)
            self.memo[lid] = U
        return self.memo[lid]


def sample_lids(n_links, count, seed=0):
    """Sampled link ids spread over the lattice and over all 8 passes."""
    rng = np.random.default_rng(seed)
    lids = rng.integers(0, n_links, size=count, dtype=np.int64)
    return np.unique(np.concatenate([lids, [0, 1, 2, 3, n_links - 1, n_links - 4]]))
