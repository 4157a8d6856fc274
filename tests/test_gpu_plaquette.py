"""GPU parity of su3_plaquette on large lattices, against the oracle's
plaquette of the same links.  FP64 lattices with at least 65536 columns x
chunks take the x3 walk (k_plaq_walk: one thread per column (x0, x1, x2) and
chunk of x3); FP32 lattices take k_plaq_partial.

The oracle is handed the links the library holds (su3_get_links: FP64, or the
stored FP32 rows widened with row 2 rebuilt in FP64), so the comparison
isolates the plaquette.  FP64: both sides sum the same SU(3) matrices in FP64,
in different orders, and agree to 1e-13.  FP32: the stored rows are unitary
only to about 2^-24, while the kernel forms every product of two links as an
SU(3) product (rows 0 and 1, row 2 rebuilt) and the oracle multiplies the full
matrices; that moves a plaquette by about 5e-9 (rms, measured on random
FP32-rounded SU(3) links) and the mean over 10^6 plaquettes by about 1e-11,
so the bound is 1e-9, still far below the 1e-7 that one misplaced or dropped
plaquette shifts the mean by.  The FP64 cases cover the chunk counts 4, 6, 8
and 156 (a ragged 6 x 10 x 14 x 626 lattice with chunks of 4 and 5 sites),
double-layered tori whose flipped x3 boundary the last site of a chunk
crosses, and the count of failing links.
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


WALK_CASES = [
    # (L, nlat, flip, precision)
    ((32, 32, 32, 32), 1, None, 64),  # the benchmark lattice: 4 chunks of 8
    ((32, 32, 32, 32), 1, None, 32),  # k_plaq_partial
    ((24, 24, 24, 24), 1, None, 64),  # 6 chunks of 4: 82944 threads
    ((16, 16, 32, 32), 2, 0xF, 64),   # DLT, every direction flipped: 8 chunks of 4
    ((16, 16, 32, 32), 2, 0x8, 64),   # DLT, only x3 flipped
    ((16, 16, 32, 32), 2, 0x8, 32),
    ((6, 10, 14, 626), 1, None, 64),  # ragged: 156 chunks of 4 or 5 sites
]


@pytest.mark.parametrize("L,nlat,flip,precision", WALK_CASES)
def test_walk_plaquette_matches_oracle_on_the_same_links(hb, L, nlat, flip, precision):
    from oracle import su3ref

    _say(f"plaquette walk L={L} nlat={nlat} flip={flip} precision={precision}")
    lat = hb.Lattice(L, nlat=nlat, flip_mask=flip, precision=precision, seed=11)
    lat.start(True)
    lat.sweep(1, 5.7)
    got = lat.plaquette()
    ref = su3ref.Oracle(L, nlat=nlat, flip_mask=flip, seed=11)
    ref.set_links(lat.get_links())
    want = ref.plaquette()
    assert got.shape == want.shape
    assert np.abs(got - want).max() < (1e-13 if precision == 64 else 1e-9), (got, want)
    # a reproducible sum
    assert lat.plaquette().tobytes() == got.tobytes()


def test_walk_counts_failing_links(hb):
    """Bad links anywhere in the walk's order are each counted once: the
    first link (the first site of the first chunk), a U_3 link in the top
    slab x3 = 31 (the last site of the last chunk, read there as an own link
    and by three neighbours), and the last link of the lattice."""
    L = (32, 32, 32, 32)
    _say(f"plaquette walk failing links L={L}")
    lat = hb.Lattice(L, precision=64, seed=2)
    lat.start(True)
    good = lat.get_links()
    lat.plaquette()
    V = int(np.prod(L))
    top = (31 * 32 * 32 * 32 + 5) * 4 + 3  # U_3 at x3 = 31
    bad = good.copy()
    bad[0, 4] = np.nan
    bad[top, 0:6] *= 1.0 + 1e-6
    bad[4 * V - 1, 7] = np.inf
    lat.set_links(bad)
    with pytest.raises(hb.SU3Error) as e:
        lat.plaquette()
    assert e.value.status == hb.su3hb.SU3_ENUMERIC and "3 links" in str(e.value)
    lat.set_links(good)
    lat.plaquette()
