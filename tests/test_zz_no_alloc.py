"""The workspace-free plaquette entry point, su3_plaquette_noalloc, against
su3_plaquette through the C ABI.  Both run the same plaquette kernels with the
same reduction order, the one on the context's scratch buffer, the other on
the library's own device array, so their values must agree bit for bit; two
calls in a row, the second on a smaller lattice (the array keeps the first
call's contents), a lattice large enough for the plaquette's x3 walk, and a
lattice with a NaN link."""
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


def _noalloc(hb, lat, n_out=None):
    import torch

    n_out = 2 + lat.nlat if n_out is None else n_out
    out = torch.full((max(n_out, 1),), -1.0, dtype=torch.float64, device="cuda")
    print(f"su3_plaquette_noalloc L={lat.L} nlat={lat.nlat} precision={lat.params.precision}", flush=True)
    hb.su3hb.su3_plaquette_noalloc(lat.params, lat.links_buf.data_ptr(), lat.links_buf.numel(), out.data_ptr(),
                                   n_out, lat.stream.cuda_stream)
    lat.stream.synchronize()
    return out.cpu().numpy()


def test_noalloc_plaquette_matches_context_plaquette(hb):
    big = hb.Lattice((8, 8, 8, 16), nlat=2, seed=4)
    big.start(True)
    big.sweep(2, 5.7)
    small = hb.Lattice((4, 4, 4, 6), nlat=1, precision=32, seed=5)
    small.start(True)
    small.sweep(1, 5.7)
    for lat in (big, small):  # the second call on the smaller lattice
        got = _noalloc(hb, lat)
        ref = lat.plaquette()
        assert np.array_equal(got[:1 + lat.nlat], ref), (got, ref)
        assert got[1 + lat.nlat] == 0.0
    # the same lattice again after the small one: the array's old contents do not leak in
    assert np.array_equal(_noalloc(hb, big)[:3], big.plaquette())


def test_noalloc_plaquette_on_the_walk_path(hb):
    """A double-layered FP64 lattice large enough for the x3 walk of the
    plaquette (32 x 32 x 16 x 16 per layer: 4 chunks of 4 sites, 65536
    threads per layer), then a small lattice, then the large one again: bit
    for bit as su3_plaquette each time."""
    big = hb.Lattice((32, 32, 16, 16), nlat=2, flip_mask=0xF, seed=7)
    big.start(True)
    big.sweep(1, 5.7)
    small = hb.Lattice((4, 6, 4, 4), nlat=2, seed=8)
    small.start(True)
    for lat in (big, small, big):
        got = _noalloc(hb, lat)
        assert np.array_equal(got[:3], lat.plaquette()), got
        assert got[3] == 0.0


def test_noalloc_plaquette_counts_bad_links(hb):
    lat = hb.Lattice((4, 4, 6, 4), seed=6)
    lat.start(True)
    links = lat.get_links()
    links[9, 2] = np.nan
    links[40, 0:6] *= 1.001
    lat.set_links(links)
    got = _noalloc(hb, lat)
    assert got[2] == 2.0
    with pytest.raises(hb.SU3Error) as e:
        lat.plaquette()
    assert e.value.status == hb.su3hb.SU3_ENUMERIC and "2 links" in str(e.value)


def test_noalloc_plaquette_rejects_bad_arguments(hb):
    lat = hb.Lattice(4, seed=1)
    lat.start(True)
    with pytest.raises(hb.SU3Error) as e:
        _noalloc(hb, lat, n_out=2)  # needs 2 + nlat = 3
    assert e.value.status == -1
    with pytest.raises(hb.SU3Error) as e:
        hb.su3hb.su3_plaquette_noalloc(lat.params, lat.links_buf.data_ptr(), lat.links_buf.numel() - 256,
                                       lat.links_buf.data_ptr(), 3, lat.stream.cuda_stream)
    assert e.value.status == -2
    bad = hb.make_params(5)
    with pytest.raises(hb.SU3Error) as e:
        hb.su3hb.su3_plaquette_noalloc(bad, lat.links_buf.data_ptr(), lat.links_buf.numel(),
                                       lat.links_buf.data_ptr(), 3, lat.stream.cuda_stream)
    assert e.value.status == -1
