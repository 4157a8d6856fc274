"""MI355X (gfx950) checkerboard SU(3) heat bath: HIP kernels behind a C ABI.

Berg & Wu, "Fortran MPI Checkerboard Code for SU(3) Lattice Gauge Theory II":
nequi checkerboard heat-bath sweeps of pure SU(3) Wilson-action LGT on
periodic and double-layered-torus lattices, here on one GPU.
"""
from .su3hb import (Lattice, SU3Error, lib, make_params, su3_counters, su3_create, su3_destroy,  # noqa: F401
                    su3_footprint, su3_gauge_transform, su3_get_link_sample, su3_get_links,
                    su3_get_sweep_index, su3_plaquette, su3_profile, su3_profile_read, su3_reunitarise,
                    su3_set_links, su3_set_sweep_index, su3_start, su3_stream_copy, su3_sweep,
                    su3_sweep_betas, su3_polyakov, su3_sweep_measure)
