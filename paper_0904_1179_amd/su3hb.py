"""ctypes binding of libsu3hb.so, the gfx950 checkerboard SU(3) heat-bath library.

The functions below carry the C-ABI names of include/su3hb.h and only marshal
arguments; every step of a sweep runs in the library's HIP kernels.  PyTorch
provides the device memory (caller-owned buffers) and the stream.  There is no
CPU fallback: importing this module without the built library raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsu3hb.so")

SU3_OK, SU3_EINVAL, SU3_ENOSPC, SU3_EDEVICE, SU3_ESTATE, SU3_ENUMERIC = 0, -1, -2, -3, -4, -5


class SU3Error(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class su3_params(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("nlat", C.c_int32), ("flip_mask", C.c_uint32),
                ("precision", C.c_int32), ("nhit", C.c_int32), ("seed", C.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    # PyTorch ships its own HIP runtime under the same soname as ROCm's
    # (libamdhip64.so.7).  Loaded first, it is the one this library binds to,
    # so device memory and streams that torch hands over belong to the same
    # runtime; loaded the other way round, the process would hold two.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    st, vp, u64, sz, dp = C.c_int, C.c_void_p, C.c_uint64, C.c_size_t, C.POINTER(C.c_double)
    P = C.POINTER(su3_params)
    sigs = {
        "su3_footprint": (st, [P, C.POINTER(sz), C.POINTER(sz)]),
        "su3_create": (st, [P, vp, sz, vp, sz, vp, C.POINTER(vp)]),
        "su3_start": (st, [vp, C.c_int32]),
        "su3_sweep": (st, [vp, C.c_int32, C.c_double]),
        "su3_plaquette": (st, [vp, dp, C.c_int32]),
        "su3_sweep_measure": (st, [vp, C.c_int32, C.c_double, dp, sz]),
        "su3_sweep_betas": (st, [vp, C.c_int32, C.c_double, C.c_double]),
        "su3_polyakov": (st, [vp, dp, C.c_int32]),
        "su3_plaquette_noalloc": (st, [P, vp, sz, vp, C.c_int32, vp]),
        "su3_reunitarise": (st, [vp]),
        "su3_get_links": (st, [vp, dp, sz]),
        "su3_set_links": (st, [vp, dp, sz]),
        "su3_get_link_sample": (st, [vp, C.POINTER(u64), sz, dp]),
        "su3_get_sweep_index": (st, [vp, C.POINTER(u64)]),
        "su3_set_sweep_index": (st, [vp, u64]),
        "su3_counters": (st, [vp, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]),
        "su3_gauge_transform": (st, [vp, u64]),
        "su3_set_lanes_per_link": (st, [vp, C.c_int32]),
        "su3_get_lanes_per_link": (st, [vp, C.POINTER(C.c_int32)]),
        "su3_profile": (st, [vp, C.c_int32]),
        "su3_profile_read": (st, [vp, dp, C.POINTER(u64)]),
        "su3_destroy": (st, [vp]),
        "su3_stream_copy": (st, [vp, vp, sz, vp]),
        "su3_strerror": (C.c_char_p, [st]),
        "su3_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status, where):
    if status != SU3_OK:
        raise SU3Error(status, where, _lib.su3_last_error().decode())


def make_params(L, nlat=1, flip_mask=None, precision=64, nhit=1, seed=1):
    if isinstance(L, int):
        L = (L, L, L, L)
    if flip_mask is None:
        flip_mask = 0x7 if nlat == 2 else 0
    p = su3_params()
    for i in range(4):
        p.L[i] = int(L[i])
    p.nlat, p.flip_mask, p.precision, p.nhit, p.seed = int(nlat), int(flip_mask), int(precision), int(nhit), int(seed)
    return p


# ----------------------------------------------------------------- C-ABI names

def su3_footprint(params):
    a, b = C.c_size_t(0), C.c_size_t(0)
    _check(_lib.su3_footprint(C.byref(params), C.byref(a), C.byref(b)), "su3_footprint")
    return a.value, b.value


def su3_create(params, d_links, link_bytes, d_scratch, scratch_bytes, stream):
    ctx = C.c_void_p(0)
    _check(_lib.su3_create(C.byref(params), C.c_void_p(d_links), link_bytes, C.c_void_p(d_scratch), scratch_bytes,
                           C.c_void_p(stream), C.byref(ctx)), "su3_create")
    return ctx


def su3_start(ctx, hot):
    _check(_lib.su3_start(ctx, int(hot)), "su3_start")


def su3_sweep(ctx, n, beta):
    _check(_lib.su3_sweep(ctx, int(n), float(beta)), "su3_sweep")


def su3_sweep_measure(ctx, n, beta, nlat):
    out = np.zeros((int(n), 1 + nlat))
    _check(_lib.su3_sweep_measure(ctx, int(n), float(beta), out.ctypes.data_as(C.POINTER(C.c_double)), out.size),
           "su3_sweep_measure")
    return out


def su3_sweep_betas(ctx, n, beta0, beta1):
    _check(_lib.su3_sweep_betas(ctx, int(n), float(beta0), float(beta1)), "su3_sweep_betas")


def su3_polyakov(ctx, nlat):
    out = np.zeros(2 * (1 + nlat))
    _check(_lib.su3_polyakov(ctx, out.ctypes.data_as(C.POINTER(C.c_double)), out.size), "su3_polyakov")
    return out[0::2] + 1j * out[1::2]


def su3_plaquette(ctx, nlat):
    out = np.zeros(1 + nlat)
    _check(_lib.su3_plaquette(ctx, out.ctypes.data_as(C.POINTER(C.c_double)), 1 + nlat), "su3_plaquette")
    return out


def su3_plaquette_noalloc(params, d_links, link_bytes, d_out, n_out, stream):
    """Asynchronous; writes 2 + nlat doubles to the device buffer d_out."""
    _check(_lib.su3_plaquette_noalloc(C.byref(params), C.c_void_p(d_links), link_bytes, C.c_void_p(d_out),
                                      int(n_out), C.c_void_p(stream)), "su3_plaquette_noalloc")


def su3_reunitarise(ctx):
    _check(_lib.su3_reunitarise(ctx), "su3_reunitarise")


def su3_get_links(ctx, n_doubles):
    out = np.empty(n_doubles, dtype=np.float64)
    _check(_lib.su3_get_links(ctx, out.ctypes.data_as(C.POINTER(C.c_double)), n_doubles), "su3_get_links")
    return out


def su3_set_links(ctx, host):
    host = np.ascontiguousarray(host, dtype=np.float64).reshape(-1)
    _check(_lib.su3_set_links(ctx, host.ctypes.data_as(C.POINTER(C.c_double)), host.size), "su3_set_links")


def su3_get_link_sample(ctx, lids):
    lids = np.ascontiguousarray(lids, dtype=np.uint64)
    out = np.empty(18 * lids.size, dtype=np.float64)
    _check(_lib.su3_get_link_sample(ctx, lids.ctypes.data_as(C.POINTER(C.c_uint64)), lids.size,
                                    out.ctypes.data_as(C.POINTER(C.c_double))), "su3_get_link_sample")
    return out.reshape(-1, 18)


def su3_get_sweep_index(ctx):
    v = C.c_uint64(0)
    _check(_lib.su3_get_sweep_index(ctx, C.byref(v)), "su3_get_sweep_index")
    return v.value


def su3_set_sweep_index(ctx, s):
    _check(_lib.su3_set_sweep_index(ctx, int(s)), "su3_set_sweep_index")


def su3_counters(ctx):
    a, b, c = C.c_uint64(0), C.c_uint64(0), C.c_uint64(0)
    _check(_lib.su3_counters(ctx, C.byref(a), C.byref(b), C.byref(c)), "su3_counters")
    return a.value, b.value, c.value


def su3_gauge_transform(ctx, gseed):
    _check(_lib.su3_gauge_transform(ctx, int(gseed)), "su3_gauge_transform")


def su3_set_lanes_per_link(ctx, lanes):
    _check(_lib.su3_set_lanes_per_link(ctx, int(lanes)), "su3_set_lanes_per_link")


def su3_get_lanes_per_link(ctx):
    v = C.c_int32(0)
    _check(_lib.su3_get_lanes_per_link(ctx, C.byref(v)), "su3_get_lanes_per_link")
    return v.value


def su3_profile(ctx, enable):
    _check(_lib.su3_profile(ctx, int(bool(enable))), "su3_profile")


def su3_profile_read(ctx):
    ms, n = C.c_double(0), C.c_uint64(0)
    _check(_lib.su3_profile_read(ctx, C.byref(ms), C.byref(n)), "su3_profile_read")
    return ms.value, n.value


def su3_destroy(ctx):
    _check(_lib.su3_destroy(ctx), "su3_destroy")


def su3_stream_copy(dst, src, nbytes, stream):
    _check(_lib.su3_stream_copy(C.c_void_p(dst), C.c_void_p(src), nbytes, C.c_void_p(stream)), "su3_stream_copy")


# ------------------------------------------------------------------ convenience

class Lattice:
    """One lattice resident in HBM: torch allocates the link and scratch
    buffers on the current device and the context runs on the current stream."""

    def __init__(self, L, nlat=1, flip_mask=None, precision=64, nhit=1, seed=1, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("su3hb needs a GPU: torch.cuda is not available")
        self.params = make_params(L, nlat, flip_mask, precision, nhit, seed)
        self.nlat = int(nlat)
        self.L = tuple(self.params.L)
        self.V = int(np.prod(self.L))
        link_bytes, scratch_bytes = su3_footprint(self.params)
        self.links_buf = torch.empty(link_bytes, dtype=torch.uint8, device="cuda")
        self.scratch_buf = torch.empty(scratch_bytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # the buffers come from the current stream's pool but the library works
        # on self.stream: tell the caching allocator, so that it does not hand
        # the memory out again while work queued on self.stream may still use it
        if self.stream != torch.cuda.current_stream():
            self.links_buf.record_stream(self.stream)
            self.scratch_buf.record_stream(self.stream)
        self.ctx = su3_create(self.params, self.links_buf.data_ptr(), link_bytes, self.scratch_buf.data_ptr(),
                              scratch_bytes, self.stream.cuda_stream)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            _lib.su3_destroy(ctx)
            self.ctx = None

    @property
    def n_doubles(self):
        return 72 * self.V * self.nlat

    def start(self, hot):
        su3_start(self.ctx, hot)

    def sweep(self, n, beta):
        su3_sweep(self.ctx, n, beta)

    def plaquette(self):
        return su3_plaquette(self.ctx, self.nlat)

    def sweep_betas(self, n, beta0, beta1):
        su3_sweep_betas(self.ctx, n, beta0, beta1)

    def polyakov(self):
        return su3_polyakov(self.ctx, self.nlat)

    def sweep_measure(self, n, beta):
        """n sweeps; returns the (n, 1 + nlat) plaquettes after each sweep."""
        return su3_sweep_measure(self.ctx, n, beta, self.nlat)

    def reunitarise(self):
        su3_reunitarise(self.ctx)

    def get_links(self):
        return su3_get_links(self.ctx, self.n_doubles).reshape(-1, 18)

    def set_links(self, host):
        su3_set_links(self.ctx, host)

    def link_sample(self, lids):
        return su3_get_link_sample(self.ctx, lids)

    @property
    def sweep_index(self):
        return su3_get_sweep_index(self.ctx)

    @sweep_index.setter
    def sweep_index(self, s):
        su3_set_sweep_index(self.ctx, s)

    def counters(self):
        return su3_counters(self.ctx)

    def gauge_transform(self, gseed):
        su3_gauge_transform(self.ctx, gseed)

    @property
    def lanes_per_link(self):
        return su3_get_lanes_per_link(self.ctx)

    @lanes_per_link.setter
    def lanes_per_link(self, lanes):
        su3_set_lanes_per_link(self.ctx, lanes)

    def profile(self, enable):
        su3_profile(self.ctx, enable)

    def profile_read(self):
        return su3_profile_read(self.ctx)
