"""ctypes binding of the FP64 CPU oracle (libsu3ref.so).

TEST INFRASTRUCTURE ONLY.  Arrays cross as numpy float64/uint64 buffers; the
canonical link layout is links[lid, row, col, reim] with lid = 4*site + mu.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Params(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("nlat", C.c_int32), ("flip_mask", C.c_uint32),
                ("nhit", C.c_int32), ("seed", C.c_uint64)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib_ = C.CDLL(_build.LIB)
    vp, i64, u64, dp = C.c_void_p, C.c_int64, C.c_uint64, C.POINTER(C.c_double)
    sig = {
        "su3ref_check_params": (C.c_int, [C.POINTER(Params)]),
        "su3ref_create": (vp, [C.POINTER(Params)]),
        "su3ref_create_geometry": (vp, [C.POINTER(Params)]),
        "su3ref_destroy": (None, [vp]),
        "su3ref_n_doubles": (i64, [vp]),
        "su3ref_links": (dp, [vp]),
        "su3ref_start": (None, [vp, C.c_int]),
        "su3ref_sweep": (None, [vp, C.c_int, C.c_double, C.c_int, u64]),
        "su3ref_plaquette": (None, [vp, dp]),
        "su3ref_reunitarise": (None, [vp]),
        "su3ref_sweep_betas": (None, [vp, C.c_int, C.c_double, C.c_double, C.c_int]),
        "su3ref_polyakov": (None, [vp, dp]),
        "su3ref_staple_betas": (None, [vp, i64, C.c_int, C.c_double, C.c_double, dp]),
        "su3ref_get_sweeps": (u64, [vp]),
        "su3ref_set_sweeps": (None, [vp, u64]),
        "su3ref_counters": (None, [vp, C.POINTER(u64), C.POINTER(u64)]),
        "su3ref_gauge_transform": (None, [vp, u64]),
        "su3ref_volume": (i64, [vp]),
        "su3ref_neighbor": (i64, [vp, i64, C.c_int, C.c_int]),
        "su3ref_parity": (C.c_int, [vp, i64]),
        "su3ref_staple_lids": (None, [vp, i64, C.c_int, C.POINTER(i64)]),
        "su3ref_staple": (None, [vp, i64, C.c_int, dp]),
        "su3ref_philox4x64": (None, [C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]),
        "su3ref_hot_link": (None, [u64, u64, dp]),
        "su3ref_gauge_element": (None, [u64, u64, dp]),
        "su3ref_staple_from_links": (None, [dp, dp]),
        "su3ref_reunit": (None, [dp]),
        "su3ref_heatbath_link": (None, [dp, dp, C.c_double, u64, u64, u64, C.c_int, C.POINTER(u64)]),
        "su3ref_kp_draws": (i64, [C.c_double, u64, i64, C.c_int, dp, C.POINTER(i64)]),
        "su3ref_single_link_chain": (None, [dp, dp, C.c_double, u64, i64, C.c_int, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib_, name)
        f.restype = res
        f.argtypes = args
    _lib = lib_
    return _lib


def lib():
    return load()


def make_params(L, nlat=1, flip_mask=None, nhit=1, seed=1):
    if isinstance(L, int):
        L = (L, L, L, L)
    if flip_mask is None:
        flip_mask = 0x7 if nlat == 2 else 0
    p = Params()
    for i in range(4):
        p.L[i] = int(L[i])
    p.nlat, p.flip_mask, p.nhit, p.seed = int(nlat), int(flip_mask), int(nhit), int(seed)
    return p


# ---------------------------------------------------------------------------
# single-link primitives
# ---------------------------------------------------------------------------

def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    load().su3ref_philox4x64(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def _mat(m):
    """complex (3,3) <-> float64 (18,) row-major (re, im)."""
    m = np.asarray(m)
    if np.iscomplexobj(m):
        out = np.empty(18)
        out[0::2] = m.reshape(9).real
        out[1::2] = m.reshape(9).imag
        return out
    return np.ascontiguousarray(m, dtype=np.float64).reshape(18)


def to_complex(a):
    a = np.asarray(a, dtype=np.float64)
    return (a[..., 0::2] + 1j * a[..., 1::2]).reshape(a.shape[:-1] + (3, 3))


def hot_link(seed, lid):
    out = np.zeros(18)
    load().su3ref_hot_link(seed, lid, _p(out, C.c_double))
    return to_complex(out)


def gauge_element(gseed, site):
    out = np.zeros(18)
    load().su3ref_gauge_element(gseed, site, _p(out, C.c_double))
    return to_complex(out)


def reunit(U):
    a = _mat(U).copy()
    load().su3ref_reunit(_p(a, C.c_double))
    return to_complex(a)


def staple_from_links(nb):
    """nb: 18 complex (3,3) matrices in the staple order."""
    arr = np.concatenate([_mat(m) for m in nb])
    out = np.zeros(18)
    load().su3ref_staple_from_links(_p(arr, C.c_double), _p(out, C.c_double))
    return to_complex(out)


def heatbath_link(U, A, beta, seed, lid, sweep, nhit=1):
    u = _mat(U).copy()
    a = _mat(A).copy()
    cnt = np.zeros(2, dtype=np.uint64)
    load().su3ref_heatbath_link(_p(u, C.c_double), _p(a, C.c_double), beta, seed, lid, sweep, nhit,
                                _p(cnt, C.c_uint64))
    return to_complex(u), int(cnt[0]), int(cnt[1])


def kp_draws(alpha, seed, n, cap=10000):
    a = np.zeros(4 * n)
    tries = C.c_int64(0)
    over = load().su3ref_kp_draws(alpha, seed, n, cap, _p(a, C.c_double), C.byref(tries))
    return a.reshape(n, 4), int(over), int(tries.value)


def single_link_chain(U, A, beta, seed, nsteps, nhit=1):
    u = _mat(U).copy()
    a = _mat(A).copy()
    obs = np.zeros(nsteps)
    load().su3ref_single_link_chain(_p(u, C.c_double), _p(a, C.c_double), beta, seed, nsteps, nhit,
                                    _p(obs, C.c_double))
    return obs, to_complex(u)


# ---------------------------------------------------------------------------
# lattice
# ---------------------------------------------------------------------------

class Geometry:
    """The oracle's site and link indexing for a lattice it does not hold:
    parity, neighbours and staple link ids only, at any size the parameters
    allow."""

    def __init__(self, L, nlat=1, flip_mask=None):
        self.params = make_params(L, nlat, flip_mask, 1, 1)
        lib_ = load()
        self._h = lib_.su3ref_create_geometry(C.byref(self.params))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.nlat = int(nlat)
        self.L = tuple(self.params.L)
        self.V = int(lib_.su3ref_volume(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.su3ref_destroy(h)
            self._h = None

    def parity(self, site):
        return int(_lib.su3ref_parity(self._h, int(site)))

    def neighbor(self, site, mu, d):
        return int(_lib.su3ref_neighbor(self._h, int(site), int(mu), int(d)))

    def staple_lids(self, site, mu):
        out = np.zeros(18, dtype=np.int64)
        _lib.su3ref_staple_lids(self._h, int(site), int(mu), _p(out, C.c_int64))
        return out


class Oracle:
    """A whole lattice held by the CPU oracle."""

    def __init__(self, L, nlat=1, flip_mask=None, nhit=1, seed=1):
        self.params = make_params(L, nlat, flip_mask, nhit, seed)
        lib_ = load()
        self._h = lib_.su3ref_create(C.byref(self.params))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.nlat = int(nlat)
        self.L = tuple(self.params.L)
        self.V = int(lib_.su3ref_volume(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.su3ref_destroy(h)
            self._h = None

    # raw view of the links: (nlinks, 18) float64, shares memory with the oracle
    def links(self):
        n = int(_lib.su3ref_n_doubles(self._h))
        ptr = _lib.su3ref_links(self._h)
        return np.ctypeslib.as_array(ptr, shape=(n,)).reshape(-1, 18)

    def set_links(self, arr):
        self.links()[...] = np.asarray(arr, dtype=np.float64).reshape(-1, 18)

    def start(self, hot):
        _lib.su3ref_start(self._h, int(bool(hot)))

    def sweep(self, n, beta, nthreads=0, order_seed=0):
        _lib.su3ref_sweep(self._h, int(n), float(beta), int(nthreads), int(order_seed))

    def plaquette(self):
        out = np.zeros(1 + self.nlat)
        _lib.su3ref_plaquette(self._h, _p(out, C.c_double))
        return out

    def reunitarise(self):
        _lib.su3ref_reunitarise(self._h)

    def sweep_betas(self, n, beta0, beta1, nthreads=0):
        _lib.su3ref_sweep_betas(self._h, int(n), float(beta0), float(beta1), int(nthreads))

    def staple_betas(self, site, mu, beta0, beta1):
        out = np.zeros(18)
        _lib.su3ref_staple_betas(self._h, int(site), int(mu), float(beta0), float(beta1), _p(out, C.c_double))
        return to_complex(out)

    def polyakov(self):
        """Complex mean Polyakov loop (Tr/3): total, then per starting layer."""
        out = np.zeros(2 + 2 * self.nlat)
        _lib.su3ref_polyakov(self._h, _p(out, C.c_double))
        return out[0::2] + 1j * out[1::2]

    @property
    def sweeps(self):
        return int(_lib.su3ref_get_sweeps(self._h))

    @sweeps.setter
    def sweeps(self, s):
        _lib.su3ref_set_sweeps(self._h, int(s))

    def counters(self):
        a, b = C.c_uint64(0), C.c_uint64(0)
        _lib.su3ref_counters(self._h, C.byref(a), C.byref(b))
        return int(a.value), int(b.value)

    def gauge_transform(self, gseed):
        _lib.su3ref_gauge_transform(self._h, int(gseed))

    def neighbor(self, site, mu, d):
        return int(_lib.su3ref_neighbor(self._h, int(site), int(mu), int(d)))

    def parity(self, site):
        return int(_lib.su3ref_parity(self._h, int(site)))

    def staple_lids(self, site, mu):
        out = np.zeros(18, dtype=np.int64)
        _lib.su3ref_staple_lids(self._h, int(site), int(mu), _p(out, C.c_int64))
        return out

    def staple(self, site, mu):
        out = np.zeros(18)
        _lib.su3ref_staple(self._h, int(site), int(mu), _p(out, C.c_double))
        return to_complex(out)
