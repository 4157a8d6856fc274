"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/su3hb.h declares, sizes buffers correctly and rejects
invalid arguments before any HIP call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "su3hb.h")).read()
    return sorted(set(re.findall(r"\b(su3_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def hb():
    import paper_0904_1179_amd as hb_

    return hb_


def test_library_exports_every_declared_symbol(hb):
    names = _declared()
    assert len(names) >= 18
    lib = C.CDLL(hb.su3hb.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_library_is_gfx950_code_object(hb):
    blob = open(hb.su3hb.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


@pytest.mark.parametrize("L,nlat,prec", [(8, 1, 64), (32, 1, 64), (32, 1, 32), (16, 2, 64), ((6, 4, 10, 2), 1, 64)])
def test_footprint(hb, L, nlat, prec):
    p = hb.make_params(L, nlat=nlat, precision=prec)
    links, scratch = hb.su3_footprint(p)
    Ls = (L,) * 4 if isinstance(L, int) else L
    V = Ls[0] * Ls[1] * Ls[2] * Ls[3]
    stride = -(-nlat * V // 2 // 64) * 64 + 64
    # 8 (direction, parity) blocks of `stride` links, each stored as rows 0 and 1 (6 complex entries)
    assert links == 48 * stride * (16 if prec == 64 else 8)
    assert links >= 6 * 4 * V * nlat * (16 if prec == 64 else 8)
    assert 65536 < scratch < (1 << 20) and scratch % 256 == 0


BAD = [dict(L=(3, 4, 4, 4)), dict(L=(0, 4, 4, 4)), dict(L=(2048, 2, 2, 2)), dict(L=4, nlat=3),
       dict(L=4, nlat=1, flip_mask=1), dict(L=4, nlat=2, flip_mask=0x10), dict(L=4, precision=16),
       dict(L=4, nhit=0), dict(L=4, nhit=65), dict(L=(1024, 1024, 1024, 2))]


@pytest.mark.parametrize("kw", BAD)
def test_invalid_params_rejected(hb, kw):
    p = hb.make_params(**kw)
    with pytest.raises(hb.SU3Error) as e:
        hb.su3_footprint(p)
    assert e.value.status == -1
    with pytest.raises(hb.SU3Error) as e:
        hb.su3_create(p, 1 << 20, 1 << 40, 1 << 20, 1 << 20, 0)
    assert e.value.status == -1


def test_create_checks_sizes_and_pointers_before_device(hb):
    p = hb.make_params(8)
    nl, ns = hb.su3_footprint(p)
    fake = 1 << 32  # never dereferenced: validation fails first
    with pytest.raises(hb.SU3Error) as e:
        hb.su3_create(p, fake, nl - 1, fake, ns, 0)
    assert e.value.status == -2
    with pytest.raises(hb.SU3Error) as e:
        hb.su3_create(p, fake, nl, fake, ns - 256, 0)
    assert e.value.status == -2
    with pytest.raises(hb.SU3Error) as e:
        hb.su3_create(p, 0, nl, fake, ns, 0)
    assert e.value.status == -1
    with pytest.raises(hb.SU3Error) as e:
        hb.su3_create(p, fake + 16, nl, fake, ns, 0)
    assert e.value.status == -1


def test_null_context_rejected(hb):
    lib = hb.lib()
    for name, args in (("su3_start", (None, 1)), ("su3_sweep", (None, 1, 5.7)), ("su3_reunitarise", (None,)),
                       ("su3_profile", (None, 1))):
        assert getattr(lib, name)(*args) == -1
    assert lib.su3_destroy(None) == 0
    assert lib.su3_strerror(-4) == b"call out of order"


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++11")])
def test_header_is_plain_c_and_cpp(tmp_path, lang, std):
    """include/su3hb.h declares a C ABI: it must compile as strict C99 (and as
    C++), with nothing but plain types in the signatures."""
    import shutil
    import subprocess

    cc = shutil.which("gcc" if lang == "c" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    src = tmp_path / "use_header.c"
    src.write_text('#include "su3hb.h"\nint main(void) { su3_params p; (void)p; return 0; }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-x", lang, "-I", inc,
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
