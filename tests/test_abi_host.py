"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects host-checkable invalid arguments before touching
the GPU.  No kernel runs here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ankh.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ankh_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2212_08284_amd as ak
    if not os.path.exists(ak.LIB_PATH):
        from paper_2212_08284_amd.build import build
        build()
    return ak.load_library()


def test_header_declares_the_abi():
    names = _declared()
    for want in ("ankh_plan", "ankh_energy", "ankh_energy_forces", "ankh_sync", "ankh_destroy"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_carries_the_c_names():
    import paper_2212_08284_amd as ak
    for name in _declared():
        assert callable(getattr(ak, name)), name
    assert sorted(ak.EXPORTS) == _declared()


def test_status_strings(lib):
    for code in range(9):
        s = lib.ankh_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.ankh_status_string(0) == b"ok"
    assert lib.ankh_status_string(8) == b"induced dipoles not converged"


def _plan(lib, n=100, rb=10.0, eps=1e-6, order=2, prec=0, ov=None):
    import paper_2212_08284_amd as ak
    h = ctypes.c_void_p()
    ovp = ctypes.byref(ov) if ov is not None else ctypes.cast(None, ctypes.POINTER(ak._Overrides))
    return lib.ankh_plan(ctypes.byref(h), n, rb, eps, order, prec, ovp, None), h


@pytest.mark.parametrize("kw", [dict(n=0), dict(n=-5), dict(rb=0.0), dict(rb=-1.0), dict(rb=float("nan")),
                                dict(eps=1e-13), dict(eps=0.5), dict(order=4), dict(order=-1), dict(prec=7)])
def test_plan_rejects_invalid_arguments(lib, kw):
    st, h = _plan(lib, **kw)
    assert st == 1          # ANKH_ERR_INVALID_ARG
    assert not h.value      # output untouched


def test_plan_rejects_bad_overrides(lib):
    import paper_2212_08284_amd as ak
    for ov in (ak._Overrides(9, 0, 0, 0.0), ak._Overrides(-1, 1, 0, 0.0), ak._Overrides(-1, 11, 0, 0.0),
               ak._Overrides(-1, 0, 99, 0.0), ak._Overrides(-1, 0, 0, float("inf")),
               ak._Overrides(-1, 0, 0, 0.0, 0, 2.0), ak._Overrides(-1, 0, 0, 0.0, 0, float("nan")),
               ak._Overrides(depth=-1, far_field=3), ak._Overrides(depth=-1, far_field=2, eq_order=1),
               ak._Overrides(depth=-1, far_field=2, eq_order=11), ak._Overrides(depth=-1, far_field=2, fft_split=2),
               ak._Overrides(depth=-1, overlap=3),
               # ANKH-FFT beyond depth 6; leaf grids: not for ANKH-FMM, at most 40 unless a power of two
               ak._Overrides(depth=7, far_field=2), ak._Overrides(depth=-1, leaves=20),
               ak._Overrides(depth=-1, far_field=2, leaves=41), ak._Overrides(depth=-1, far_field=2, leaves=65),
               ak._Overrides(depth=-1, far_field=2, leaves=-1)):
        st, h = _plan(lib, ov=ov)
        assert st == 1 and not h.value


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of ankh_overrides and ankh_plan_stats have the C layout: the size and every
    field offset, from a C program compiled against the header."""
    import shutil
    import subprocess
    import paper_2212_08284_amd as ak
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ankh.h"', 'int main(void) {']
    for cname, py in (("ankh_overrides", ak._Overrides), ("ankh_plan_stats", ak._Stats)):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for cname, py in (("ankh_overrides", ak._Overrides), ("ankh_plan_stats", ak._Stats)):
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_mixed_precision_accuracy_floor(lib):
    st, h = _plan(lib, eps=1e-9, prec=1)
    assert st == 5          # ANKH_ERR_ACCURACY_UNREACHABLE
    assert not h.value


def test_null_plan_and_null_outputs(lib):
    vp = ctypes.c_void_p
    assert lib.ankh_energy(None, vp(8), vp(8), None, None, vp(8)) == 1
    assert lib.ankh_energy_forces(None, vp(8), vp(8), None, None, vp(8), vp(8), None) == 1
    assert lib.ankh_sync(None) == 1
    assert lib.ankh_set_timing(None, 1) == 1
    assert lib.ankh_last_terms(None, None) == 1
    assert lib.ankh_plan(None, 10, 1.0, 1e-6, 0, 0, None, None) == 1
    assert lib.ankh_induce(None, vp(8), vp(8), None, None, vp(8), 1e-8, 10, vp(8), None, None, None, None) == 1
    assert lib.ankh_energy_derivs(None, vp(8), vp(8), None, None, vp(8), None, None, vp(8), None) == 1
    assert lib.ankh_energy_derivs_noalloc(None, vp(8), vp(8), None, None, vp(8), None, None, vp(8), None) == 1
    assert lib.ankh_energy_octupole(None, vp(8), vp(8), None, None, vp(8), vp(8), None, None) == 1
    lib.ankh_destroy(None)   # no-op
