"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every symbol
that include/laph.h declares, and its host-only logic (the dilution parser of Sec. II,
error strings) behaves.  No compute call is made here."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "laph.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^LAPH_API [^(]*?\b([a-z_0-9]+)\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_1104_3870_amd as P

    return P.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 22
    for n in names:
        assert hasattr(L, n), n
    import paper_1104_3870_amd as P

    assert set(names) == set(P.EXPORTS), set(names) ^ set(P.EXPORTS)


def test_only_abi_symbols_exported():
    import subprocess

    import paper_1104_3870_amd as P

    out = subprocess.check_output(["nm", "-D", "--defined-only", P.LIB_PATH]).decode()
    text_syms = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert text_syms == set(_declared())


def test_library_allocates_no_device_memory():
    """The library takes every device buffer from the caller's workspace: it does not even
    link the runtime's device allocators (pinned host memory for the solver's scalar
    readback is the one allocation it makes)."""
    import subprocess

    import paper_1104_3870_amd as P

    out = subprocess.check_output(["nm", "-D", "--undefined-only", P.LIB_PATH]).decode()
    syms = {l.split()[-1].split("@")[0] for l in out.splitlines() if l.strip()}
    alloc = {s for s in syms if s.startswith("hip") and ("Malloc" in s or "Free" in s or "Alloc" in s)}
    assert alloc <= {"hipHostMalloc", "hipHostFree"}, alloc


def test_strerror(L):
    for code in range(7):
        assert L.laph_strerror(code)
    assert L.laph_strerror(99) == b"unknown status"


@pytest.mark.parametrize("spec,nt,nv", [("TF,SF,LI8", 128, 112), ("(TI16, SF, LI8)", 128, 112),
                                        ("T1,S1,LB4", 8, 8), ("TB2,SI2,LF", 8, 48), ("TI8,SB4,LI6", 32, 48)])
def test_parse_matches_oracle(L, spec, nt, nv):
    import paper_1104_3870_amd as P

    d = P.laph_parse_dilution(spec, nt, nv)
    ref = oracle.parse_dilution(spec, nt, nv)
    got = [d.type[0], d.J[0], d.type[1], d.J[1], d.type[2], d.J[2]]
    for k in range(3):  # J is ignored for "1" and "F"
        if ref[2 * k] in (0, 1):
            got[2 * k + 1] = ref[2 * k + 1] = 0
    assert got == ref
    assert P.laph_dilution_count(d, nt, nv) == oracle.dilution_count(ref, nt, nv)


@pytest.mark.parametrize("spec,code", [("TI3,SF,LF", 2), ("TF,SB3,LF", 2), ("SF,TF,LF", 1), ("TF,SF", 1),
                                       ("TF,SF,LF,X", 1), ("TQ2,SF,LF", 1), ("TI0,SF,LF", 1)])
def test_parse_errors(L, spec, code):
    import paper_1104_3870_amd as P

    with pytest.raises(P.LaphError) as e:
        P.laph_parse_dilution(spec, 8, 8)
    assert e.value.code == code


def test_create_rejects_odd_extents(L):
    import paper_1104_3870_amd as P

    h = ctypes.c_void_p()
    assert L.laph_create(ctypes.byref(h), ctypes.byref(P.laph_geom(5, 8)), None) == P.LAPH_EINVAL
    assert L.laph_create(ctypes.byref(h), ctypes.byref(P.laph_geom(4, 7)), None) == P.LAPH_EINVAL
    assert L.laph_create(None, ctypes.byref(P.laph_geom(4, 8)), None) == P.LAPH_EINVAL


_STRUCTS = ["laph_geom", "laph_stout", "laph_lanczos", "laph_eig_stats", "laph_dilution", "laph_dirac", "laph_hop",
            "laph_solver", "laph_solve_stats", "laph_adam", "laph_tune_entry", "laph_tune_report",
            "laph_kernel_timing", "laph_timing", "laph_ws_params"]


def test_binding_structs_match_header(tmp_path):
    """The ctypes mirrors of the header's parameter and result structs have the size and
    the field offsets that a C compiler gives the header's own definitions (the binding
    passes them by pointer, so a field added to one side only would shift the rest)."""
    import subprocess

    import paper_1104_3870_amd as P

    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "laph.h"', "int main(void) {"]
    for name in _STRUCTS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in getattr(P, name)._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for name in _STRUCTS:
        S = getattr(P, name)
        assert int(got["%s size" % name]) == ctypes.sizeof(S), name
        for f, _ in S._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(S, f).offset, (name, f)
