"""The C ABI (no GPU needed): the built library loads, exports every entry
point the public header declares, and the Python binding's structs match the
header's layout (checked by compiling the header with the host compiler)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcc_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding_list():
    from paper_2407_19151_amd import native
    assert declared_functions() == sorted(native.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2407_19151_amd import native
    lib = native.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert set(declared_functions()) <= exported


def test_host_only_calls():
    """Entry points that touch no GPU: defaults and status strings."""
    from paper_2407_19151_amd import native
    lib = native.load()
    p = native.mcc_params()
    lib.mcc_default_params(C.byref(p))
    assert p.method == native.MCC_N97 and p.precision == native.MCC_FP64
    assert p.moment_correction == 1 and p.sort_by_weight == 1 and p.max_passes == 1
    assert p.f_E == 0.05 and p.eps0 == 1.0
    for code in (0, -1, -2, -3, -4, -5):
        s = lib.mcc_status_string(code)
        assert s and len(s) >= 2


def test_struct_layout_matches_header():
    from paper_2407_19151_amd import native
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "mcc.h"
#define F(T, m) printf("%s.%s %zu %zu\n", #T, #m, offsetof(T, m), sizeof(((T*)0)->m));
int main(void) {
  F(mcc_params, method) F(mcc_params, precision) F(mcc_params, relativistic)
  F(mcc_params, moment_correction) F(mcc_params, sort_by_weight) F(mcc_params, max_passes)
  F(mcc_params, on_failure) F(mcc_params, diagnostics) F(mcc_params, pairing)
  F(mcc_params, f_E) F(mcc_params, eps0) F(mcc_params, c)
  F(mcc_stats, pairs) F(mcc_stats, corr_pairs) F(mcc_stats, failed)
  F(mcc_stats, collisions) F(mcc_stats, max_rel_dP) F(mcc_stats, max_rel_dE)
  F(mcc_species, mass) F(mcc_species, charge) F(mcc_collision, a) F(mcc_collision, b)
  F(mcc_collision, cross_section)
  printf("sizeof mcc_params %zu\nsizeof mcc_stats %zu\n", sizeof(mcc_params), sizeof(mcc_stats));
  printf("sizeof mcc_species %zu\nsizeof mcc_collision %zu\n", sizeof(mcc_species),
         sizeof(mcc_collision));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    structs = {"mcc_params": native.mcc_params, "mcc_stats": native.mcc_stats,
               "mcc_species": native.mcc_species, "mcc_collision": native.mcc_collision}
    for line in filter(None, lines):
        if line.startswith("sizeof"):
            _, name, size = line.split()
            assert C.sizeof(structs[name]) == int(size), line
            continue
        field, off, size = line.split()
        sname, m = field.split(".")
        desc = getattr(structs[sname], m)
        assert (desc.offset, desc.size) == (int(off), int(size)), line
