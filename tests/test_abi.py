"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chem.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(chem_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2105_12070_amd import chem
    if not os.path.exists(chem.LIB_PATH):
        from paper_2105_12070_amd import build
        build.build()
    return chem.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    from paper_2105_12070_amd import chem
    assert sorted(chem.EXPORTED) == names


def test_adjoint_record_budget_setter(L):
    # host-side setting only; restores the default
    assert L.chem_set_adjoint_record_budget(C.c_uint64(0)) == 0
    assert L.chem_set_adjoint_record_budget(C.c_uint64(8 << 30)) == 0


def test_max_n(L):
    assert L.chem_max_n() == 255  # wavefront path up to 64, workgroup path above


def test_invalid_arguments_are_rejected_on_host(L):
    out = C.c_void_p()
    assert L.chem_load_mechanism(None, C.byref(out)) == -1
    assert b"null" in L.chem_last_error()
    assert L.chem_integrate(None, 4, 4, None, None, 1e5, 1e-6, 1e-6, 1e-10, None, None, None, None, None) == -1
    assert L.chem_lu_solve(1, 0, None, None, None, None) == -1


def test_mechanism_validation_on_host(L):
    from paper_2105_12070_amd import chem
    from paper_2105_12070_amd.inputs import WORKLOADS
    m = WORKLOADS["c1_10sp"].mechanism()
    bad = dict(m)
    bad["W"] = m["W"].copy()
    bad["W"][3] = -1.0
    with pytest.raises(chem.ChemError, match="EINVAL"):
        chem.Mechanism(bad)
    bad = dict(m)
    bad["reac"] = m["reac"].copy()
    bad["reac"][0, 0] = 99
    with pytest.raises(chem.ChemError, match="EINVAL"):
        chem.Mechanism(bad)
    bad = dict(m)
    bad["nasa7"] = m["nasa7"].copy()
    bad["nasa7"][2, 1:8] = [-5.0, 0, 0, 0, 0, 0, 0]
    bad["nasa7"][2, 8:15] = [-5.0, 0, 0, 0, 0, 0, 0]
    with pytest.raises(chem.ChemError, match="cp <= 0"):
        chem.Mechanism(bad)
    big = dict(m)
    big["n_species"] = 300
    with pytest.raises(chem.ChemError, match="EUNSUPPORTED"):
        chem.Mechanism(big)


def test_element_balance_is_validated_on_host(L):
    """A reaction that does not conserve an element is rejected before any
    device work; a mechanism without element data skips the check."""
    from paper_2105_12070_amd import chem
    from paper_2105_12070_amd.inputs import WORKLOADS
    m = WORKLOADS["c2_54sp"].mechanism()
    assert m["elem"].shape == (54, 4)
    bad = dict(m)
    bad["prod"] = m["prod"].copy()
    r = int(np.nonzero(m["rtype"] == 0)[0][5])
    bad["prod"][r] = m["prod"][r][::-1]  # same molecules in other slots: still balanced
    try:  # passes validation (without a GPU the upload then fails with another code)
        chem.Mechanism(bad)
    except chem.ChemError as e:
        assert e.code != -1, str(e)
    # swapping a product for another species of different composition breaks balance
    k = int(bad["prod"][r][-1] if bad["prod"][r][-1] >= 0 else bad["prod"][r][0])
    other = int(np.nonzero(np.any(m["elem"] != m["elem"][k], axis=1))[0][0])
    bad["prod"] = bad["prod"].copy()
    bad["prod"][r][bad["prod"][r] == k] = other
    with pytest.raises(chem.ChemError, match="does not conserve element"):
        chem.Mechanism(bad)
    # without element data the check is skipped
    skip = dict(bad)
    skip["elem"] = None
    try:
        chem.Mechanism(skip)
    except chem.ChemError as e:
        assert e.code != -1, str(e)


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of chem_options, chem_refmap and chem_mech_desc have
    the C header's size and field offsets (compiled with gcc here)."""
    import subprocess
    from paper_2105_12070_amd import chem
    structs = {"chem_options": chem.Options, "chem_refmap": chem.RefMap, "chem_mech_desc": chem._Desc}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "chem.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
