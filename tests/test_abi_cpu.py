"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and rejects bad arguments before touching
the device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "agal.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"AGAL_API\s+[\w\s\*]+?\b(agal_\w+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = _declared()
    for n in ("agal_import_faces", "agal_bin_faces", "agal_near_wall_refine", "agal_link_fractions",
              "agal_link_fractions_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2502_16310_amd as agal
    out = subprocess.run(["nm", "-D", "--defined-only", agal.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in out.stdout.splitlines() if " T " in line}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    # nothing else leaks out of the library
    extra = sorted(n for n in exported if not n.startswith("agal_"))
    assert not extra, extra[:10]


def test_binding_has_the_same_names():
    import paper_2502_16310_amd as agal
    for n in _declared():
        assert callable(getattr(agal, n)), n


def test_lattice_vectors_match_oracle(orc):
    import paper_2502_16310_amd as agal
    for Q in (9, 19, 27):
        lib = np.array(agal.agal_lattice_vectors(Q))
        assert np.array_equal(lib, orc.lattice(Q))


def test_invalid_arguments_rejected_on_host():
    import paper_2502_16310_amd as agal
    lib = agal._lib
    out = C.c_void_p()
    assert lib.agal_import_faces(None, 3, 1, 3, None, 1, None, C.byref(out)) == agal.AGAL_EINVAL
    assert lib.agal_lattice_vectors(7, (C.c_int32 * 30)()) == agal.AGAL_EINVAL
    assert "unknown lattice" in agal.agal_last_error()
    assert lib.agal_bin_faces(None, None, None, 4, None, C.byref(out)) == agal.AGAL_EINVAL
    assert lib.agal_link_fractions(None, None, None, 19, None, C.byref(out)) == agal.AGAL_EINVAL
    assert lib.agal_near_wall_refine(None, None, None, None, C.byref(out)) == agal.AGAL_EINVAL
    with pytest.raises(agal.AgalError):
        agal.agal_lattice_vectors(8)
    for s in range(6):
        assert agal.agal_status_string(s).startswith("AGAL_")


def test_build_flags_keep_fp_exact():
    from paper_2502_16310_amd import build
    assert "-ffp-contract=off" in build.CXXFLAGS
    assert "--offload-arch=gfx950" in build.CXXFLAGS
    i = build.CXXFLAGS.index("-packed-fp32-ops")
    assert build.CXXFLAGS[i - 1] == "-Xclang" and build.CXXFLAGS[i - 2] == "-target-feature"
