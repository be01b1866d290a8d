"""The binding's constants equal the header's (host only): every integer `#define CMBX_<NAME>`
of include/cmbx.h that the ctypes binding mirrors as `<NAME>` has the same value there, so
neither can drift from the other."""
import os
import re

from paper_2507_15703_amd import cmbx

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cmbx.h")


def _defines():
    out = {}
    for line in open(HEADER):
        m = re.match(r"#define CMBX_([A-Z0-9_]+)\s+(\S+)", line)
        if not m:
            continue
        name, val = m.group(1), m.group(2)
        if re.fullmatch(r"-?\d+", val):
            out[name] = int(val)
        elif re.fullmatch(r"CMBX_LANES\(\d+\)", val.replace("ENS_", "")):
            out[name] = int(re.search(r"\d+", val).group()) << 8
    return out


def test_binding_constants_match_header():
    defs = _defines()
    checked = 0
    for name, value in defs.items():
        if hasattr(cmbx, name):
            assert getattr(cmbx, name) == value, name
            checked += 1
    # the options, dtypes, interpolants, errors, modes and slab choices at least
    for name in ("OPT_FIXED_DIRS", "OPT_PLAN_Z", "SLAB_OPT_DIRECT", "ENS_PIPELINED", "ENS_TWO_LANES", "TRICUBIC",
                 "F64", "ESTATE", "SLAB_HYBRID", "ENS_MAX_LANES"):
        assert name in defs and hasattr(cmbx, name), name
    assert checked >= 25


def test_direct_modes_match_header():
    defs = _defines()
    assert cmbx._DIRECT == {"auto": defs["SLAB_DIRECT_AUTO"], "never": defs["SLAB_DIRECT_NEVER"],
                            "always": defs["SLAB_DIRECT_ALWAYS"]}
