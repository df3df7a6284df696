"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: only host-side calls that launch nothing)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heston.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(heston_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    import paper_2309_10477_amd as hm
    return hm.lib()


def test_every_declared_function_is_exported(L):
    names = declared_functions()
    assert "heston_price_greeks" in names and len(names) >= 9
    for n in names:
        assert hasattr(L, n), n


def test_host_only_calls(L):
    import paper_2309_10477_amd as hm
    import paper_2309_10477_amd as hm
    assert L.heston_abi_version() == hm.ABI_VERSION
    assert L.heston_status_str(-1) == b"invalid argument"
    o = hm.COpts()
    assert L.heston_default_opts(ctypes.byref(o)) == 0
    assert o.struct_size == ctypes.sizeof(hm.COpts)
    assert (o.precision, o.rng, o.scheme, o.greeks) == (0, 0, 0, 3)
    assert o.bump_S0_rel == 0.01 and o.bump_r_abs == 1e-4 and o.bump_T_abs == 1 / 365
    assert L.heston_default_opts(None) == -1


def test_struct_layout_matches_header():
    """Sizes of the ABI structs as laid out by a C compiler."""
    import subprocess
    import tempfile
    import paper_2309_10477_amd as hm
    src = ('#include "heston.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(void){'
           'printf("%zu %zu %zu %zu %zu %zu %zu %d %d %d\\n", sizeof(heston_params),'
           ' sizeof(heston_opts), sizeof(heston_result), offsetof(heston_opts, fixing_steps),'
           ' offsetof(heston_result, device_ms), offsetof(heston_opts, control_variate),'
           ' offsetof(heston_result, cv_mean), HESTON_CONTROL_GEOMETRIC, HESTON_VALID_CONTROL,'
           ' HESTON_CONTROL_MAX_FIXINGS); printf("%zu\\n", offsetof(heston_result, latency_ms));'
           ' return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(hm.CParams), ctypes.sizeof(hm.COpts), ctypes.sizeof(hm.CResult),
            hm.COpts.fixing_steps.offset, hm.CResult.device_ms.offset,
            hm.COpts.control_variate.offset, hm.CResult.cv_mean.offset, hm.CONTROL_GEOMETRIC,
            hm.VALID_CONTROL, hm.CONTROL_MAX_FIXINGS, hm.CResult.latency_ms.offset]
    assert got == want


def test_enum_constants_match_binding():
    """The binding's constants are the header's values."""
    import subprocess
    import tempfile
    import paper_2309_10477_amd as hm
    names = ["HESTON_ABI_VERSION", "HESTON_EURO_CALL", "HESTON_EURO_PUT", "HESTON_ASIAN_CALL", "HESTON_ASIAN_PUT",
             "HESTON_GEO_ASIAN_CALL", "HESTON_GEO_ASIAN_PUT", "HESTON_FP64", "HESTON_FP32", "HESTON_RNG_PHILOX", "HESTON_RNG_SOBOL_BRIDGE",
             "HESTON_FULL_TRUNCATION", "HESTON_ABSORPTION", "HESTON_QE",
             "HESTON_EULER_FULL_TRUNCATION", "HESTON_EULER_ABSORPTION",
             "HESTON_PARTIAL_TRUNCATION", "HESTON_REFLECTION", "HESTON_EXACT",
             "HESTON_EXACT_MAX_STEPS",
             "HESTON_GREEKS_PATHWISE", "HESTON_GREEKS_BUMP_FUSED", "HESTON_GREEKS_BUMP_PLAIN"]
    src = ('#include "heston.h"\n#include <stdio.h>\nint main(void){printf("'
           + " ".join(["%d"] * len(names)) + '\\n", ' + ", ".join(f"(int){n}" for n in names)
           + "); return 0;}\n")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [hm.ABI_VERSION, hm.EURO_CALL, hm.EURO_PUT, hm.ASIAN_CALL, hm.ASIAN_PUT, hm.GEO_ASIAN_CALL,
            hm.GEO_ASIAN_PUT, hm.FP64, hm.FP32, hm.PHILOX, hm.SOBOL_BRIDGE, hm.FULL_TRUNCATION, hm.ABSORPTION,
            hm.QE, hm.EULER_FULL_TRUNCATION, hm.EULER_ABSORPTION, hm.PARTIAL_TRUNCATION,
            hm.REFLECTION, hm.EXACT, hm.EXACT_MAX_STEPS, hm.GREEKS_PATHWISE, hm.GREEKS_BUMP_FUSED,
            hm.GREEKS_BUMP_PLAIN]
    assert got == want
