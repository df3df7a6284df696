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
    assert L.heston_abi_version() == hm.ABI_VERSION
    assert L.heston_status_str(-1) == b"invalid argument"
    o = hm.COpts()
    assert L.heston_default_opts(ctypes.byref(o)) == 0
    assert o.struct_size == ctypes.sizeof(hm.COpts)
    assert (o.precision, o.rng, o.scheme, o.greeks) == (0, 0, 0, 3)
    assert o.bump_S0_rel == 0.01 and o.bump_r_abs == 1e-4 and o.bump_T_abs == 1 / 365
    assert L.heston_default_opts(None) == -1


def test_fused_r_bump_range_checked_on_the_host(L):
    """A fused r bump of an arithmetic Asian takes its bumped averages from a
    Taylor series in the bump; outside the series' range (bump_r_abs * T above
    1e-3 in FP64, 3e-3 in FP32) the call is rejected while checking its
    arguments, before any device work."""
    import paper_2309_10477_amd as hm
    from workloads import BASE
    res = hm.CResult()
    for prec, h, T, typ in ((hm.FP64, 2e-3, 1.0, hm.ASIAN_CALL), (hm.FP64, 1e-4, 20.0, hm.ASIAN_PUT),
                            (hm.FP32, 4e-3, 1.0, hm.ASIAN_CALL)):
        o = hm._OptsHolder(hm.Options(precision=prec, bump_r_abs=h), 8)
        cp = hm._cparams(dict(BASE, T=T))
        st = L.heston_price_greeks_noalloc(ctypes.byref(cp), typ, 1000, 8, 1, ctypes.byref(o.c),
                                           None, ctypes.byref(res))
        assert st == -1, (prec, h, T)
        assert b"bump_r_abs" in L.heston_last_error()


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


def test_result_unpacking_matches_the_struct():
    """The binding reads heston_result as one packed record: every field set to
    a distinct value comes back under its own name."""
    import paper_2309_10477_amd as hm
    r = hm.CResult()
    v = 1.0
    for n in hm.EST_NAMES + ("cv_price",):
        getattr(r, n).value, getattr(r, n).std_err = v, v + 0.5
        v += 1.0
    for k in range(7):
        r.adj[k].value, r.adj[k].std_err = v, v + 0.5
        v += 1.0
    r.n_paths, r.valid_mask, r.reserved = 12345678901, hm.VALID_CONTROL | hm.VALID_ADJOINT, 7
    r.device_ms, r.cv_beta, r.cv_mean, r.latency_ms = 101.5, 102.5, 103.5, 104.5
    d = hm._result_dict(r)
    for n in hm.EST_NAMES:
        assert d[n] == (getattr(r, n).value, getattr(r, n).std_err), n
    assert d["adj"] == [(r.adj[k].value, r.adj[k].std_err) for k in range(7)]
    assert d["cv_price"] == (r.cv_price.value, r.cv_price.std_err)
    assert (d["n_paths"], d["valid_mask"]) == (r.n_paths, r.valid_mask)
    assert (d["device_ms"], d["cv_beta"], d["cv_mean"], d["latency_ms"]) == (101.5, 102.5, 103.5,
                                                                               104.5)
    r.valid_mask = hm.VALID_PRICE
    assert "cv_price" not in hm._result_dict(r)


def test_options_holder_cache_keys_on_every_field():
    import paper_2309_10477_amd as hm
    a = hm._OptsHolder.get(hm.Options(precision=hm.FP32), 50)
    assert hm._OptsHolder.get(hm.Options(precision=hm.FP32), 50) is a
    for other in (hm.Options(precision=hm.FP64), hm.Options(precision=hm.FP32, bump_T_abs=0.01),
                  hm.Options(precision=hm.FP32, fixings=[5, 10]),
                  hm.Options(precision=hm.FP32, scheme=hm.QE)):
        b = hm._OptsHolder.get(other, 50)
        assert b is not a
        assert (b.c.precision, b.c.scheme, b.c.bump_T_abs, b.c.n_fixings) == (
            other.precision, other.scheme, other.bump_T_abs,
            0 if other.fixings is None else len(other.fixings))
