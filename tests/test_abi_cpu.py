"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
declared symbol, validates arguments and reports a missing device as an error."""
import ctypes
import os
import re

import pytest

from paper_2503_09203_amd import mgx
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(mgx_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = mgx.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(mgx.SIGNATURES)


def test_loader_refuses_a_library_built_from_other_sources(tmp_path):
    """The library carries the digest of the sources it was compiled from; the loader
    accepts it against an identical copy of the sources and refuses it once one byte of a
    kernel source differs."""
    import shutil
    from paper_2503_09203_amd import build as B
    L = mgx.lib()
    assert mgx.mgx_build_hash() == B.source_hash() != "unknown"
    pkg = os.path.basename(B.PKG)
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    shutil.copytree(os.path.join(B.PKG, "csrc"), tmp_path / pkg / "csrc")
    mgx.check_build(L, str(tmp_path))
    f = tmp_path / pkg / "csrc" / "step.hpp"
    f.write_text(f.read_text() + "\n")
    with pytest.raises(ImportError, match="other sources"):
        mgx.check_build(L, str(tmp_path))


def test_version_and_status_strings():
    assert mgx.mgx_version() >= 100
    assert mgx.lib().mgx_status_string(mgx.MGX_E_INVALID) == b"invalid argument"


def test_step_cost_counts():
    f6, o6 = mgx.mgx_step_cost(6)
    f8, o8 = mgx.mgx_step_cost(8)
    assert 250 < f6 < 500 and 150 < o6 < 350
    # each extra thruster: lag (1 sub + 1 fma), thrust (1 mul), six fused multiply-adds
    assert f8 - f6 == 2 * (1 + 2 + 1 + 12)
    with pytest.raises(mgx.MgxError):
        mgx.mgx_step_cost(9)
    # shaped thrust per thruster: |n| - dead zone (1 flop), max, mag^2 (1 flop), the
    # direction's gain ratio (select, 1-flop product), sign: +2 flops and +5 operations
    # over the plain n|n|
    fs, os_ = mgx.mgx_step_cost(6, mgx.COST_SHAPED)
    assert fs - f6 == 2 * 6 and os_ - o6 == 5 * 6
    # the reverse sweep given the step's stored forward quantities: per extra thruster six
    # fused multiply-adds into the thrust adjoint, its chain through the derivative
    # (1 product + 1 sum), the command adjoint (1 product) and the carried rotor adjoint
    # (1 sub + 1 product)
    v6, w6 = mgx.mgx_vjp_cost(6)
    v8, w8 = mgx.mgx_vjp_cost(8)
    assert f6 < v6 < 4 * f6 and o6 < w6
    assert v8 - v6 == 2 * (12 + 2 + 1 + 2)
    with pytest.raises(mgx.MgxError):
        mgx.mgx_vjp_cost(0)


def test_class_validation():
    c = synth.plain_class()
    cid = mgx.mgx_class_define(c)
    assert cid >= 0
    bad = synth.plain_class()
    bad.k = bad.k.copy()
    bad.k[0] = -1.0
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_class_define(bad)
    assert e.value.status == mgx.MGX_E_INVALID and "k must be > 0" in str(e.value)
    bad = synth.plain_class()
    bad.e = bad.e.copy()
    bad.e[2] = 0.0
    with pytest.raises(mgx.MgxError):
        mgx.mgx_class_define(bad)


def test_batch_create_validates_before_touching_a_device():
    cid = mgx.mgx_class_define(synth.plain_class())
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_batch_create([cid], [0], 0.01)
    assert e.value.status == mgx.MGX_E_INVALID
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_batch_create([cid], [10], -1.0)
    assert e.value.status == mgx.MGX_E_INVALID
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_batch_create([12345], [10], 0.01)
    assert e.value.status == mgx.MGX_E_INVALID


def test_batch_create_without_gpu_is_a_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    cid = mgx.mgx_class_define(synth.plain_class())
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_batch_create([cid], [10], 0.01)
    assert e.value.status == mgx.MGX_E_DEVICE


def test_null_batch_calls_are_rejected():
    L = mgx.lib()
    assert L.mgx_batch_step(None, None, 1, 0, 1, 1, 0, None, None) == mgx.MGX_E_INVALID
    assert L.mgx_batch_destroy(None) == mgx.MGX_OK
    d = mgx.StationDesc(**mgx.STATION_DEFAULTS)
    h = ctypes.c_void_p()
    assert L.mgx_station_create(None, ctypes.byref(d), ctypes.byref(h)) == mgx.MGX_E_INVALID
    assert L.mgx_station_step(None, None, 1, None, None, None, None, None) == mgx.MGX_E_INVALID
    assert L.mgx_station_reset(None, 0, None) == mgx.MGX_E_INVALID
    assert L.mgx_station_destroy(None) == mgx.MGX_OK
    assert L.mgx_station_resample(None, None, None, 0) == mgx.MGX_E_INVALID


def test_binding_structures_match_the_header(tmp_path):
    """Every ctypes mirror has the size of its C struct (compiled from the header with
    gcc), so a field added to one side only cannot go unnoticed."""
    pairs = {"mgx_class_desc": mgx.ClassDesc, "mgx_batch_desc": mgx.BatchDesc, "mgx_layout": mgx.Layout,
             "mgx_dr_dist": mgx.DrDist, "mgx_dr_spec": mgx.DrSpec,
             "mgx_env_params": mgx.EnvParams, "mgx_stats": mgx.Stats, "mgx_launch_shape": mgx.LaunchShape,
             "mgx_server_desc": mgx.ServerDesc, "mgx_request": mgx.Request,
             "mgx_request_status": mgx.RequestStatus, "mgx_server_stats": mgx.ServerStats,
             "mgx_station_desc": mgx.StationDesc}
    src = tmp_path / "sizes.c"
    body = "".join(f'    printf("{n} %zu\\n", sizeof({n}));\n' for n in pairs)
    src.write_text(f'#include <stdio.h>\n#include "mgx.h"\nint main(void) {{\n{body}    return 0;\n}}\n')
    exe = tmp_path / "sizes"
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    sizes = {line.split()[0]: int(line.split()[1]) for line in out.splitlines()}
    for name, cls in pairs.items():
        assert ctypes.sizeof(cls) == sizes[name], (name, ctypes.sizeof(cls), sizes[name])


def test_propeller_variant_validation():
    bad = synth.propeller_variants(synth.plain_class())
    bad.k_rev = bad.k_rev.copy()
    bad.k_rev[2] = -1.0
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_class_define(bad)
    assert "k_rev must be >= 0" in str(e.value)
    bad = synth.propeller_variants(synth.plain_class())
    bad.reaction = bad.reaction.copy()
    bad.reaction[0] = float("nan")
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_class_define(bad)
    assert "reaction must be finite" in str(e.value)
    assert mgx.mgx_class_define(synth.propeller_variants(synth.plain_class())) >= 0


def test_fin_class_validation():
    import dataclasses
    assert mgx.mgx_class_define(synth.rudder_class()) >= 0
    cases = [("span", lambda c: c.span.__setitem__(1, 0.0), "zero-length span"),
             ("span", lambda c: c.span.__setitem__(2, [1.0, 0.0, 0.0]), "chord parallel to the span"),
             ("fin_max", lambda c: c.fin_max.__setitem__(3, 2.0), "fin_max must be in (0, pi/2]"),
             ("fin_lift", lambda c: c.fin_lift.__setitem__(4, -1.0), "lift and drag gains"),
             ("kind", lambda c: c.kind.__setitem__(1, 7), "kind must be")]
    for field, spoil, msg in cases:
        c = synth.rudder_class()
        c = dataclasses.replace(c, **{field: getattr(c, field).copy()})
        spoil(c)
        with pytest.raises(mgx.MgxError) as e:
            mgx.mgx_class_define(c)
        assert msg in str(e.value), (field, str(e.value))


def test_class_step_cost_follows_the_body():
    """The per-class count equals the generic one for plain and shaped classes; a class
    with fins counts the fin forces on top (and no thrust for its fins)."""
    plain = mgx.mgx_class_step_cost(mgx.mgx_class_define(synth.plain_class()))
    assert plain == mgx.mgx_step_cost(6)
    shaped = mgx.mgx_class_step_cost(mgx.mgx_class_define(synth.propeller_variants(synth.plain_class())))
    assert shaped == mgx.mgx_step_cost(6, mgx.COST_SHAPED)
    rudder = mgx.mgx_class_step_cost(mgx.mgx_class_define(synth.rudder_class()))
    one_prop = mgx.mgx_step_cost(1, mgx.COST_SHAPED)
    assert rudder[0] > one_prop[0] + 4 * 40 and rudder[1] > one_prop[1] + 4 * 30
