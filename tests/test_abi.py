"""Host-only checks of the C-ABI library: it loads, exports every function the
header declares, and the Python structure layouts match the C ones (the
layout is measured by compiling a small C probe of include/ddamg.h with gcc).
No compute call is made here: those need the GPU."""
import ctypes
import os
import subprocess
import tempfile

import pytest

import paper_2201_03872_amd as dd


def test_library_exports_every_declared_symbol():
    lib = dd.load()
    names = dd.header_symbols()
    assert "ddamg_setup" in names and "ddamg_solve" in names and "ddamg_apply_op" in names
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_is_static_and_host_only():
    lib = dd.load()
    for code in (dd.OK, dd.NOT_CONVERGED, dd.EINVAL, dd.ENOMEM, dd.EDEVICE, dd.EBREAKDOWN, dd.ESTATE, 1234):
        assert lib.ddamg_strerror(code)


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "ddamg.h"
#define F(s, f) printf(#s "." #f " %zu %zu\n", offsetof(s, f), sizeof(((s*)0)->f));
int main(void) {
  printf("ddamg_params %zu\n", sizeof(ddamg_params));
  printf("ddamg_col_info %zu\n", sizeof(ddamg_col_info));
  printf("ddamg_stats %zu\n", sizeof(ddamg_stats));
%s
  return 0;
}
"""


def test_struct_layouts_match_header():
    fields = []
    for sname, cls in (("ddamg_params", dd.Params), ("ddamg_col_info", dd.ColInfo), ("ddamg_stats", dd.Stats)):
        for f, _ in cls._fields_:
            fields.append(f"  F({sname}, {f})")
    src = PROBE.replace("%s", "\n".join(fields))
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(dd.HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        parts = line.split()
        if len(parts) == 2:
            got[parts[0]] = int(parts[1])
        elif len(parts) == 3:
            got[parts[0]] = (int(parts[1]), int(parts[2]))
    assert got["ddamg_params"] == ctypes.sizeof(dd.Params)
    assert got["ddamg_col_info"] == ctypes.sizeof(dd.ColInfo)
    assert got["ddamg_stats"] == ctypes.sizeof(dd.Stats)
    for sname, cls in (("ddamg_params", dd.Params), ("ddamg_col_info", dd.ColInfo), ("ddamg_stats", dd.Stats)):
        for f, _ in cls._fields_:
            d = getattr(cls, f)
            assert got[f"{sname}.{f}"] == (d.offset, d.size), (sname, f)


def test_default_params_are_the_papers_tolerances():
    p = dd.default_params()
    assert p.tol == 1e-10
    assert abs(p.r_m - 7e-2) < 1e-15 and abs(p.r_b - 1e-1) < 1e-15
    assert p.coarse_mu_factor == 1.0


@pytest.mark.parametrize("kw,reason", [
    (dict(sap_oddeven=1, sap_block=(2, 2, 2, 2)), "odd-even SAP"),
    (dict(sap_oddeven=1, csw=1.0), "odd-even SAP"),
    (dict(sap_oddeven=2), "sap_oddeven"),
    (dict(csw=float("nan")), "csw"),
    (dict(n_levels=4), "n_levels"),
    (dict(kappa=0.0), "kappa"),
    (dict(coarse_gamma5=3), "coarse_gamma5"),
    (dict(col_tile=16), "col_tile"),
    (dict(dims=(8, 8, 8, 6)), "SAP block extents must divide"),
    (dict(sap_block=(2, 2, 2, 4)), "16 or 256 sites"),
    (dict(n_levels=2, agg=[(4, 4, 4, 4)], n_tv=[3]), "test vector counts"),
    (dict(n_levels=2, agg=[(2, 2, 2, 2)], n_tv=[8]), "first-level aggregates"),
    (dict(sap_mr_iters=0), "SAP cycle counts"),
    (dict(outer_restart=64), "outer_restart"),
    (dict(middle_restart=0), "middle_restart"),
    (dict(bottom_restart=64), "bottom_restart"),
    (dict(bottom_restart=10, bottom_dr_k=9), "bottom_dr_k"),
    (dict(coarse_fp16=2), "coarse_fp16"),
    (dict(transfer_fp16=-1), "transfer_fp16"),
    (dict(setup_boot=17), "setup_boot"),
    (dict(setup_fine_iters=64), "setup_fine_iters"),
    (dict(setup_coarse_iters=0), "setup_coarse_iters"),
    (dict(tol=0.0), "tolerances"),
    (dict(precision=7), "precision"),
    (dict(smoother=5), "smoother"),
    (dict(smoother_cycles=65), "smoother_cycles"),
    (dict(max_active_cols=-1), "max_active_cols"),
    (dict(inner_tol=1.0), "inner_iters / inner_tol"),
])
def test_setup_rejects_bad_parameters_on_the_host(kw, reason):
    """Parameter validation is host logic: ddamg_setup returns DDAMG_EINVAL
    with a message before it touches the device."""
    lib = dd.load()
    p = dd.default_params(**dict(dict(dims=(8, 8, 8, 8), kappa=0.15, n_levels=1, sap_block=(4, 4, 4, 4)), **kw))
    gauge = (ctypes.c_double * 8)()
    h = ctypes.c_void_p()
    st = lib.ddamg_setup(ctypes.byref(p), gauge, 0, None, None, ctypes.byref(h))
    assert st == dd.EINVAL
    assert reason in lib.ddamg_last_error().decode()
    assert not h.value


NULL_PROBE = r"""
import ctypes, json, sys
sys.path.insert(0, sys.argv[1])
import paper_2201_03872_amd as dd
lib = dd.load()
host_only = {"ddamg_default_params", "ddamg_setup", "ddamg_destroy", "ddamg_strerror", "ddamg_last_error"}
out = {}
for name in dd.header_symbols():
    if name in host_only:
        continue
    f = getattr(lib, name)
    args = [1 if t in (ctypes.c_int, ctypes.c_uint64) else 1e-3 if t is ctypes.c_double else None
            for t in f.argtypes]
    out[name] = [f(*args), lib.ddamg_last_error().decode()]
lib.ddamg_destroy(None)
print(json.dumps(out))
"""


def test_every_entry_point_rejects_a_null_context_on_the_host():
    """Every call that takes a context returns DDAMG_EINVAL with a message
    when handed a null context (and null buffers), before it touches the
    device; ddamg_destroy(NULL) is a no-op.  Run in a child process so that a
    crash would fail this test rather than end the suite."""
    import json
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", NULL_PROBE, root], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    got = json.loads(r.stdout.strip().splitlines()[-1])
    expected = set(dd.header_symbols()) - {"ddamg_default_params", "ddamg_setup", "ddamg_destroy",
                                          "ddamg_strerror", "ddamg_last_error"}
    assert set(got) == expected
    for name, (status, msg) in got.items():
        assert status == dd.EINVAL, (name, status, msg)
        assert msg, name
