"""C-ABI checks that need no GPU: the library loads, exports every function
``include/ebe.h`` declares, reports statuses, carries the paper's solver
defaults, and rejects invalid meshes in its host-side validation (which runs
before any device call)."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1710_08679_amd import ebe, meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return ebe.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "ebe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebe_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported(lib):
    names = header_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ebe.EXPORTED)


def test_status_strings_and_build_info(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10):
        s = lib.ebe_status_string(code).decode()
        assert s and s != "unknown status"
    assert b"gfx950" in lib.ebe_build_info()


def test_default_options_follow_table2(lib):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table2_inner_loops.json")))
    o = ebe.default_opts()
    assert o.precond == ebe.PREC_MG3 and o.mode == ebe.MODE_MIXED
    assert o.inner_eps[0] == g["levels"]["0"]["tolerance"]
    assert o.inner_eps[1] == g["levels"]["1"]["tolerance"]
    assert o.inner_max[0] == g["levels"]["0"]["max_iterations"]
    assert o.inner_max[1] == g["levels"]["1"]["max_iterations"]
    assert o.inner_eps[2] == g["levels"]["2"]["tolerance"]
    assert o.inner_max[2] == g["levels"]["2"]["max_iterations"]
    assert o.tol == g["outer_tolerance"]["value"]


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures match the C header, field by field:
    a C program built from include/ebe.h prints sizes and offsets."""
    assert ctypes.sizeof(ebe.PcgOpts) == 80
    assert ctypes.sizeof(ebe.PcgStats) == 64
    fields = {"ebe_pcg_opts": ebe.PcgOpts, "ebe_pcg_stats": ebe.PcgStats}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ebe.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for ln in out:
        if not ln:
            continue
        cname, what, val = ln.split()
        py = fields[cname]
        if what == "size":
            assert ctypes.sizeof(py) == int(val), (cname, "size")
        else:
            assert getattr(py, what).offset == int(val), (cname, what)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in fields.values())


def create(m, **over):
    xyz = over.get("xyz", m.xyz)
    conn = over.get("conn", m.conn)
    nv = over.get("nv", m.n_vertices)
    E = over.get("E", m.young)
    nu = over.get("nu", m.poisson)
    with pytest.raises(ebe.EbeError) as ei:
        ebe.Mesh(xyz, conn, nv, E, nu, curved=over.get("curved", False))
    if "message" in over:
        over["message"].append(str(ei.value))
    return ei.value.status


def test_validation_rejects_bad_meshes(lib):
    m = meshgen.kuhn_mesh(2, 2, 2)
    c = m.conn.copy()
    c[3, 7] = m.n_nodes + 5
    assert create(m, conn=c) == ebe.ERR_INDEX
    c = m.conn.copy()
    c[0, 1], c[0, 2] = m.conn[0, 2], m.conn[0, 1]  # swap two corners -> negative volume
    assert create(m, conn=c) == ebe.ERR_INVERTED
    x = m.xyz.copy()
    x[m.conn[0, 5]] += 0.01  # move an edge node off its midpoint
    assert create(m, xyz=x) == ebe.ERR_CURVED
    E = m.young.copy()
    E[4] = -1.0
    assert create(m, E=E) == ebe.ERR_MATERIAL
    nu = m.poisson.copy()
    nu[4] = 0.5
    assert create(m, nu=nu) == ebe.ERR_MATERIAL
    c = m.conn.copy()
    c[0, 4] = m.conn[0, 0]  # a corner used as an edge node
    assert create(m, conn=c) == ebe.ERR_NUMBERING
    x = m.xyz.copy()
    x[0, 0] = np.nan
    assert create(m, xyz=x) == ebe.ERR_NONFINITE
    assert create(m, nv=m.n_nodes + 1) == ebe.ERR_ARG
    c = m.conn.copy()
    c[c == m.n_nodes - 1] = m.conn[0, 9]  # node n-1 unused (and an edge node reused inconsistently)
    assert create(m, conn=c) in (ebe.ERR_INDEX, ebe.ERR_CURVED)


def test_curved_mesh_validation(lib):
    """ebe_mesh_create_curved accepts edge nodes off their midpoints but checks
    the Jacobian of each element's quadratic map at its quadrature points and
    nodes; the other checks are those of ebe_mesh_create."""
    m = meshgen.kuhn_mesh(2, 2, 2)
    c0, c1 = m.conn[0, 0], m.conn[0, 1]
    x = m.xyz.copy()
    # the edge node of edge (0, 1) past the quarter point toward corner 0:
    # the map folds over, det J < 0 at corner 0
    x[m.conn[0, 4]] = m.xyz[c0] + 0.1 * (m.xyz[c1] - m.xyz[c0])
    msg = []
    assert create(m, xyz=x, curved=True, message=msg) == ebe.ERR_INVERTED
    assert "det J" in msg[0] and "ebe_mesh_create_curved" in msg[0]
    assert create(m, xyz=x) == ebe.ERR_CURVED
    c = m.conn.copy()
    c[0, 1], c[0, 2] = m.conn[0, 2], m.conn[0, 1]
    assert create(m, conn=c, curved=True) == ebe.ERR_INVERTED
    E = m.young.copy()
    E[2] = 0.0
    assert create(m, E=E, curved=True) == ebe.ERR_MATERIAL


def test_null_arguments_are_rejected(lib):
    out = ctypes.c_void_p()
    st = lib.ebe_mesh_create(None, 10, 4, None, 1, None, None, None, None, ctypes.byref(out))
    assert st == ebe.ERR_ARG
    assert out.value is None
    assert b"null" in lib.ebe_last_error()
    assert lib.ebe_matvec(None, 0, 1, None, None, 0, None) == ebe.ERR_ARG
    assert lib.ebe_pcg_solve(None, 1, None, None, None, None, None) == ebe.ERR_ARG
    b = ctypes.c_void_p()
    assert lib.ebe_batch_create(None, 0, None, ctypes.byref(b)) == ebe.ERR_ARG
    assert lib.ebe_autotune(None, 0, ebe.F32, 4, None, None) == ebe.ERR_ARG
    assert lib.ebe_set_product_form(None, 0, ebe.F32, 4, ebe.FORM_GATHER) == ebe.ERR_ARG
    f = ctypes.c_int32()
    assert lib.ebe_get_product_form(None, 0, ebe.F32, 4, ctypes.byref(f)) == ebe.ERR_ARG
    assert lib.ebe_batch_solve(None, None, None, None, None, None) == ebe.ERR_ARG
    assert lib.ebe_adjoint_grad(None, ebe.F64, 1, None, None, None, None) == ebe.ERR_ARG
    assert lib.ebe_level2_info(None, None, None) == ebe.ERR_ARG
    assert lib.ebe_matvec_l2(None, ebe.F32, 1, None, None, 0, None) == ebe.ERR_ARG
    assert lib.ebe_prolong_l2(None, ebe.F32, 1, None, None, None) == ebe.ERR_ARG
    assert lib.ebe_restrict_l2(None, ebe.F32, 1, None, None, None) == ebe.ERR_ARG
