"""Host-side checks of libnsn.so that need no GPU: every symbol declared in
include/nsn.h is exported, and descriptor validation in nsn_query_workspace
rejects malformed inputs with NSN_EINVAL / NSN_EUNSUPPORTED."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import scene_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1907_04587_amd import _lib as L
    return L, L.lib()


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    header = open(os.path.join(ROOT, "include", "nsn.h")).read()
    names = sorted(set(re.findall(r"\b(nsn_\w+)\s*\(", header)))
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _query(envs):
    from paper_1907_04587_amd.scene import _Marshal
    L, lib = _lib()
    m = _Marshal(envs)
    n = C.c_size_t(0)
    st = lib.nsn_query_workspace(m.c, len(envs), None, C.byref(n))
    return st, n.value, lib.nsn_last_error().decode()


def test_workspace_query_valid_scenes():
    st, n, _ = _query([si.cube_stack(0)])
    assert st == 0 and n > 0
    st2, n2, _ = _query([si.cube_stack(0), si.tet_block_with_boxes(0, cells=3, n_boxes=2)])
    assert st2 == 0 and n2 > n


@pytest.mark.parametrize("mutate,expect", [
    (lambda d: d.tet_ids.__setitem__((0, 1), 99), -1),
    (lambda d: d.tet_material.__setitem__((0, 1), 0.5), -1),
    (lambda d: d.tet_material.__setitem__((0, 0), -1.0), -1),
])
def test_workspace_query_rejects_bad_tets(mutate, expect):
    d = si.single_tet()
    mutate(d)
    st, _, msg = _query([d])
    assert st == expect and "tet" in msg


def test_workspace_query_rejects_bad_rigid_and_joint():
    d = si.cube_stack(n=2)
    d.rigid_inertia[0, 2] = 0.0
    st, _, msg = _query([d])
    assert st == -1 and "inertia" in msg
    d = si.pendulum_drive()
    d.joint_body[0] = (0, 0)
    st, _, msg = _query([d])
    assert st == -1 and "joint" in msg
    d = si.cube_stack(n=1)
    d.rigid_mass[0] = -1.0
    st, _, _ = _query([d])
    assert st == -1


def test_python_layer_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1907_04587_amd import _lib as L
    monkeypatch.setattr(L, "_L", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L.lib()


def test_record_types_match_c_structs(tmp_path):
    """The binding's numpy record types and ctypes structures have the sizes and field
    offsets of the C structs in include/nsn.h (compiled here with the host C
    compiler).  A stale mirror lets the library write past a host buffer."""
    import shutil
    import subprocess

    from paper_1907_04587_amd import _lib as L
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(ROOT, "include")
    fields = {"nsn_step_stats": L.STATS_DTYPE, "nsn_accum": L.ACC_DTYPE}
    cstructs = {"nsn_env_desc": L.EnvDescC, "nsn_solver_params": L.ParamsC}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "nsn.h"', "int main(void) {"]
    names = {st: [n for n in dt.names if n != "pad"] for st, dt in fields.items()}
    names.update({st: [f[0] for f in cls._fields_] for st, cls in cstructs.items()})
    for st, ns in names.items():
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for name in ns:
            lines.append(f'  printf("{st} {name} %zu\\n", offsetof({st}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            st, name, val = ln.split()
            got[(st, name)] = int(val)
    for st, dt in fields.items():
        assert got[(st, "size")] == dt.itemsize, st
        for name in dt.names:
            if name != "pad":
                assert got[(st, name)] == dt.fields[name][1], (st, name)
    for st, cls in cstructs.items():
        assert got[(st, "size")] == C.sizeof(cls), st
        for name, _ in cls._fields_:
            assert got[(st, name)] == getattr(cls, name).offset, (st, name)


def _query_p(envs, params):
    from paper_1907_04587_amd.scene import _Marshal, params_c
    L, lib = _lib()
    m = _Marshal(envs)
    n = C.c_size_t(0)
    pc = params_c(params) if params is not None else None
    st = lib.nsn_query_workspace(m.c, len(envs), C.byref(pc) if pc is not None else None, C.byref(n))
    return st, n.value


def test_workspace_query_reserves_optional_buffers():
    """The parameters decide the optional buffers: island mode and line search each
    add to the workspace; NULL parameters are the defaults; bad parameters are
    rejected."""
    envs = [si.cube_stack(0), si.tet_block_with_boxes(0, cells=3, n_boxes=2)]
    st0, n0 = _query_p(envs, None)
    st1, n1 = _query_p(envs, si.SolverParams())
    st2, n2 = _query_p(envs, si.SolverParams(islands=1))
    st3, n3 = _query_p(envs, si.SolverParams(line_search=1))
    assert st0 == st1 == st2 == st3 == 0
    assert n0 == n1 < n2 and n1 < n3
    st, _ = _query_p(envs, si.SolverParams(watchdog=2))
    assert st == -1
    st, _ = _query_p(envs, si.SolverParams(ncp=5))
    assert st == -1
