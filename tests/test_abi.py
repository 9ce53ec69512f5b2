"""CPU checks of the C ABI: the library loads without a GPU, exports every
function the header declares, and the ctypes structs match the C layouts."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2601_16911_amd import cvw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cvw.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cvw_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = cvw.load()
    names = _declared()
    assert "cvw_residual" in names and "cvw_mesh_build" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(cvw.SYMBOLS)
    assert lib.cvw_abi_version() == 12


def test_struct_layouts_match_header():
    code = r'''
#include <stdio.h>
#include <stddef.h>
#include "cvw.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(cvw_params), sizeof(cvw_mesh_desc),
         sizeof(cvw_mesh_info), offsetof(cvw_params, fixed_gamma), offsetof(cvw_mesh_desc, periodic),
         offsetof(cvw_mesh_info, hx), offsetof(cvw_params, mlp), sizeof(cvw_batch_instance),
         offsetof(cvw_batch_instance, dt), offsetof(cvw_mesh_info, grid_ny), offsetof(cvw_params, bc),
         offsetof(cvw_params, bc_state));
  return 0;
}
'''
    import ctypes as C
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(code)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    exp = [C.sizeof(cvw.ParamsC), C.sizeof(cvw.MeshDescC), C.sizeof(cvw.MeshInfoC),
           cvw.ParamsC.fixed_gamma.offset, cvw.MeshDescC.periodic.offset, cvw.MeshInfoC.hx.offset,
           cvw.ParamsC.mlp.offset, C.sizeof(cvw.BatchInstanceC), cvw.BatchInstanceC.dt.offset,
           cvw.MeshInfoC.grid_ny.offset, cvw.ParamsC.bc.offset, cvw.ParamsC.bc_state.offset]
    assert got == exp


def test_last_error_and_null_arguments_without_gpu():
    lib = cvw.load()
    assert lib.cvw_mesh_build(None, None) == cvw.EINVAL
    assert b"null" in lib.cvw_last_error()
    assert lib.cvw_workspace_bytes(None, None, 0) == 0
    assert lib.cvw_workspace_bytes(None, None, cvw.OP_POS) == 0
    assert lib.cvw_positivity(None, None, None, None, 1e-13, None, 0, None) == cvw.EINVAL
    assert b"null" in lib.cvw_last_error()


def test_params_defaults_marshal():
    import synth
    p = cvw.make_params(synth.Params())
    assert p.eps_vertex == 1e-6 and p.eps_cell == 1e-6 and p.r == 2 and p.c_gamma == 0.9
    assert p.lin_w_vertex == 1e-3 and p.sc_on == 1 and p.q_sensor == 1.0
    assert list(p.bc) == [0, 0]
    q = cvw.make_params(synth.modified_sod_params(), cvw.F64)
    assert list(q.bc) == [synth.BC_INFLOW, synth.BC_WALL]
    assert list(q.bc_state[0])[:3] == pytest.approx([1.0, 0.75, 1.0 / 0.4 + 0.5 * 0.75 ** 2], rel=1e-15)


def test_mesh_plan_without_gpu():
    """cvw_mesh_plan is host work only: a byte count, 256-aligned, reproducible,
    growing with the mesh; cvw_mesh_build_in refuses a buffer that is too small
    before touching it."""
    import ctypes as C
    import synth
    lib = cvw.load()
    a = cvw.mesh_plan(synth.quad_mesh(8, 8), 3, cvw.DG)
    b = cvw.mesh_plan(synth.quad_mesh(8, 8), 3, cvw.DG)
    c = cvw.mesh_plan(synth.quad_mesh(16, 16), 3, cvw.DG)
    assert a == b and a > 0 and a % 256 == 0 and c > a
    d, keep = cvw._mesh_desc(synth.quad_mesh(8, 8), 3, cvw.DG)
    h = C.c_void_p()
    st = lib.cvw_mesh_build_in(C.byref(d), C.c_void_p(4096), 256, C.byref(h))
    assert st == cvw.EINVAL and not h.value
    assert b"too small" in lib.cvw_last_error()
