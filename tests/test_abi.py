"""The C ABI as seen from the host, without a GPU.

* every function declared in include/dg.h is exported by the built library,
  and the Python binding lists exactly those functions;
* the ctypes mirrors of dg_mesh, dg_params and dg_stats have the header's
  size and field offsets (a C probe compiled against the header prints them);
* dg_default_params fills in the constants of the paper's table, the same
  numbers the reference implementation uses;
* on a host with no GPU, creating a handle fails with an error status and a
  message instead of falling back to anything.
"""
import ctypes as ct
import os
import re
import subprocess
import tempfile

import pytest

import oracle as O
from paper_2305_13847_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


def _declared():
    inc = os.path.join(ROOT, "include")
    text = "\n".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(dg_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_documented_calls():
    names = _declared()
    for core in ("dg_create", "dg_rhs", "dg_saturation_split", "dg_rk_step", "dg_rhs_vjp"):
        assert core in names
    assert len(names) >= 20


def test_every_declared_function_is_exported():
    L = lib.load()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_exactly_the_header():
    assert sorted(lib.EXPORTS) == _declared()


PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "dg.h"
#include "dg_tri.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("dg_mesh %zu\ndg_params %zu\ndg_stats %zu\n", sizeof(dg_mesh), sizeof(dg_params), sizeof(dg_stats));
  F(dg_mesh, dim) F(dg_mesh, n) F(dg_mesh, lo) F(dg_mesh, hi) F(dg_mesh, bc)
  F(dg_params, g) F(dg_params, pref) F(dg_params, rain) F(dg_params, vr_mode) F(dg_params, vr_const)
  F(dg_params, q_au) F(dg_params, precision) F(dg_params, rk) F(dg_params, newton_rtol)
  F(dg_params, newton_maxit) F(dg_params, sponge_zD) F(dg_params, sponge_alpha) F(dg_params, basis) F(dg_params, sip_gamma) F(dg_params, sip_sigma)
  F(dg_stats, splits) F(dg_stats, nonconverged) F(dg_stats, max_iters) F(dg_stats, nonfinite)
  printf("dg_tri_mesh %zu\n", sizeof(dg_tri_mesh));
  F(dg_tri_mesh, ne) F(dg_tri_mesh, xy) F(dg_tri_mesh, nb) F(dg_tri_mesh, nbf) F(dg_tri_mesh, z0)
  F(dg_tri_mesh, dz) F(dg_tri_mesh, nz)
  return 0;
}
"""


def test_struct_layouts_match_the_header():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "probe.cpp"), os.path.join(d, "probe")
        open(src, "w").write(PROBE)
        cmd = ["g++", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
               src, "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("cannot compile the header probe: " + r.stderr[-300:])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    structs = {"dg_mesh": lib.dg_mesh, "dg_params": lib.dg_params, "dg_stats": lib.dg_stats,
               "dg_tri_mesh": lib.dg_tri_mesh}
    for key, val in got.items():
        if "." in key:
            s, f = key.split(".")
            assert getattr(structs[s], f).offset == int(val), key
        else:
            assert ct.sizeof(structs[key]) == int(val), key


def test_default_params_are_the_paper_constants():
    L = lib.load()
    p = lib.dg_params()
    L.dg_default_params(ct.byref(p))
    ref = O.default_params()
    for name, _ in lib.dg_params._fields_:
        if hasattr(ref, name) and name not in ("precision", "rk"):
            assert getattr(p, name) == getattr(ref, name), name
    assert p.precision == lib.DG_FP64 and p.rk == lib.DG_SSPRK43


def test_create_without_a_device_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2305_13847_amd import synth
    c = synth.periodic_smooth(n=(4, 4), order=2, seed=1)
    with pytest.raises(lib.DGError) as e:
        lib.for_case(c, precision=lib.DG_FP64)
    assert "dg status" in str(e.value)


@pytest.mark.parametrize("dim,order", [(3, 5), (2, 8), (2, 0)])
def test_order_range_is_checked_before_the_device(dim, order):
    # orders 1..7 in 2D and 1..4 in 3D; the check runs before any device call
    from paper_2305_13847_amd import synth
    c = synth.periodic_smooth(n=(2,) * dim, order=max(order, 1), dim=dim, seed=1)
    with pytest.raises(lib.DGError) as e:
        lib.DG(c.mesh, order, c.nvars, lib.params_for_case(c, lib.DG_FP64))
    assert e.value.status == lib.DG_EINVAL, str(e.value)


def test_triangle_create_without_a_device_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2305_13847_amd import synth
    c = synth.tri_bubble(n=(4, 2), order=2)
    with pytest.raises(lib.DGError) as e:
        lib.for_tri_case(c)
    assert "dg status" in str(e.value)


@pytest.mark.parametrize("order", [0, 5])
def test_triangle_order_range_is_checked_before_the_device(order):
    from paper_2305_13847_amd import synth
    c = synth.tri_bubble(n=(4, 2), order=2)
    c.mesh.order = order
    with pytest.raises(lib.DGError) as e:
        lib.DGTri(c.mesh, c.nvars, lib.default_params())
    assert e.value.status == lib.DG_EINVAL, str(e.value)


def test_triangle_tables_are_checked_before_the_device():
    from paper_2305_13847_amd import synth
    c = synth.tri_bubble(n=(4, 2), order=2)
    bad = synth.tri_mesh((4, 2), (0.0, 0.0), (20e3, 10e3), (0, 1), 2)
    bad.nbf[0, 1] = (bad.nbf[0, 1] + 1) % 3          # no longer symmetric
    with pytest.raises(lib.DGError) as e:
        lib.DGTri(bad, c.nvars, lib.default_params())
    assert e.value.status == lib.DG_EINVAL and "symmetric" in str(e.value)
    flip = synth.tri_mesh((4, 2), (0.0, 0.0), (20e3, 10e3), (0, 1), 2)
    flip.xy[3] = flip.xy[3][::-1].copy()              # clockwise
    with pytest.raises(lib.DGError) as e:
        lib.DGTri(flip, c.nvars, lib.default_params())
    assert e.value.status == lib.DG_EINVAL and "counter-clockwise" in str(e.value)


def test_triangle_empty_mesh_is_refused_before_the_device():
    from paper_2305_13847_amd import synth
    c = synth.tri_bubble(n=(4, 2), order=2)
    empty = synth.tri_mesh((4, 2), (0.0, 0.0), (20e3, 10e3), (0, 1), 2)
    empty.xy = empty.xy[:0].copy()
    empty.nb = empty.nb[:0].copy()
    empty.nbf = empty.nbf[:0].copy()
    with pytest.raises(lib.DGError) as e:
        lib.DGTri(empty, c.nvars, lib.default_params())
    assert e.value.status == lib.DG_EINVAL
