"""dg_rhs_noalloc, the right-hand side whose split scratch lives in the
library's static device array, against dg_rhs on the same handle and input.

Both run the same kernels on the same state, so the results agree bit for bit
(the parity bar of integer work applies here, tighter than the FP tolerance).
Two calls in a row, the second on a smaller handle, show that the shared
array carries nothing from one call to the next; a handle larger than the
array is refused before anything runs.
"""
import numpy as np
import pytest

from paper_2305_13847_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_2305_13847_amd import lib
    return lib


def _check_against_rhs(case, prec):
    lib = _lib()
    print("case", case.name, "precision", prec, flush=True)
    dg = lib.for_case(case, precision=prec)
    dt = torch.float64 if prec == lib.DG_FP64 else torch.float32
    U = torch.tensor(case.U, dtype=dt, device="cuda").contiguous()
    out = torch.full_like(U, float("nan"))
    dg.rhs_noalloc(U, out)
    ref = dg.rhs(U)
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    assert np.isfinite(a).all()
    assert np.array_equal(a, b)
    assert dg.stats()["status"] == 0
    dg.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_rhs_equals_rhs_twice_then_smaller(prec):
    big = synth.warm_rain_3d(n=(8, 6, 5), order=3, seed=41)        # 15,360 nodes
    small = synth.moist_bubble(n=(6, 4), order=2, seed=42)         # 216 nodes
    _check_against_rhs(big, prec)
    _check_against_rhs(small, prec)


def test_noalloc_rhs_refuses_what_it_cannot_hold():
    lib = _lib()
    c = synth.warm_rain_3d(n=(8, 6, 5), order=3, seed=43)
    mesh = synth.Mesh(3, [34, 32, 32], c.mesh.lo, c.mesh.hi, c.mesh.bc, 3)   # 2,228,224 nodes > 2^21
    bg = synth.background(mesh, 300.0, lambda z: 0.8 + 0.0 * z)
    dg = lib.DG(mesh, 3, 7, lib.default_params(rain=1, precision=lib.DG_FP32_BULK))
    dg.set_background(0, bg["rho_d"], bg["rho_m"], bg["rho_r"], bg["E"])
    U = torch.zeros(dg.shape, dtype=torch.float32, device="cuda")
    out = torch.empty_like(U)
    with pytest.raises(lib.DGError) as ei:
        dg.rhs_noalloc(U, out)
    assert ei.value.status == lib.DG_EINVAL and "at most" in str(ei.value)
    dg.close()
    # and the Gauss basis is not covered
    g = synth.moist_bubble(n=(6, 4), order=2, seed=44, basis="gauss")
    dg = lib.for_case(g, precision=lib.DG_FP64)
    Ug = torch.tensor(g.U, device="cuda")
    with pytest.raises(lib.DGError) as ei:
        dg.rhs_noalloc(Ug, torch.empty_like(Ug))
    assert ei.value.status == lib.DG_EUNSUPPORTED
