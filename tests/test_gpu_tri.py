"""GPU parity on triangles (Section 3.1 P^k space, Duffy-mapped rule of the
Section 3.4 footnote, gathered faces) against the reference's triangle
variant, through the C ABI.

The two share no arithmetic: the reference evaluates the basis by forward-mode
differentiation of one recurrence and assembles element by element in FP64;
the library builds its own tables (explicit derivative recurrences, its own
Gauss rule) and runs one thread per element.  Inputs are the reference's
projection of a seeded bubble (with rain: a falling rain blob) onto P^k, fed
to both.

Tolerances: FP64 one right-hand side to 1e-9 and ten SSPRK(4,3) steps to
1e-9 (relative max per variable: the two splits stop at different but
converged iterates, 1e-14 relative in T, and the assembly order differs);
FP32 bulk to 2e-4 for one right-hand side (the fluxes are differences of
terms ~1e5 larger than the tendency of the momentum) and 1e-4 after ten steps.
Sizes span several 64-element blocks and a ragged tail.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_2305_13847_amd import lib
    return lib


def rel_max(a, b):
    return np.array([np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(a.shape[0])])


CASES = {
    # (cells per axis, order, rain, vr_mode, jitter): 2 n0 n1 triangles
    "p1": dict(n=(19, 9), order=1),
    "p2-jitter": dict(n=(15, 7), order=2, jitter=0.15),
    "p3": dict(n=(12, 7), order=3),
    "p3-rain": dict(n=(12, 7), order=3, rain=True),
    "p4-rain-jitter": dict(n=(9, 5), order=4, rain=True, jitter=0.1),
    "p2-rain": dict(n=(16, 8), order=2, rain=True),
}


def _case(name, **extra):
    kw = dict(CASES[name])
    kw.update(extra)
    return synth.tri_bubble(seed=11, noise=1e-4, **kw)


def _pair(c, prec, vr_mode=0):
    lib = _lib()
    o = O.TriOracle.for_case(c, vr_mode=vr_mode)
    C = o.state(c.point_state)
    dg = lib.for_tri_case(c, precision=prec, vr_mode=vr_mode)
    dt = torch.float64 if prec == lib.DG_FP64 else torch.float32
    Cg = torch.tensor(C, dtype=dt, device="cuda").contiguous()
    return o, C, dg, Cg


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 2e-4)])
def test_rhs_matches_reference(name, prec, tol):
    c = _case(name)
    print("case", name, c.name, "prec", prec, flush=True)
    o, C, dg, Cg = _pair(c, prec)
    R = dg.rhs(Cg).double().cpu().numpy()
    ref = o.rhs(C)
    err = rel_max(R, ref)
    print("rel max per variable", err)
    assert np.all(err < tol), err
    assert dg.stats()["status"] == 0


@pytest.mark.parametrize("name", ["p3-rain", "p2-rain"])
def test_rhs_with_the_cosmo_fall_speed(name):
    c = _case(name)
    o, C, dg, Cg = _pair(c, 0, vr_mode=1)
    err = rel_max(dg.rhs(Cg).cpu().numpy(), o.rhs(C))
    print("rel max per variable", err)
    assert np.all(err < 1e-9), err


@pytest.mark.parametrize("name", ["p1", "p3", "p3-rain", "p4-rain-jitter"])
def test_split_matches_reference(name):
    c = _case(name)
    o, C, dg, Cg = _pair(c, 0)
    Tc, Rc = dg.split(Cg)
    Tr, Rr, bad = o.split(C)
    assert bad == 0
    assert np.abs(Tc.cpu().numpy() - Tr).max() < 1e-11 * np.abs(Tr).max()
    assert np.abs(Rc.cpu().numpy() - Rr).max() < 1e-11 * np.abs(Rr).max()


@pytest.mark.parametrize("name", ["p1", "p2-jitter", "p3-rain", "p4-rain-jitter"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-4)])
def test_ten_rk_steps(name, prec, tol):
    c = _case(name)
    o, C, dg, Cg = _pair(c, prec)
    dg.rk_step(Cg, c.dt, 10)
    ref, _ = o.rk(C, c.dt, 10)
    err = rel_max(Cg.double().cpu().numpy(), ref)
    print("rel max per variable", err)
    assert np.all(err < tol), err
    st = dg.stats()
    assert st["status"] == 0 and st["nonconverged"] == 0
    nq = (c.mesh.order + 1) * (c.mesh.order + 2)
    assert st["splits"] == c.mesh.ne * nq * (1 + 4 * 10)


def test_rk33_matches_reference():
    c = _case("p2-rain")
    lib = _lib()
    o = O.TriOracle.for_case(c)
    C = o.state(c.point_state)
    dg = lib.for_tri_case(c, precision=lib.DG_FP64, rk=lib.DG_SSPRK33)
    Cg = torch.tensor(C, device="cuda")
    dg.rk_step(Cg, c.dt, 5)
    ref, _ = o.rk(C, c.dt, 5, scheme=1)
    assert np.all(rel_max(Cg.cpu().numpy(), ref) < 1e-9)


@pytest.mark.parametrize("prec", [0, 1])
def test_projection_matches_reference(prec):
    c = _case("p3-rain")
    lib = _lib()
    o = O.TriOracle.for_case(c)
    dg = lib.for_tri_case(c, precision=prec)
    pts = o.points()
    assert np.allclose(dg.points(), pts, rtol=0, atol=1e-9)
    vals = c.point_state(pts)
    got = dg.project(torch.tensor(vals, device="cuda")).double().cpu().numpy()
    ref = o.project(vals)
    tol = 1e-13 if prec == 0 else 1e-6
    assert np.all(rel_max(got, ref) < tol)


def test_one_partial_block_and_walls_all_round():
    # 2 x 3 cells = 12 triangles (a single, mostly empty block), slip walls on all sides
    lib = _lib()
    mesh = synth.tri_mesh((2, 3), (0.0, 0.0), (3e3, 3e3), (synth.WALL, synth.WALL), 2, jitter=0.1, seed=3)
    c = synth.tri_bubble(n=(2, 3), order=2, noise=1e-4)
    c.mesh = mesh
    o = O.TriOracle.for_case(c)
    C = o.state(c.point_state)
    dg = lib.for_tri_case(c, precision=lib.DG_FP64)
    Cg = torch.tensor(C, device="cuda")
    assert np.all(rel_max(dg.rhs(Cg).cpu().numpy(), o.rhs(C)) < 1e-9)
    dg.rk_step(Cg, c.dt, 3)
    ref, _ = o.rk(C, c.dt, 3)
    assert np.all(rel_max(Cg.cpu().numpy(), ref) < 1e-9)


def test_benchmark_size_rhs_and_step():
    # the benchmarked workload's shape: 512 x 256 cells, P3, FP32 bulk; one
    # right-hand side in full and one step on every element
    lib = _lib()
    c = synth.tri_bubble(n=(512, 256), order=3, noise=1e-4)
    print("case", c.name, flush=True)
    o = O.TriOracle.for_case(c)
    C = o.state(c.point_state)
    dg = lib.for_tri_case(c, precision=lib.DG_FP32_BULK)
    Cg = torch.tensor(C, dtype=torch.float32, device="cuda")
    err = rel_max(dg.rhs(Cg).double().cpu().numpy(), o.rhs(C))
    print("rhs rel max per variable", err)
    assert np.all(err < 2e-4), err
    dg.rk_step(Cg, c.dt, 1)
    ref, _ = o.rk(C, c.dt, 1)
    err = rel_max(Cg.double().cpu().numpy(), ref)
    print("step rel max per variable", err)
    assert np.all(err < 1e-4), err
    assert dg.stats()["status"] == 0


def test_rhs_rejects_aliasing():
    lib = _lib()
    c = _case("p1")
    o, C, dg, Cg = _pair(c, 0)
    with pytest.raises(lib.DGError):
        dg.rhs(Cg, out=Cg)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_dry_mass_is_conserved_at_benchmark_size(prec, tol):
    # periodic in x, slip walls in z: the dry mass sum_e det A_e c_0 / sqrt(2)
    # (the mean mode of the orthonormal basis) is conserved by every step
    lib = _lib()
    c = synth.tri_bubble(n=(512, 256), order=3, noise=1e-4)
    dg = lib.for_tri_case(c, precision=prec)
    C = dg.state(c.point_state)
    xy = c.mesh.xy
    det = torch.tensor((xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1])
                       - (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1]), device="cuda")

    def masses(X):
        return [float(torch.sum(det * X[v, :, 0].double())) / np.sqrt(2.0) for v in (0, 1)]
    # relative to the summed magnitude of the perturbation's element masses
    scale = [float(torch.sum(torch.abs(det * C[v, :, 0].double()))) / np.sqrt(2.0) for v in (0, 1)]
    m0 = masses(C)
    dg.rk_step(C, c.dt, 5)
    m1 = masses(C)
    print("mass before/after", m0, m1, "scale", scale)
    assert all(abs(a - b) < tol * sc for a, b, sc in zip(m0, m1, scale)), (m0, m1, scale)
    assert dg.stats()["status"] == 0
