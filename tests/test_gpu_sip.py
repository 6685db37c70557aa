"""GPU parity of the artificial diffusion (Section 3.5; symmetric interior
penalty on the Lobatto basis) against the reference, through the C ABI.

The states carry a mean wind (10 m/s on the cases with gravity), so the
viscosity is of the size the paper's rain runs use (gamma 0.3 here).
- The diffusive tendency alone, dg_rhs with and without it, against the
  reference's: 1e-10 relative (FP64).
- One right-hand side: 1e-11 (FP64) and 1e-4 (FP32 bulk), relative max per
  variable.
- Ten SSPRK(4,3) steps: 1e-11 (FP64) and 1e-4 (FP32), relative L2.
- Launch shapes and the captured graph give the same bits. The adjoint
  calls and the Gauss basis refuse the diffusion.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth
from exact import node_weights

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GAM = 0.3


def _lib():
    from paper_2305_13847_amd import lib
    return lib


def rel_l2(mesh, a, b, floor=1e-300):
    W = node_weights(mesh)
    return np.array([np.sqrt(np.sum(W * (a[v] - b[v]) ** 2)) / max(np.sqrt(np.sum(W * b[v] ** 2)), floor)
                     for v in range(a.shape[0])])


def rel_max(a, b):
    return np.array([np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(a.shape[0])])


def _windy(c, u=10.0):
    if c.g == 0.0:
        return c
    rho = (c.bg["rho_d"] + c.bg["rho_m"] + c.bg["rho_r"])[synth.height_index(c.mesh)]
    c.U[2 + c.rain] += u * rho
    return c


CASES = {
    "periodic2d_q2": lambda: synth.periodic_smooth(n=(16, 16), order=2),
    "bubble2d_q1": lambda: _windy(synth.moist_bubble(n=(20, 9), order=1, seed=16)),
    "bubble2d_q3": lambda: _windy(synth.moist_bubble(n=(13, 7), order=3, seed=13)),
    "bubble2d_q4": lambda: _windy(synth.moist_bubble(n=(12, 6), order=4, seed=12)),
    "rain3d_q2": lambda: _windy(synth.warm_rain_3d(n=(5, 4, 3), order=2, seed=15)),
    "rain3d_q3": lambda: _windy(synth.warm_rain_3d(n=(4, 4, 3), order=3, seed=14)),
    "rain3d_q1": lambda: _windy(synth.warm_rain_3d(n=(6, 5, 4), order=1, seed=17)),
    "rain3d_q4": lambda: _windy(synth.warm_rain_3d(n=(3, 3, 3), order=4, seed=18)),
}


def _gpu(case, prec, **over):
    lib = _lib()
    dg = lib.for_case(case, precision=prec, **over)
    dt = torch.float64 if prec == lib.DG_FP64 else torch.float32
    U = torch.tensor(case.U, dtype=dt, device="cuda").contiguous()
    return dg, U


@pytest.mark.parametrize("name", list(CASES))
def test_diffusive_tendency_alone(name):
    c = CASES[name]()
    print("case", name, c.digest(), flush=True)
    lib = _lib()
    on, U = _gpu(c, lib.DG_FP64, sip_gamma=GAM)
    off, _ = _gpu(c, lib.DG_FP64)
    S = (on.rhs(U) - off.rhs(U)).cpu().numpy().reshape(c.U.shape)
    ref = O.Oracle.for_case(c, sip_gamma=GAM).sip(c.U)
    err = rel_max(S, ref)
    print("rel max per variable", err)
    assert np.all(err < 1e-10), err


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-4)])
def test_rhs_parity(name, prec, tol):
    c = CASES[name]()
    print("case", name, prec, c.digest(), flush=True)
    dg, U = _gpu(c, prec, sip_gamma=GAM)
    R = dg.rhs(U)
    torch.cuda.synchronize()
    ref = O.Oracle.for_case(c, sip_gamma=GAM).rhs(U.double().cpu().numpy().reshape(c.U.shape))
    err = rel_max(R.double().cpu().numpy().reshape(c.U.shape), ref)
    print("rel max per variable", err)
    assert np.all(err < tol), err


@pytest.mark.parametrize("name", ["bubble2d_q1", "bubble2d_q4", "rain3d_q3"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-4)])
def test_ten_rk_steps(name, prec, tol):
    c = CASES[name]()
    print("case", name, prec, c.digest(), flush=True)
    dg, U = _gpu(c, prec, sip_gamma=GAM)
    dg.rk_step(U, c.dt, 10)
    torch.cuda.synchronize()
    assert dg.stats()["status"] == 0
    ref, _ = O.Oracle.for_case(c, sip_gamma=GAM).rk(c.U, c.dt, 10)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
    err = rel_l2(c.mesh, U.double().cpu().numpy().reshape(c.U.shape), ref, floor=floor)
    print("rel L2 per variable", err)
    assert np.all(err < tol), err


def test_launch_shapes_and_graph_agree():
    c = CASES["bubble2d_q3"]()
    lib = _lib()
    outs = []
    for epb, persist, graph in [(None, 0, False), (4, 0, False), (8, 1, False), (None, 0, True)]:
        dg, U = _gpu(c, lib.DG_FP32_BULK, sip_gamma=GAM)
        if epb is not None:
            dg.set_launch(epb, persist)
        if graph:
            dg.rk_step_graph(U, c.dt, 3)
        else:
            dg.rk_step(U, c.dt, 3)
        torch.cuda.synchronize()
        outs.append(U.cpu().numpy())
        dg.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_refused_combinations():
    lib = _lib()
    c = CASES["bubble2d_q3"]()
    dg, U = _gpu(c, lib.DG_FP64, sip_gamma=GAM)
    with pytest.raises(lib.DGError) as ei:
        dg.rhs_vjp(U, torch.ones_like(U))
    assert ei.value.status == lib.DG_EUNSUPPORTED
    g = synth.moist_bubble(n=(6, 4), order=2, basis="gauss")
    with pytest.raises(lib.DGError) as ei:
        lib.for_case(g, precision=lib.DG_FP64, sip_gamma=GAM)
    assert ei.value.status == lib.DG_EUNSUPPORTED


def test_batch_members_match_single_runs():
    # two members of different size: per-member vertex tables and offsets
    cases = [_windy(synth.moist_bubble(n=(10, 5), order=3, seed=21)),
             _windy(synth.moist_bubble(n=(14, 7), order=3, seed=22, amp=1.0), u=6.0)]
    lib = _lib()
    dg = lib.for_ensemble(cases, precision=lib.DG_FP64, sip_gamma=GAM)
    U = torch.cat([torch.tensor(c.U).reshape(c.nvars, -1) for c in cases], dim=1).contiguous().cuda()
    U = U.reshape(dg.shape)
    dts = np.array([c.dt for c in cases])
    dg.rk_step(U, dts, 4)
    Uh = U.cpu().numpy().reshape(5, -1)
    off = 0
    for c in cases:
        n = c.mesh.ne * c.mesh.npe
        got = Uh[:, off:off + n].reshape(c.U.shape)
        off += n
        ref, _ = O.Oracle.for_case(c, sip_gamma=GAM).rk(c.U, c.dt, 4)
        floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
        err = rel_l2(c.mesh, got, ref, floor=floor)
        assert np.all(err < 1e-11), err


@pytest.mark.parametrize("name", ["rain3d_q2", "rain3d_q3"])
@pytest.mark.parametrize("scheme", [0, 1])
def test_with_sponge_and_both_schemes(name, scheme):
    # the last stage of every step carries both flags (diffusion, sponge); on
    # Q3 hexahedra every stage also forms alpha_K of the (sponged) state it
    # writes for the next stage
    c = CASES[name]()
    print("case", name, scheme, c.digest(), flush=True)
    lib = _lib()
    over = dict(sip_gamma=GAM, sponge_zD=5.0e3, sponge_alpha=0.5)
    dg, U = _gpu(c, lib.DG_FP64, rk=lib.DG_SSPRK43 if scheme == 0 else lib.DG_SSPRK33, **over)
    dg.rk_step(U, c.dt, 5)
    ref, _ = O.Oracle.for_case(c, **over).rk(c.U, c.dt, 5, scheme=scheme)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
    err = rel_l2(c.mesh, U.cpu().numpy().reshape(c.U.shape), ref, floor=floor)
    assert np.all(err < 1e-11), err


def test_batch_of_q3_hexahedra_matches_the_reference():
    # members of different size: the stage kernel writes alpha_K per member
    # offset, and the tendency kernel averages it at each member's vertices
    cases = [_windy(synth.warm_rain_3d(n=(4, 3, 3), order=3, seed=31)),
             _windy(synth.warm_rain_3d(n=(5, 4, 2), order=3, seed=32), u=6.0)]
    lib = _lib()
    dg = lib.for_ensemble(cases, precision=lib.DG_FP64, sip_gamma=GAM)
    U = torch.cat([torch.tensor(c.U).reshape(c.nvars, -1) for c in cases], dim=1).contiguous().cuda()
    U = U.reshape(dg.shape)
    dts = np.array([c.dt for c in cases])
    dg.rk_step(U, dts, 4)
    Uh = U.cpu().numpy().reshape(cases[0].nvars, -1)
    off = 0
    for c in cases:
        n = c.mesh.ne * c.mesh.npe
        got = Uh[:, off:off + n].reshape(c.U.shape)
        off += n
        ref, _ = O.Oracle.for_case(c, sip_gamma=GAM).rk(c.U, c.dt, 4)
        floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
        err = rel_l2(c.mesh, got, ref, floor=floor)
        assert np.all(err < 1e-11), err


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-4)])
def test_rain3d_16x16x8_ten_steps(prec, tol):
    # the benchmarked diffusion workload's shape (3D warm rain, Q3, walls at
    # top and bottom) at a size that spans many work items
    c = _windy(synth.warm_rain_3d(n=(16, 16, 8), order=3, seed=33))
    print("case rain3d 16x16x8", prec, c.digest(), flush=True)
    dg, U = _gpu(c, prec, sip_gamma=GAM)
    dg.rk_step(U, c.dt, 10)
    torch.cuda.synchronize()
    assert dg.stats()["status"] == 0
    ref, _ = O.Oracle.for_case(c, sip_gamma=GAM).rk(c.U, c.dt, 10)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
    err = rel_l2(c.mesh, U.double().cpu().numpy().reshape(c.U.shape), ref, floor=floor)
    print("rel L2 per variable", err)
    assert np.all(err < tol), err


def test_q3_launch_shapes_and_graph_agree():
    # the Q3 hexahedral stage kernel forms alpha_K of the state it writes:
    # other block widths and a captured graph give the same bits
    c = CASES["rain3d_q3"]()
    lib = _lib()
    outs = []
    for epb, graph in [(None, False), (2, False), (1, False), (None, True)]:
        dg, U = _gpu(c, lib.DG_FP32_BULK, sip_gamma=GAM)
        if epb is not None:
            dg.set_launch(epb, 0)
        if graph:
            dg.rk_step_graph(U, c.dt, 3)
        else:
            dg.rk_step(U, c.dt, 3)
        torch.cuda.synchronize()
        outs.append(U.cpu().numpy())
        dg.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
