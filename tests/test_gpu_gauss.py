"""GPU parity of the Gauss basis (the paper's Legendre modes with Gauss
quadrature, held by values at the Gauss points) against the reference's modal
variant, through the C ABI.

The two share no arithmetic: the reference projects onto Legendre modes,
evaluates every face trace from the modes, and lifts by the modes; the GPU
interpolates along the normal lines and lifts to the nodes of each line.
Tolerances as for the Lobatto basis: one right-hand side to 1e-11 in FP64 and
1e-4 in FP32 bulk (relative max per variable); ten SSPRK(4,3) steps to 1e-11
(FP64) and 1e-4 (FP32), relative L2 with the quadrature weights of the Gauss
nodes.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth
from exact import node_weights

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_2305_13847_amd import lib
    return lib


def rel_l2(mesh, a, b, floor=1e-300):
    W = node_weights(mesh)
    return np.array([np.sqrt(np.sum(W * (a[v] - b[v]) ** 2)) / max(np.sqrt(np.sum(W * b[v] ** 2)), floor)
                     for v in range(a.shape[0])])


def rel_max(a, b):
    return np.array([np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(a.shape[0])])


G = "gauss"
CASES = {
    "periodic2d_q2": lambda: synth.periodic_smooth(n=(16, 16), order=2, basis=G),
    "periodic3d_q2": lambda: synth.periodic_smooth(n=(5, 4, 3), order=2, dim=3, basis=G),
    "bubble2d_q1": lambda: synth.moist_bubble(n=(20, 9), order=1, seed=16, basis=G),
    "bubble2d_q3": lambda: synth.moist_bubble(n=(13, 7), order=3, seed=13, basis=G),
    "bubble2d_q4": lambda: synth.moist_bubble(n=(12, 6), order=4, seed=12, basis=G),
    "rain3d_q2": lambda: synth.warm_rain_3d(n=(5, 4, 3), order=2, seed=15, basis=G),
    "rain3d_q3": lambda: synth.warm_rain_3d(n=(4, 4, 3), order=3, seed=14, basis=G),
    "rain3d_q1": lambda: synth.warm_rain_3d(n=(6, 5, 4), order=1, seed=17, basis=G),
    "rain3d_q4": lambda: synth.warm_rain_3d(n=(3, 3, 3), order=4, seed=18, basis=G),
}


def _gpu(case, prec, **over):
    lib = _lib()
    dg = lib.for_case(case, precision=prec, **over)
    dt = torch.float64 if prec == lib.DG_FP64 else torch.float32
    U = torch.tensor(case.U, dtype=dt, device="cuda").contiguous()
    return dg, U


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_parity_fp64(name):
    c = CASES[name]()
    print("case", name, c.digest(), flush=True)
    lib = _lib()
    dg, U = _gpu(c, lib.DG_FP64)
    R = dg.rhs(U)
    torch.cuda.synchronize()
    ref = O.Oracle.for_case(c).rhs(c.U)
    err = rel_max(R.cpu().numpy().reshape(c.U.shape), ref)
    print("rel max per variable", err)
    assert np.all(err < 1e-11), err


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_parity_fp32(name):
    c = CASES[name]()
    print("case", name, c.digest(), flush=True)
    lib = _lib()
    dg, U = _gpu(c, lib.DG_FP32_BULK)
    R = dg.rhs(U)
    torch.cuda.synchronize()
    ref = O.Oracle.for_case(c).rhs(U.double().cpu().numpy().reshape(c.U.shape))
    err = rel_max(R.double().cpu().numpy().reshape(c.U.shape), ref)
    print("rel max per variable", err)
    assert np.all(err < 1e-4), err


@pytest.mark.parametrize("name", ["periodic2d_q2", "periodic3d_q2", "bubble2d_q4", "rain3d_q3", "bubble2d_q1"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-4)])
def test_ten_rk_steps(name, prec, tol):
    c = CASES[name]()
    print("case", name, prec, c.digest(), flush=True)
    dg, U = _gpu(c, prec)
    dg.rk_step(U, c.dt, 10)
    torch.cuda.synchronize()
    assert dg.stats()["status"] == 0
    ref, _ = O.Oracle.for_case(c).rk(c.U, c.dt, 10)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
    err = rel_l2(c.mesh, U.double().cpu().numpy().reshape(c.U.shape), ref, floor=floor)
    print("rel L2 per variable", err)
    assert np.all(err < tol), err


@pytest.mark.parametrize("k", [2, 3])
def test_hydrostatic_rest_state_is_steady(k):
    c = synth.moist_bubble(n=(8, 6), order=k, noise=0.0, amp=0.0, basis=G)
    lib = _lib()
    dg, U = _gpu(c, lib.DG_FP64)
    R = dg.rhs(torch.zeros_like(U)).cpu().numpy()
    assert np.abs(R).max() < 1e-12 * 9.81 * c.bg["rho_d"].max(), np.abs(R).max()


def test_sponge_steps():
    c = CASES["rain3d_q2"]()
    lib = _lib()
    dg, U = _gpu(c, lib.DG_FP64, sponge_zD=5.0e3, sponge_alpha=0.5)
    dg.rk_step(U, c.dt, 5)
    ref, _ = O.Oracle.for_case(c, sponge_zD=5.0e3, sponge_alpha=0.5).rk(c.U, c.dt, 5)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
    err = rel_l2(c.mesh, U.cpu().numpy().reshape(c.U.shape), ref, floor=floor)
    assert np.all(err < 1e-11), err


@pytest.mark.parametrize("vr_mode", [0, 1])
def test_masses_and_unsupported_calls(vr_mode):
    # dry mass, total water and the rain outflow through the walls at the
    # Gauss points of the floor and lid faces, against the reference's modal
    # form (its outflow is the Lax-Friedrichs flux of rho_r at the walls)
    c = CASES["rain3d_q2"]()
    lib = _lib()
    dg, U = _gpu(c, lib.DG_FP64, vr_mode=vr_mode)
    m = dg.reduce_mass(U)
    ref = O.Oracle.for_case(c, vr_mode=vr_mode).mass(c.U)
    assert m[0] == pytest.approx(ref[0], rel=1e-12, abs=1e-9 * abs(ref[1]))
    assert m[1] == pytest.approx(ref[1], rel=1e-12)
    assert m[2] != 0.0 and m[2] == pytest.approx(ref[2], rel=1e-10)
    with pytest.raises(lib.DGError) as ei:
        dg.rhs_vjp(U, torch.ones_like(U))
    assert ei.value.status == lib.DG_EUNSUPPORTED


def test_launch_shapes_and_graph_agree():
    # every launch geometry and the captured graph give the same bits
    c = CASES["bubble2d_q3"]()
    lib = _lib()
    outs = []
    for epb, persist, graph in [(None, 0, False), (4, 0, False), (8, 1, False), (None, 0, True)]:
        dg, U = _gpu(c, lib.DG_FP32_BULK)
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


def test_batch_members_match_single_runs():
    cases = [synth.moist_bubble(n=(10, 5), order=3, seed=21, basis=G),
             synth.moist_bubble(n=(14, 7), order=3, seed=22, amp=1.0, basis=G)]
    lib = _lib()
    dg = lib.for_ensemble(cases, precision=lib.DG_FP64)
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
        ref, _ = O.Oracle.for_case(c).rk(c.U, c.dt, 4)
        floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
        err = rel_l2(c.mesh, got, ref, floor=floor)
        assert np.all(err < 1e-11), err


def test_mixed_calls_on_one_handle():
    # steps with an odd count, then dg_rhs, then more steps: every call starts
    # from traces of its own input state, whatever buffer the last stage left
    c = CASES["bubble2d_q3"]()
    lib = _lib()
    dg, U = _gpu(c, lib.DG_FP64)
    o = O.Oracle.for_case(c)
    dg.rk_step(U, c.dt, 3)
    ref3, _ = o.rk(c.U, c.dt, 3)
    R = dg.rhs(U).cpu().numpy().reshape(c.U.shape)
    err = rel_max(R, o.rhs(ref3))
    assert np.all(err < 1e-10), err
    dg.rk_step(U, c.dt, 2)
    ref5, _ = o.rk(ref3, c.dt, 2)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref5[-1] ** 2))
    err = rel_l2(c.mesh, U.cpu().numpy().reshape(c.U.shape), ref5, floor=floor)
    assert np.all(err < 1e-11), err


def test_state_above_64_mib_with_the_reversed_walk():
    # a state of more than 64 MiB: every other stage walks its work items in
    # reverse (each XCD its own range, top down); one SSPRK(4,3) step in FP64
    # against the reference
    c = synth.warm_rain_3d(n=(32, 32, 22), order=3, basis=G)
    assert c.U.nbytes > 64 * 2 ** 20
    print("case", c.name, c.digest(), flush=True)
    dg, U = _gpu(c, 0)
    dg.rk_step(U, c.dt, 1)
    torch.cuda.synchronize()
    assert dg.stats()["status"] == 0
    ref, _ = O.Oracle.for_case(c).rk(c.U, c.dt, 1)
    floor = 1e-12 * np.sqrt(np.sum(node_weights(c.mesh) * ref[-1] ** 2))
    err = rel_l2(c.mesh, U.double().cpu().numpy().reshape(c.U.shape), ref, floor=floor)
    print("rel L2 per variable", err)
    assert np.all(err < 1e-11), err
