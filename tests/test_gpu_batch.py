"""Batched ensembles, launch geometry, graph replay and the autotuner.

* an uneven ensemble advanced by one handle equals every member advanced
  alone, bitwise (the per-element arithmetic does not depend on batching);
* results do not depend on the launch geometry (elements per block,
  persistent grid), bitwise;
* hipGraph replays equal eager stepping, replay after replay, with eager
  work and synchronisation between replays;
* the ensemble matches the CPU reference member by member.
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


def _members(n=5, seed=31):
    return synth.ensemble(nmembers=n, order=3, seed=seed, nsteps=4, lo=4, hi=12)


def _pack(cases, dtype):
    return torch.cat([torch.tensor(c.U, dtype=dtype).reshape(c.nvars, -1) for c in cases], dim=1).contiguous().cuda()


def _unpack(U, cases):
    out, off = [], 0
    for c in cases:
        n = c.mesh.ne * c.mesh.npe
        out.append(U[:, off:off + n].reshape(c.U.shape))
        off += n
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_ensemble_equals_members_bitwise(prec):
    lib = _lib()
    cases = _members()
    dt = np.array([c.dt for c in cases])
    dg = lib.for_ensemble(cases, precision=prec)
    dtype = torch.float64 if prec == 0 else torch.float32
    U = _pack(cases, dtype).reshape(dg.shape)
    dg.rk_step(U, dt, 4)
    got = _unpack(U.reshape(cases[0].nvars, -1).cpu().numpy(), cases)
    for m, c in enumerate(cases):
        d1 = lib.for_case(c, precision=prec)
        Um = torch.tensor(c.U, dtype=dtype, device="cuda")
        d1.rk_step(Um, c.dt, 4)
        assert np.array_equal(got[m], Um.cpu().numpy()), m


def test_ensemble_matches_reference():
    lib = _lib()
    cases = _members(3, seed=7)
    dt = np.array([c.dt for c in cases])
    dg = lib.for_ensemble(cases, precision=0)
    U = _pack(cases, torch.float64).reshape(dg.shape)
    dg.rk_step(U, dt, 3)
    got = _unpack(U.reshape(cases[0].nvars, -1).cpu().numpy(), cases)
    for m, c in enumerate(cases):
        ref, _ = O.Oracle.for_case(c).rk(c.U, c.dt, 3)
        W = node_weights(c.mesh)
        floor = 1e-12 * np.sqrt(np.sum(W * ref[-1] ** 2))
        for v in range(c.nvars):
            err = np.sqrt(np.sum(W * (got[m][v] - ref[v]) ** 2)) / max(np.sqrt(np.sum(W * ref[v] ** 2)), floor)
            assert err < 1e-11, (m, v, err)


@pytest.mark.parametrize("prec", [0, 1])
def test_launch_geometry_does_not_change_results(prec):
    lib = _lib()
    c = synth.warm_rain_3d(n=(6, 5, 4), order=3, seed=3)
    dtype = torch.float64 if prec == 0 else torch.float32
    outs = []
    emax = lib.for_case(c, precision=prec).get_launch()[0]      # 4 in FP32, 2 in FP64 (Q3 3D)
    geos = [(emax, 0), (max(1, emax // 2), 0), (1, 0), (emax, 1), (max(1, emax // 2), 2), (1, 4)]
    for epb, persist in geos:
        dg = lib.for_case(c, precision=prec)
        dg.set_launch(epb, persist)
        assert dg.get_launch() == (epb, persist)
        U = torch.tensor(c.U, dtype=dtype, device="cuda")
        dg.rk_step(U, c.dt, 3)
        outs.append(U.cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_graph_replays_match_eager():
    lib = _lib()
    cases = _members(4, seed=11)
    dt = np.array([c.dt for c in cases])
    dg = lib.for_ensemble(cases, precision=1)
    U0 = _pack(cases, torch.float32).reshape(dg.shape)
    Ue = U0.clone()
    Ug = U0.clone()
    for rep in range(3):
        dg.rk_step(Ue, dt, 2)                 # eager
        dg.rk_step_graph(Ug, dt, 2)           # captured on the first call, replayed after
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(Ue.cpu().numpy(), Ug.cpu().numpy()), rep
    assert float(junk) == float(junk)


def test_autotune_picks_a_valid_geometry(tmp_path):
    lib = _lib()
    cases = _members(4, seed=13)
    dt = np.array([c.dt for c in cases])
    dg = lib.for_ensemble(cases, precision=1)
    U = _pack(cases, torch.float32).reshape(dg.shape)
    U0 = U.clone()
    cache = str(tmp_path / "tune.json")
    rec = dg.autotune(U, dt, nsteps=2, cache=cache, key="ens")
    assert torch.equal(U, U0)                # the tuner works on a copy
    assert dg.get_launch() == (rec["elems_per_block"], rec["persist_per_cu"])
    assert 1 <= rec["elems_per_block"] <= 16 and rec["persist_per_cu"] in (0, 1, 2, 4)
    dg2 = lib.for_ensemble(cases, precision=1)
    rec2 = dg2.autotune(U, dt, cache=cache, key="ens")      # from the cache
    assert rec2["elems_per_block"] == rec["elems_per_block"]


@pytest.mark.parametrize("basis,sip", [("lobatto", 0.0), ("gauss", 0.0), ("lobatto", 0.3)])
def test_persistent_grid_covers_every_item(basis, sip):
    # one element per block and one persistent block per CU: with 384
    # elements the grid is smaller than the item count, so every kernel must
    # either walk the items or be launched on the full grid
    lib = _lib()
    c = synth.warm_rain_3d(n=(8, 8, 6), order=3, seed=9, basis=basis)
    print("case", basis, sip, c.digest(), flush=True)
    outs = []
    for persist in (0, 1):
        dg = lib.for_case(c, precision=1, sip_gamma=sip)
        dg.set_launch(1, persist)
        U = torch.tensor(c.U, dtype=torch.float32, device="cuda")
        R = dg.rhs(U).cpu().numpy()
        T = dg.saturation_split(U)[0].cpu().numpy()
        dg.rk_step(U, c.dt, 2)
        outs.append((R, T, U.cpu().numpy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("order3", [2, 3])
def test_item_order_does_not_change_results(order3):
    # the order of the work items (y-bands, plain, wide bands) changes only
    # which elements run together, never the arithmetic
    lib = _lib()
    c = synth.warm_rain_3d(n=(6, 9, 4), order=order3, seed=19)
    outs = []
    for order in (0, 1, 2, 3):
        dg = lib.for_case(c, precision=1)
        dg.set_item_order(order)
        assert dg.get_item_order() == order
        U = torch.tensor(c.U, dtype=torch.float32, device="cuda")
        dg.rk_step(U, c.dt, 2)
        outs.append(U.cpu().numpy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    with pytest.raises(lib.DGError):
        dg.set_item_order(4)
