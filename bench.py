#!/usr/bin/env python3
"""Throughput of the moist DG hot path on one MI355X.

A step is one SSPRK(4,3) step (four stages: split, right-hand side and stage
update) of the 3D warm-rain workload: 64 x 64 x 32 hexahedra, Q3, seven
variables, Kessler rain falling at 5 m/s, FP32 bulk arithmetic with the FP64
split.  The metric is DoF-stage updates per second (variables x nodes x
stages / wall time) with the state resident in HBM.

Also reported on the same line: the roofline of the dominant kernel (the fused
stage kernel: algorithmic bytes per launch / its HIP-event-timed duration
against 8 TB/s), the FP64 run of the same workload, the same FP32 workload
with the Rayleigh sponge layer on, with the artificial diffusion on, and in
the paper's Legendre/Gauss basis (FP32 and FP64), the 2D moist bubble
(128 x 64, Q4) in FP64 and FP32, the batched ensemble, and the FP64 CPU
reference timed on a bounded sample of the 3D workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


# the sources the FP32 fused stage kernel is compiled from
STAGE_SOURCES = ("dg_common.h", "dg_device.h", "dg_kernels.h", "dg_f32.hip")


def csrc_hash() -> str:
    """Hash of the stage kernel's sources: a committed traffic figure is used
    only while it matches."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2305_13847_amd", "csrc")
    for f in STAGE_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprof counter runs, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("csrc_hash") != csrc_hash():
        return None
    return ent.get("bytes_per_launch")


def time_workload(case, precision, steps, warmup, lib, torch, kernel_timing=True, **over):
    dg = lib.for_case(case, precision=precision, **over)
    dt = torch.float64 if precision == lib.DG_FP64 else torch.float32
    U = torch.tensor(case.U, dtype=dt, device="cuda").contiguous()
    dofs = case.U.size
    if warmup:
        dg.rk_step(U, case.dt, warmup)
    torch.cuda.synchronize()
    if kernel_timing:
        dg.timing(True)
    t0 = time.perf_counter()
    dg.rk_step(U, case.dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = dict(seconds=el, dofs=dofs, steps=steps,
               dof_stage_per_s=dofs * 4 * steps / el,
               ms_per_step=1e3 * el / steps)
    if kernel_timing:
        for name, k in (("stage", lib.DG_K_STAGE), ("split", lib.DG_K_SPLIT), ("other", lib.DG_K_OTHER)):
            ms, n = dg.timing_read(k)
            out[name + "_us"] = 1e3 * ms / max(n, 1)
            out[name + "_launches"] = n
        dg.timing(False)
    st = dg.stats()
    out["newton_max_iters"] = st["max_iters"]
    out["status"] = st["status"]
    dg.close()
    return out


def time_ensemble(steps, lib, torch, synth):
    """64 uneven 2D bubbles (Q3, 5 vars) in one handle, FP32 bulk, hipGraph replay, autotuned."""
    cases = synth.ensemble(nmembers=64, order=3, nsteps=steps)
    dts = np.array([c.dt for c in cases])
    dg = lib.for_ensemble(cases, precision=lib.DG_FP32_BULK)
    U = torch.cat([torch.tensor(c.U, dtype=torch.float32).reshape(c.nvars, -1) for c in cases],
                  dim=1).contiguous().cuda().reshape(dg.shape)
    dofs = sum(c.U.size for c in cases)
    tune = dg.autotune(U, dts, nsteps=2)
    dg.rk_step_graph(U, dts, steps)          # capture + first replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dg.rk_step_graph(U, dts, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    dg.rk_step(U, dts, steps)                # eager, for comparison
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    st = dg.stats()
    dg.close()
    return {"dof_stage_per_s": dofs * 4 * steps / el, "ms_per_step": 1e3 * el / steps,
            "eager_ms_per_step": 1e3 * el_eager / steps, "members": len(cases), "dofs": dofs,
            "elements": sum(c.mesh.ne for c in cases), "launch": tune, "status": st["status"]}


def cpu_baseline(synth, oracle_mod):
    """FP64 reference, two RK steps on a 32 x 32 x 32 column sample of the 3D case."""
    import multiprocessing
    c = synth.warm_rain_3d(n=(32, 32, 32))
    o = oracle_mod.Oracle.for_case(c)
    t0 = time.perf_counter()
    o.rk(c.U, c.dt, 2)
    el = time.perf_counter() - t0
    return {"value": c.U.size * 8 / el, "unit": "DoF-stage updates/s", "cores": 1, "kind": "oracle",
            "sample": "two SSPRK(4,3) steps of the 3D warm-rain case on a 32x32x32-element column "
                      "sample (Q3, 7 vars, %d DoFs, same vertical structure and physics), single "
                      "thread, %.1f s; host has %d cores" % (c.U.size, el, multiprocessing.cpu_count())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--copy-only", type=int, default=0, metavar="MIB",
                    help="only copy a device buffer of this size (traffic-counter calibration)")
    args = ap.parse_args()
    if args.copy_only:
        import torch
        a = torch.ones(args.copy_only * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_only, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the single-GPU kernel is the product here; "
              "multi-GPU runs are not part of this build (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_13847_amd import lib, synth
    lib.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)

    case = synth.warm_rain_3d()
    res = time_workload(case, lib.DG_FP32_BULK, args.steps, args.warmup, lib, torch)
    s_bytes = 4
    nvars, nodes = case.nvars, case.U.size // case.nvars
    # algorithmic bytes of one fused stage launch: SSPRK(4,3) moves 9 state
    # passes over 4 stages (read U_s, write U_{s+1}, plus U_n once)
    alg_stage = 2.25 * s_bytes * nvars * nodes
    achieved = alg_stage / (res["stage_us"] * 1e-6) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_for("stage", "rain-3d-q3-64x64x32-fp32"),
            "kernel": "rhs_kernel<float,3,3,rain,stage>", "kernel_us": res["stage_us"],
            "alg_bytes_per_launch": alg_stage,
            # the stand-alone split runs once per dg_rk_step call (the fused stage
            # kernels split every later stage state); the step-level fraction
            # counts everything between the synchronisations
            "call_split_kernel_us": res["split_us"],
            "step_level_frac": 4 * alg_stage / (res["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}

    extra = {}
    if not args.no_extra:
        r64 = time_workload(case, lib.DG_FP64, max(2, args.steps // 4), 1, lib, torch)
        extra["rain3d_fp64"] = {k: r64[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us", "split_us")}
        # the same FP32 workload with the Rayleigh sponge above 7 km, fused into
        # the last stage of every step
        rsp = time_workload(case, lib.DG_FP32_BULK, args.steps, args.warmup, lib, torch,
                            sponge_zD=7.0e3, sponge_alpha=0.5)
        extra["rain3d_fp32_sponge"] = {k: rsp[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us")}
        # the same FP32 workload with the artificial diffusion (gamma 0.6, the
        # paper's 3D value); its three kernels per stage are the "other" class
        rsi = time_workload(case, lib.DG_FP32_BULK, args.steps, args.warmup, lib, torch, sip_gamma=0.6)
        extra["rain3d_fp32_sip"] = {k: rsi[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us")}
        extra["rain3d_fp32_sip"]["sip_us_per_stage"] = rsi["other_us"]
        del case
        # the paper's own basis: Legendre modes with Gauss quadrature
        case_g = synth.warm_rain_3d(basis="gauss")
        for prec, nm, st in ((lib.DG_FP32_BULK, "rain3d_fp32_gauss", args.steps),
                             (lib.DG_FP64, "rain3d_fp64_gauss", max(2, args.steps // 4))):
            rg = time_workload(case_g, prec, st, 1, lib, torch)
            sb = 4 if prec == lib.DG_FP32_BULK else 8
            extra[nm] = {k: rg[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us")}
            extra[nm]["roofline_frac"] = 2.25 * sb * nvars * nodes / (rg["stage_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
        del case_g
        bub = synth.moist_bubble()
        for prec, nm in ((lib.DG_FP64, "bubble2d_q4_fp64"), (lib.DG_FP32_BULK, "bubble2d_q4_fp32")):
            r = time_workload(bub, prec, 50, 5, lib, torch)
            extra[nm] = {k: r[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us", "split_us")}
        extra["ensemble64_q3_fp32_graph"] = time_ensemble(20, lib, torch, synth)
    cpu = None
    if not args.no_cpu:
        import oracle as oracle_mod
        cpu = cpu_baseline(synth, oracle_mod)

    line = {
        "metric": "DG DoF-stage updates/s (FP64 plain vs FP32/batched) + % of HBM roofline",
        "value": res["dof_stage_per_s"],
        "unit": "DoF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 split)",
        "data": "synthetic",
        "config": {"workload": "3D warm rain, 64x64x32 hexahedra, Q3, 7 variables, Kessler rain "
                               "v_r = 5 m/s, SSPRK(4,3), FP32 bulk + FP64 split",
                   "dofs": res["dofs"], "stages_per_step": 4, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
        "newton_max_iters": res["newton_max_iters"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
