#!/usr/bin/env python3
"""Throughput of the moist DG hot path on one MI355X.

A step is one SSPRK(4,3) step (four stages: split, right-hand side and stage
update) of the 3D warm-rain workload: 64 x 64 x 32 hexahedra, Q3, seven
variables, Kessler rain falling at 5 m/s, FP32 bulk arithmetic with the FP64
split.  The metric is DoF-stage updates per second (variables x nodes x
stages / wall time) with the state resident in HBM.

Timing: W untimed warm-up steps, then R replays of exactly K steps, each
bracketed by device synchronisations, with no instrumentation inside; the
headline is the median replay.  Per-kernel durations come from a separate
pass with the library's HIP-event kernel timing switched on.

Also reported on the same line: the roofline of the dominant kernel (the fused
stage kernel: algorithmic bytes per launch / its HIP-event-timed duration
against 8 TB/s) for FP32 bulk and for FP64 (the paper's precision), the same
FP32 workload with the Rayleigh sponge, with the artificial diffusion, and in
the paper's Legendre/Gauss basis (FP32 and FP64), the 2D moist bubble
(128 x 64, Q4) in FP64 and FP32, the batched 64-member ensemble, the bubble on
a triangulation (512 x 256 cells, two P3 triangles each), and the FP64
CPU reference (two steps of the full 3D workload on all cores, one step of a
column sample on one thread), with the per-field error of the GPU's FP32 bulk
and FP64 runs against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the warm start of the split: one FP64 temperature per node read and written
# (the stored pair (T, rho_vs(T)) moves twice this)
WARM_START_BYTES_PER_NODE = 16

# the sources the fused stage kernels are compiled from (both precisions)
STAGE_SOURCES = ("dg_common.h", "dg_device.h", "dg_kernels.h", "dg_q3.h", "dg_f32.hip", "dg_f64.hip",
                 "dg_launch.h", "dg_api.hip")
TRI_SOURCES = ("dg_common.h", "dg_device.h", "dg_tri_dev.h", "dg_tri_api.hip")

MAIN = "rain-3d-q3-64x64x32"
TRI = "bubble-2d-p3-512x256x2"


def csrc_hash(sources=STAGE_SOURCES) -> str:
    """Hash of a kernel's sources: a committed traffic figure is used only
    while it matches."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2305_13847_amd", "csrc")
    for f in sources:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str, sources=STAGE_SOURCES):
    """HBM bytes per launch from committed rocprof counter runs, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("csrc_hash") != csrc_hash(sources):
        return None
    return ent.get("bytes_per_launch")


def stage_alg_bytes(s_bytes: int, nvars: int, nodes: int) -> float:
    """Algorithmic bytes of one fused SSPRK(4,3) stage launch: 9 state passes
    over 4 stages (read U_s, write U_{s+1}, U_n once) plus the warm start."""
    return 2.25 * s_bytes * nvars * nodes + WARM_START_BYTES_PER_NODE * nodes


def roofline(kernel: str, kernel_us: float, alg: float, traffic=None) -> dict:
    achieved = alg / (kernel_us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel, "kernel_us": kernel_us,
            "alg_bytes_per_launch": alg}


def _sync(torch):
    torch.cuda.synchronize()


def timed_replays(step, steps, warmup, replays, torch):
    """Warm-up, then `replays` regions of exactly `steps` steps; seconds per region."""
    if warmup:
        step(warmup)
    _sync(torch)
    out = []
    for _ in range(replays):
        _sync(torch)
        t0 = time.perf_counter()
        step(steps)
        _sync(torch)
        out.append(time.perf_counter() - t0)
    return out


def kernel_pass(dg, step, steps, lib, torch):
    """Per-kernel average durations (HIP events) over `steps` more steps."""
    dg.timing(True)
    step(steps)
    _sync(torch)
    out = {}
    for name, k in (("stage", lib.DG_K_STAGE), ("split", lib.DG_K_SPLIT), ("other", lib.DG_K_OTHER)):
        ms, n = dg.timing_read(k)
        out[name + "_us"] = 1e3 * ms / max(n, 1)
        out[name + "_launches"] = n
    dg.timing(False)
    return out


def time_workload(case, precision, steps, warmup, replays, lib, torch, kernels=True, **over):
    dg = lib.for_case(case, precision=precision, **over)
    dt = torch.float64 if precision == lib.DG_FP64 else torch.float32
    U = torch.tensor(case.U, dtype=dt, device="cuda").contiguous()
    step = lambda n: dg.rk_step(U, case.dt, n)
    secs = timed_replays(step, steps, warmup, replays, torch)
    med = float(np.median(secs))
    dofs = case.U.size
    out = dict(dofs=dofs, steps=steps, replays=replays, dof_stage_per_s=dofs * 4 * steps / med,
               ms_per_step=1e3 * med / steps, replay_ms_per_step=[1e3 * s / steps for s in secs])
    if kernels:
        out.update(kernel_pass(dg, step, max(2, steps // 2), lib, torch))
    st = dg.stats()
    out["newton_max_iters"] = st["max_iters"]
    out["status"] = st["status"]
    dg.close()
    return out


def tri_alg_bytes(s_bytes: int, nvars: int, order: int, ne: int) -> float:
    """Algorithmic bytes of one fused triangle stage launch: the coefficients
    read and written (and U_n in one stage of four), the projected T and rho_v
    read and written in FP64, and 60 bytes of geometry and neighbour table."""
    npk = (order + 1) * (order + 2) // 2
    return ne * (2.25 * s_bytes * nvars * npk + 4 * 8 * npk + 60)


def time_tri(precision, steps, warmup, replays, lib, torch, synth, n=(512, 256), order=3):
    """The 2D moist bubble on a triangulation of n[0] x n[1] cells (two
    triangles each), P^k, projected onto the library's basis on the GPU."""
    case = synth.tri_bubble(n=n, order=order, noise=1e-4)
    dg = lib.for_tri_case(case, precision=precision)
    C = dg.state(case.point_state)
    step = lambda k: dg.rk_step(C, case.dt, k)
    secs = timed_replays(step, steps, warmup, replays, torch)
    med = float(np.median(secs))
    dofs = C.numel()
    out = dict(workload=case.name, dofs=dofs, elements=case.mesh.ne, dof_stage_per_s=dofs * 4 * steps / med,
               ms_per_step=1e3 * med / steps)
    out.update(kernel_pass(dg, step, max(2, steps // 2), lib, torch))
    sb = 8 if precision == lib.DG_FP64 else 4
    out["roofline"] = roofline("tri_stage_kernel<%s,%d,dry,stage>" % ("double" if sb == 8 else "float", order),
                               out["stage_us"], tri_alg_bytes(sb, case.nvars, order, case.mesh.ne),
                               traffic_for("stage", "%s-fp%d" % (case.name, 8 * sb), TRI_SOURCES))
    out["status"] = dg.stats()["status"]
    dg.close()
    return out


def time_ensemble(steps, replays, lib, torch, synth):
    """64 uneven 2D bubbles (Q3, 5 vars) in one handle, FP32 bulk: hipGraph
    replays and eager stepping after autotuning."""
    cases = synth.ensemble(nmembers=64, order=3, nsteps=steps)
    dts = np.array([c.dt for c in cases])
    dg = lib.for_ensemble(cases, precision=lib.DG_FP32_BULK)
    U = torch.cat([torch.tensor(c.U, dtype=torch.float32).reshape(c.nvars, -1) for c in cases],
                  dim=1).contiguous().cuda().reshape(dg.shape)
    dofs = sum(c.U.size for c in cases)
    nodes = dofs // cases[0].nvars
    tune = dg.autotune(U, dts, nsteps=2)
    graph = timed_replays(lambda n: dg.rk_step_graph(U, dts, n), steps, 1, replays, torch)
    eager = timed_replays(lambda n: dg.rk_step(U, dts, n), steps, 1, replays, torch)
    kt = kernel_pass(dg, lambda n: dg.rk_step(U, dts, n), max(2, steps // 2), lib, torch)
    st = dg.stats()
    dg.close()
    g, e = float(np.median(graph)), float(np.median(eager))
    alg = stage_alg_bytes(4, cases[0].nvars, nodes)
    return {"dof_stage_per_s": dofs * 4 * steps / g, "ms_per_step": 1e3 * g / steps,
            "eager_ms_per_step": 1e3 * e / steps, "eager_dof_stage_per_s": dofs * 4 * steps / e,
            "members": len(cases), "dofs": dofs, "elements": sum(c.mesh.ne for c in cases), "launch": tune,
            "stage_us": kt["stage_us"], "split_us": kt["split_us"],
            "roofline_frac": alg / (kt["stage_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "step_level_frac": 4 * alg / (g / steps) / 1e9 / HBM_PEAK_GBS, "status": st["status"]}


def host_cpu() -> dict:
    """Model, sockets, cores and SMT of the host, from lscpu."""
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except Exception:
        pass
    def num(k):
        try:
            return int(info.get(k, ""))
        except ValueError:
            return None
    return {"model": info.get("Model name"), "sockets": num("Socket(s)"),
            "cores_per_socket": num("Core(s) per socket"), "threads_per_core": num("Thread(s) per core"),
            "logical_cpus": num("CPU(s)"), "os_cpu_count": os.cpu_count()}


def _weights(case):
    """Quadrature weight times Jacobian of every node (Lobatto nodes, or the
    Gauss points of the Legendre basis)."""
    m = case.mesh
    k, p1 = m.order, m.order + 1
    if getattr(m, "basis", "lobatto") == "gauss":
        w = np.polynomial.legendre.leggauss(p1)[1]
    else:
        x = synth_mod().lobatto_points(k)
        Pk = np.polynomial.legendre.legval(x, [0] * k + [1])
        w = 2.0 / (k * (k + 1) * Pk ** 2)
    W = np.ones(p1 ** m.dim)
    for a in range(m.dim):
        W *= w[(np.arange(p1 ** m.dim) // p1 ** a) % p1]
    return W[None, :] * np.prod(m.h) / 2 ** m.dim


def synth_mod():
    from paper_2305_13847_amd import synth
    return synth


def error_table(got, ref, case):
    W = _weights(case)
    floor = 1e-12 * np.sqrt(np.sum(W * ref[-1] ** 2))
    l2 = [float(np.sqrt(np.sum(W * (got[v] - ref[v]) ** 2)) / max(np.sqrt(np.sum(W * ref[v] ** 2)), floor))
          for v in range(ref.shape[0])]
    mx = [float(np.abs(got[v] - ref[v]).max() / max(np.abs(ref[v]).max(), 1e-300)) for v in range(ref.shape[0])]
    return {"rel_l2": l2, "rel_max": mx}


def cpu_baseline(synth, oracle_mod, lib, torch):
    """The FP64 reference (the oracle) on the host cores, beside the GPU.

    Timing: two SSPRK(4,3) steps (eight stages) of the full 3D warm-rain
    workload (64 x 64 x 32 elements, Q3, 7 variables) after one warm-up
    right-hand side, on all cores (OpenMP over elements); and one step on one
    thread of a 32 x 32 x 32-element column sample (same vertical structure
    and physics).  The same reference run for ten steps is the yardstick of
    the GPU's per-field error in FP32 bulk and FP64: on 16 x 16 x 8 elements
    of the 3D workload, on 8 x 8 x 4 elements of it in the Legendre/Gauss
    basis, and on the 2D bubble (32 x 16, Q4).
    """
    c = synth.warm_rain_3d()
    o = oracle_mod.Oracle.for_case(c)
    nthreads = oracle_mod.get_threads()
    o.rhs(c.U)
    t0 = time.perf_counter()
    o.rk(c.U, c.dt, 2)
    el_all = time.perf_counter() - t0
    dofs_all = c.U.size
    del o, c
    c = synth.warm_rain_3d(n=(32, 32, 32))
    o = oracle_mod.Oracle.for_case(c)
    oracle_mod.set_threads(1)
    try:
        o.rhs(c.U)
        t0 = time.perf_counter()
        o.rk(c.U, c.dt, 1)
        el_one = time.perf_counter() - t0
    finally:
        oracle_mod.set_threads(nthreads)
    del o
    # per-field error of the GPU against the reference, ten steps
    def field_errors(e, names, label):
        ref, _ = oracle_mod.Oracle.for_case(e).rk(e.U, e.dt, 10)
        out = {}
        for prec, name in ((lib.DG_FP32_BULK, "fp32_bulk"), (lib.DG_FP64, "fp64")):
            dg = lib.for_case(e, precision=prec)
            U = torch.tensor(e.U, dtype=torch.float32 if prec == lib.DG_FP32_BULK else torch.float64,
                             device="cuda").contiguous()
            dg.rk_step(U, e.dt, 10)
            _sync(torch)
            out[name] = error_table(U.double().cpu().numpy().reshape(e.U.shape), ref, e)
            dg.close()
        out["variables"] = names
        out["case"] = label + ", 10 SSPRK(4,3) steps, quadrature-weighted relative L2 and max"
        return out

    v3 = ["rho_d'", "rho_m'", "rho_r'", "m_x", "m_y", "m_z", "E'"]
    errs = field_errors(synth.warm_rain_3d(n=(16, 16, 8)), v3, "3D warm rain 16x16x8 Q3")
    errs["others"] = {
        "rain3d_q3_gauss": field_errors(synth.warm_rain_3d(n=(8, 8, 4), basis="gauss"), v3,
                                        "3D warm rain 8x8x4 Q3, Legendre/Gauss basis"),
        "bubble2d_q4": field_errors(synth.moist_bubble(n=(32, 16)), ["rho_d'", "rho_m'", "m_x", "m_z", "E'"],
                                    "2D moist bubble 32x16 Q4"),
    }
    return {"value": dofs_all * 8 / el_all, "unit": "DoF-stage updates/s", "cores": nthreads, "kind": "oracle",
            "sample": "two SSPRK(4,3) steps (8 stages) of the full 3D warm-rain workload (64x64x32 elements, "
                      "Q3, 7 vars, %d DoFs), OpenMP over elements on %d threads, %.1f s"
                      % (dofs_all, nthreads, el_all),
            "single_thread": {"value": c.U.size * 4 / el_one, "cores": 1,
                              "sample": "one step (4 stages) of a 32x32x32-element column sample of the same "
                                        "workload (%d DoFs), %.1f s" % (c.U.size, el_one)},
            "host": host_cpu()}, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="steps per timed replay")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replays", type=int, default=5, help="timed replays (the median is reported)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", choices=["fp32", "fp64", "gauss-fp32", "gauss-fp64", "sip-fp32", "tri-fp32",
                                       "tri-fp64"],
                    help="time one 3D warm-rain variant only, without kernel timing (for profilers)")
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

    if args.only and args.only.startswith("tri"):
        prec = lib.DG_FP64 if args.only.endswith("fp64") else lib.DG_FP32_BULK
        case = synth.tri_bubble(n=(512, 256), order=3, noise=1e-4)
        dg = lib.for_tri_case(case, precision=prec)
        C = dg.state(case.point_state)
        secs = timed_replays(lambda k: dg.rk_step(C, case.dt, k), args.steps, args.warmup, args.replays, torch)
        print(json.dumps({"only": args.only, "ms_per_step": 1e3 * float(np.median(secs)) / args.steps}))
        return
    if args.only:
        basis = "gauss" if args.only.startswith("gauss") else "lobatto"
        prec = lib.DG_FP64 if args.only.endswith("fp64") else lib.DG_FP32_BULK
        over = {"sip_gamma": 0.6} if args.only.startswith("sip") else {}
        case = synth.warm_rain_3d(basis=basis)
        r = time_workload(case, prec, args.steps, args.warmup, args.replays, lib, torch, kernels=False, **over)
        print(json.dumps({"only": args.only, **r}))
        return

    case = synth.warm_rain_3d()
    nvars, nodes = case.nvars, case.U.size // case.nvars
    res = time_workload(case, lib.DG_FP32_BULK, args.steps, args.warmup, args.replays, lib, torch)
    roof = roofline("rhs_q3_kernel<float,rain,stage>", res["stage_us"], stage_alg_bytes(4, nvars, nodes),
                    traffic_for("stage", MAIN + "-fp32"))
    # the stand-alone split runs once per dg_rk_step call (the fused stage
    # kernels split every later stage state); the step-level fraction counts
    # everything between the synchronisations
    roof["call_split_kernel_us"] = res["split_us"]
    roof["step_level_frac"] = 4 * roof["alg_bytes_per_launch"] / (res["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS

    extra = {}
    if not args.no_extra:
        r64 = time_workload(case, lib.DG_FP64, max(2, args.steps // 2), 1, args.replays, lib, torch)
        extra["rain3d_fp64"] = {k: r64[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us", "split_us")}
        extra["rain3d_fp64"]["roofline"] = roofline("rhs_q3_kernel<double,rain,stage>", r64["stage_us"],
                                                    stage_alg_bytes(8, nvars, nodes),
                                                    traffic_for("stage", MAIN + "-fp64"))
        extra["rain3d_fp32_over_fp64"] = r64["ms_per_step"] / res["ms_per_step"]
        # the same FP32 workload with the Rayleigh sponge above 7 km, fused into
        # the last stage of every step
        rsp = time_workload(case, lib.DG_FP32_BULK, args.steps, args.warmup, args.replays, lib, torch,
                            sponge_zD=7.0e3, sponge_alpha=0.5)
        extra["rain3d_fp32_sponge"] = {k: rsp[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us")}
        # the same FP32 workload with the artificial diffusion (gamma 0.6, the
        # paper's 3D value); its kernels per stage are the "other" class
        rsi = time_workload(case, lib.DG_FP32_BULK, args.steps, args.warmup, args.replays, lib, torch,
                            sip_gamma=0.6)
        extra["rain3d_fp32_sip"] = {k: rsi[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us")}
        extra["rain3d_fp32_sip"]["sip_us_per_stage"] = rsi["other_us"]
        del case
        # the paper's own basis: Legendre modes with Gauss quadrature
        case_g = synth.warm_rain_3d(basis="gauss")
        for prec, nm, st in ((lib.DG_FP32_BULK, "rain3d_fp32_gauss", args.steps),
                             (lib.DG_FP64, "rain3d_fp64_gauss", max(2, args.steps // 2))):
            rg = time_workload(case_g, prec, st, 1, args.replays, lib, torch)
            sb = 4 if prec == lib.DG_FP32_BULK else 8
            extra[nm] = {k: rg[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us")}
            extra[nm]["roofline_frac"] = stage_alg_bytes(sb, nvars, nodes) / (rg["stage_us"] * 1e-6) / 1e9 \
                / HBM_PEAK_GBS
        del case_g
        bub = synth.moist_bubble()
        for prec, nm in ((lib.DG_FP64, "bubble2d_q4_fp64"), (lib.DG_FP32_BULK, "bubble2d_q4_fp32")):
            r = time_workload(bub, prec, 50, 5, args.replays, lib, torch)
            extra[nm] = {k: r[k] for k in ("dof_stage_per_s", "ms_per_step", "stage_us", "split_us")}
        extra["ensemble64_q3_fp32"] = time_ensemble(20, args.replays, lib, torch, synth)
        # triangles (the simplicial P^k space): the 2D bubble on 512 x 256 x 2 triangles, P3
        for prec, nm in ((lib.DG_FP32_BULK, "bubble2d_tri_p3_fp32"), (lib.DG_FP64, "bubble2d_tri_p3_fp64")):
            extra[nm] = time_tri(prec, 10, 2, args.replays, lib, torch, synth)
    cpu = None
    if not args.no_cpu:
        import oracle as oracle_mod
        cpu, errs = cpu_baseline(synth, oracle_mod, lib, torch)
        extra["error_vs_oracle"] = errs

    line = {
        "metric": "DG DoF-stage updates/s (FP64 plain vs FP32/batched) + % of HBM roofline",
        "value": res["dof_stage_per_s"],
        "unit": "DoF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "replays": args.replays,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 split)",
        "data": "synthetic",
        "config": {"workload": "3D warm rain, 64x64x32 hexahedra, Q3, 7 variables, Kessler rain "
                               "v_r = 5 m/s, SSPRK(4,3), FP32 bulk + FP64 split",
                   "dofs": res["dofs"], "stages_per_step": 4, "parallelism": "single GPU",
                   "replay_ms_per_step": res["replay_ms_per_step"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
        "newton_max_iters": res["newton_max_iters"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
