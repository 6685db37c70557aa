"""Space-time self-convergence of the GPU path on the gravity-wave case
(Section 4.1, convergence study of its results).

Meshes are nested: level r has 30 r x r elements (h = 10 km / r).
- Every run is stopped at nsnap equidistant times.
- A coarse solution is interpolated (its own Lagrange basis on its nodes) to
  the nodes of the reference level.
- The error is the l2(L2) norm over the snapshots:
  sum_i ||x_h(t_i) - x_ref(t_i)||^2_L2, with the reference level's
  quadrature. It is reported per conserved variable, relative to the same
  norm of the reference.
- The basis is the Lobatto collocation or the paper's Legendre space with
  Gauss quadrature (held by its values at the Gauss points); the reference
  run uses the same basis as the levels.

Everything here drives the library through its C ABI (dg_rk_step); torch only
holds the arrays and does the interpolation.

    python -m paper_2305_13847_amd.ex1_convergence --levels 2 4 8 --ref 16 --t-end 600
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lib, synth

VARS = ("rho_d'", "rho_m'", "m_x", "m_z", "E'")


def _lagrange(xn: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[a, b] = l_b(x_a) for the Lagrange basis on nodes xn."""
    L = np.ones((len(x), len(xn)))
    for b in range(len(xn)):
        for c in range(len(xn)):
            if c != b:
                L[:, b] *= (x - xn[c]) / (xn[b] - xn[c])
    return L


def run(r: int, k: int, t_end: float, nsnap: int, prec=lib.DG_FP64, cfl=0.5, log=None, qw=0.02,
        basis="lobatto"):
    """Snapshots (nsnap, nvars, ne, npe) on the device of the level-r, order-k run."""
    import torch
    c = synth.gravity_waves(n=(30 * r, r), order=k, t_end=t_end, cfl=cfl, qw=qw, basis=basis)
    dt_cfl = synth.cfl_dt(c.mesh, 20.0, 0.0, cfl)
    per = int(np.ceil((t_end / nsnap) / dt_cfl))
    dt = t_end / nsnap / per
    dg = lib.for_case(c, precision=prec)
    U = torch.tensor(c.U, device="cuda", dtype=torch.float64 if prec == lib.DG_FP64 else torch.float32)
    snaps = []
    t0 = time.perf_counter()
    for i in range(nsnap):
        dg.rk_step(U, dt, per)
        snaps.append(U.double().clone())
        if log:
            torch.cuda.synchronize()
            log("  r=%d k=%d snapshot %d/%d (%d steps of %.4g s, %.1f s)" % (r, k, i + 1, nsnap, per, dt,
                                                                          time.perf_counter() - t0))
    st = dg.stats()
    dg.close()
    if st["status"] != 0:
        raise RuntimeError("run r=%d k=%d reported status %d" % (r, k, st["status"]))
    return c, torch.stack(snaps), per * nsnap


def _points(k: int, basis: str) -> np.ndarray:
    return synth.gauss_points(k) if basis == "gauss" else synth.lobatto_points(k)


def to_reference(Uc, rc: int, kc: int, rf: int, kf: int, basis: str = "lobatto"):
    """Interpolate (..., nvars, ne, npe) fields of level rc / order kc onto level rf / order kf."""
    import torch
    s = rf // rc
    assert s * rc == rf
    xc, xf = _points(kc, basis), _points(kf, basis)
    nxc, nzc, nxf, nzf = 30 * rc, rc, 30 * rf, rf
    lead = Uc.shape[:-2]
    A = Uc.reshape(*lead, nzc, nxc, kc + 1, kc + 1)           # [.., ez, ex, j(z), i(x)]
    out = torch.empty(*lead, nzf, nxf, kf + 1, kf + 1, dtype=Uc.dtype, device=Uc.device)
    for oz in range(s):
        Lz = torch.tensor(_lagrange(xc, -1.0 + (2 * oz + 1.0 + xf) / s), dtype=Uc.dtype, device=Uc.device)
        for ox in range(s):
            Lx = torch.tensor(_lagrange(xc, -1.0 + (2 * ox + 1.0 + xf) / s), dtype=Uc.dtype, device=Uc.device)
            V = torch.einsum("aj,...zxji->...zxai", Lz, A)
            V = torch.einsum("bi,...zxai->...zxab", Lx, V)
            out[..., oz::s, ox::s, :, :] = V
    return out.reshape(*lead, nzf * nxf, (kf + 1) ** 2)


def l2_sq(F, rf: int, kf: int, basis: str = "lobatto"):
    """L2 norm squared of (..., ne, npe) fields on level rf (h = 10 km / rf), by the
    quadrature of the basis' nodes."""
    import torch
    w = np.polynomial.legendre.leggauss(kf + 1)[1] if basis == "gauss" else synth_weights(kf)
    h = 10.0e3 / rf
    W = torch.tensor(np.outer(w, w).reshape(-1) * (0.5 * h) ** 2, dtype=F.dtype, device=F.device)
    return (F * F * W).sum(dim=(-2, -1))


def synth_weights(k: int) -> np.ndarray:
    """Lobatto weights 2 / (k (k+1) P_k(x)^2) (for the error norm only)."""
    x = synth.lobatto_points(k)
    P = np.polynomial.legendre.legval(x, [0] * k + [1])
    return 2.0 / (k * (k + 1) * P * P)


def study(levels, orders, ref: int, kref: int, t_end: float, nsnap: int, log=print, cfl=0.5, qw=0.02,
          basis="lobatto"):
    import torch
    log("reference: r=%d (h=%g m), k=%d, cfl %g, %s basis" % (ref, 10e3 / ref, kref, cfl, basis))
    cref, Sref, nref = run(ref, kref, t_end, nsnap, log=log, cfl=cfl, qw=qw, basis=basis)
    norm = torch.sqrt(l2_sq(Sref, ref, kref, basis).sum(dim=0))     # per variable
    rows = []
    for k in orders:
        prev = None
        for r in levels:
            c, S, n = run(r, k, t_end, nsnap, log=log, cfl=cfl, qw=qw, basis=basis)
            E = torch.sqrt(l2_sq(to_reference(S, r, k, ref, kref, basis) - Sref, ref, kref, basis).sum(dim=0)) / norm
            err = E.cpu().numpy()
            rate = None if prev is None else (np.log(prev / err) / np.log(2.0)).tolist()
            rows.append(dict(k=k, r=r, h=10e3 / r, steps=n, err=err.tolist(), rate=rate))
            log("k=%d h=%6.0f m: rel l2(L2) err %s%s" % (k, 10e3 / r, " ".join("%.3e" % e for e in err),
                "" if rate is None else "  rates " + " ".join("%.2f" % q for q in rate)))
            prev = err
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--levels", type=int, nargs="+", default=[10, 20, 40])
    ap.add_argument("--orders", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--ref", type=int, default=80)
    ap.add_argument("--kref", type=int, default=4)
    ap.add_argument("--t-end", type=float, default=3600.0)
    ap.add_argument("--nsnap", type=int, default=30)
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--qw", type=float, default=0.02, help="total water ratio (0: the dry case)")
    ap.add_argument("--basis", default="lobatto", choices=["lobatto", "gauss"])
    ap.add_argument("--json", default=None, help="write the table here")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 3
    torch.zeros(1, device="cuda")          # the device runtime is up before any handle
    lib.load()
    rows = study(a.levels, a.orders, a.ref, a.kref, a.t_end, a.nsnap,
                 log=lambda m: print(m, flush=True), cfl=a.cfl, qw=a.qw, basis=a.basis)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(dict(args=vars(a), vars=VARS, rows=rows), f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
