"""The pins can fail: plausible mistakes planted in a copy of the reference.

Each case edits one expression of oracle/dg_oracle.cpp in a temporary copy
(on the CPU), builds it, and runs the named pin files against that build in a
child process (DG_ORACLE_LIB).  The case passes when the pins fail.  The
committed reference is never modified.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dg_oracle.cpp")

# (name, text in the reference, planted replacement, pin files)
MUTATIONS = [
    # terminal rain speed (Section 2.1)
    ("vr exponent", "q.vr = pref * pw(pos(q.rr), 0.125);", "q.vr = pref * pw(pos(q.rr), 0.13);",
     ["test_oracle_rain_speed.py"]),
    ("vr prefactor", "P.v0r * std::tgamma(4.5) / 6.0", "P.v0r * std::tgamma(4.0) / 6.0",
     ["test_oracle_rain_speed.py"]),
    ("rain falls up", "q.F[j][v_rr(c)] = q.rr * (q.u[j] - vz);", "q.F[j][v_rr(c)] = q.rr * (q.u[j] + vz);",
     ["test_oracle_rain_speed.py"]),
    # viscosity of the artificial diffusion and its Q1 carry (Section 3.5)
    ("swapped corner weights", "wq *= ((corner >> a) & 1) ? 0.5 * (1.0 + xi) : 0.5 * (1.0 - xi);",
     "wq *= ((corner >> a) & 1) ? 0.5 * (1.0 - xi) : 0.5 * (1.0 + xi);", ["test_oracle_sip.py"]),
    ("periodic vertex clamped, not wrapped", "if (c.M.bc[a] == 0) va %= c.M.n[a];",
     "if (c.M.bc[a] == 0) va = std::min(va, c.M.n[a] - 1);", ["test_oracle_sip.py"]),
    ("rain viscosity with u + v_r", "const double ur = (i == d - 1) ? ui - val(qq.vr) : ui;",
     "const double ur = (i == d - 1) ? ui + val(qq.vr) : ui;", ["test_oracle_sip.py"]),
    # the core right-hand side (Sections 2.3, 3.2, 3.3)
    ("gravity sign", "q.G[v_m(c, z)] = -rhop * P.g;", "q.G[v_m(c, z)] = rhop * P.g;",
     ["test_oracle_rhs.py"]),
    ("jump sign", "b.F[j][v]) + 0.5 * L * (Ua[v] - Ub[v]);", "b.F[j][v]) + 0.5 * L * (Ub[v] - Ua[v]);",
     ["test_oracle_rhs.py"]),
    ("wall not reflected", "Ug[v_m(c, j)] = -Ua[v_m(c, j)];", "Ug[v_m(c, j)] = Ua[v_m(c, j)];",
     ["test_oracle_rhs.py"]),
    ("v_r left out of the wave speed", "q.lam[j] = absr(q.u[j]) + absr(vz) + q.cm;",
     "q.lam[j] = absr(q.u[j]) + q.cm;", ["test_oracle_rhs.py"]),
    ("transposed volume matrix", "s += c.tab.Dhat[ij * p1 + a] *", "s += c.tab.Dhat[a * p1 + ij] *",
     ["test_oracle_rhs.py"]),
    # triangles (Section 3.1 space, Section 3.4 rule, Section 3.2 flux)
    ("Duffy weight without the collapse factor", "R.w.push_back(ga.w[i] * gb.w[j] * (1.0 - s) / 4.0);",
     "R.w.push_back(ga.w[i] * gb.w[j] / 4.0);", ["test_oracle_tri.py"]),
    ("triangle normal turned the wrong way", "g.n[f][0] = dzz / g.len[f];", "g.n[f][0] = -dzz / g.len[f];",
     ["test_oracle_tri.py"]),
    ("inverse Jacobian not transposed", "g.G[0][1] = -a10 / g.det;", "g.G[0][1] = -a01 / g.det;",
     ["test_oracle_tri.py"]),
    ("neighbour's face points not reversed", "&c.psi_f[((size_t)f2 * nf + (k - i)) * np]",
     "&c.psi_f[((size_t)f2 * nf + i) * np]", ["test_oracle_tri.py"]),
    ("triangle wall reflects all momentum",
     "Ug[v_m(c.base, a)] = Ut[v_m(c.base, a)] - 2.0 * mn * g.n[f][a];",
     "Ug[v_m(c.base, a)] = -Ut[v_m(c.base, a)];", ["test_oracle_tri.py"]),
    ("triangle wave speed without v_r", "R lb = absr(b.u[0] * n[0] + b.u[1] * n[1]) + absr(b.vr * n[1]) + b.cm;",
     "R lb = absr(b.u[0] * n[0] + b.u[1] * n[1]) + b.cm;", ["test_oracle_tri.py"]),
    ("triangle jump sign", "b.F[1][v]) * n[1]) + 0.5 * L * (Ua[v] - Ub[v]);",
     "b.F[1][v]) * n[1]) + 0.5 * L * (Ub[v] - Ua[v]);", ["test_oracle_tri.py"]),
    ("triangle face weight doubled", "const double wf = g.len[f] * 0.5 * c.gf.w[i] / g.det;",
     "const double wf = g.len[f] * c.gf.w[i] / g.det;", ["test_oracle_tri.py"]),
    ("RK weight", "us[i] = (2.0 / 3.0) * u0[i] + (1.0 / 3.0) * us[i] + (dt / 6.0) * L[i];",
     "us[i] = (2.0 / 3.0) * u0[i] + (1.0 / 3.0) * us[i] + (dt / 5.0) * L[i];",
     ["test_oracle_rhs.py", "test_oracle_convergence.py"]),
]


@pytest.mark.parametrize("name,old,new,files", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(name, old, new, files, tmp_path):
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, "mutation site not unique: " + name
    mutated = tmp_path / "dg_oracle_mutated.cpp"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libdgoracle_mutated.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-o", str(lib),
                           str(mutated)])
    env = dict(os.environ, DG_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + \
          [os.path.join(ROOT, "tests", f) for f in files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, "%s: pins passed with the planted mistake\n%s" % (name, r.stdout[-2000:])
