"""The oracle's pins catch plausible mistakes: each case below plants one mistake in a copy of the
oracle's source (a flipped sign, a shifted index, a dropped or misplaced term), builds it, and runs the
fast pins of tests/test_oracle_pins.py (forward) or tests/test_oracle_adjoint.py (adjoint) against that
build, which must fail; the unaltered copy, built the same way, must pass them.  Everything runs on
the host."""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tfl_oracle.c")
# the pins that finish in about a second (the cube, the reflection-versus-frequency experiment, the
# free-space CPML reference and the 26 000-step skin-depth run are left to the main suite)
FAST = ("not table6_cube and not reflection_versus_frequency and not free_space and not config1")

# (name, text in the oracle's source, replacement): one plausible mistake each
MUTANTS = [
    ("curl E sign", "return o_dB(s, c, a1, s->E[a2], ijk, e, advance) - o_dB(s, c, a2, s->E[a1], ijk, e, advance);",
     "return o_dB(s, c, a1, s->E[a2], ijk, e, advance) + o_dB(s, c, a2, s->E[a1], ijk, e, advance);"),
    ("curl H sign", "double cH = o_dE(s, c, a1, H[a2], ijk, e) - o_dE(s, c, a2, H[a1], ijk, e);",
     "double cH = o_dE(s, c, a2, H[a1], ijk, e) - o_dE(s, c, a1, H[a2], ijk, e);"),
    ("curl E transposed operands", "return o_dB(s, c, a1, s->E[a2], ijk, e, advance) - o_dB(s, c, a2, s->E[a1], ijk, e, advance);",
     "return o_dB(s, c, a1, s->E[a1], ijk, e, advance) - o_dB(s, c, a2, s->E[a2], ijk, e, advance);"),
    ("forward difference taken backward", "    p[a] += 1;\n    double dF = (F[o_idx(s, p[0], p[1], p[2])] - F[e]) / s->d[a];",
     "    p[a] -= 1;\n    double dF = (F[e] - F[o_idx(s, p[0], p[1], p[2])]) / s->d[a];"),
    ("spacing of the other axis", "double dF = (F[e] - F[o_idx(s, p[0], p[1], p[2])]) / s->d[a];",
     "double dF = (F[e] - F[o_idx(s, p[0], p[1], p[2])]) / s->d[(a + 1) % 3];"),
    ("Js dropped from the E update", " - dt / eps * js) / (1.0 + th * sg);", ") / (1.0 + th * sg);"),
    ("theta weights swapped", "- (1.0 - th) * sg * En - dt / eps * js) / (1.0 + th * sg);",
     "- th * sg * En - dt / eps * js) / (1.0 + (1.0 - th) * sg);"),
    ("London half step doubled", "s->J[c][e] += 0.5 * s->dt * s->E[c][e] * s->ell[c][e] / O_MU0;",
     "s->J[c][e] += s->dt * s->E[c][e] * s->ell[c][e] / O_MU0;"),
    ("edge rule: mean over all four cells", "if (nsc > 0 && !(ell[cc] > 0.0)) continue;", "if (0) continue;"),
    ("edge rule: divide by four", "s->sig[c][e] = ss / (double)cnt;", "s->sig[c][e] = ss / 4.0;"),
    ("conductivity over eps0 instead of eps", "double sg = s->sig[c][e] * dt / eps;",
     "double sg = s->sig[c][e] * dt / O_EPS0;"),
    ("source one step early", "double t = (double)(s->step + 1) * dt;", "double t = (double)(s->step) * dt;"),
    ("DFT sign", "q->dft_im[f] -= sum * s->dt * sin(ph);", "q->dft_im[f] += sum * s->dt * sin(ph);"),
    ("CPML E-side variable without decay", "s->psiE[c][a][e] = s->bn[a][ia] * s->psiE[c][a][e] + s->cn[a][ia] * dF;",
     "s->psiE[c][a][e] = s->psiE[c][a][e] + s->cn[a][ia] * dF;"),
    ("PEC wall also on the edge's own axis", "if (a != c && s->pml[a] && ijk[a] == 0) return 1;",
     "if (s->pml[a] && ijk[a] == 0) return 1;"),
    ("CPML grading one order higher", "double sg = smax * pow(depth, m);", "double sg = smax * pow(depth, m + 1.0);"),
    ("CPML convolution coefficient sign", "* (*b - 1.0) : 0.0;", "* (1.0 - *b) : 0.0;"),
    ("CPML H-side variable not advanced", "o_half_B(s, 1);   /* 5.", "o_half_B(s, 0);   /* 5."),
    ("H taken as B", "H[c][e] = s->B[c][e] / O_MU0;", "H[c][e] = s->B[c][e];"),
    ("full step in the B half steps", "int advance_psi)\n{\n    double h = 0.5 * s->dt;",
     "int advance_psi)\n{\n    double h = s->dt;"),
    ("second Js half step dropped", "o_half_J(s);      /* 4.", "(void)0;      /* 4."),
    ("probe sample one index late", "if (n < q->cap) q->series[n] = sum;",
     "if (n + 1 < q->cap) q->series[n + 1] = sum;"),
    ("energy: B correction sign", "wb += (s->B[c][e] * s->B[c][e] - hb * hb) / (2.0 * O_MU0);",
     "wb += (s->B[c][e] * s->B[c][e] + hb * hb) / (2.0 * O_MU0);"),
    ("energy: Js term without 1/ell", "wj += O_MU0 * (s->J[c][e] * s->J[c][e] - hj * hj) / (2.0 * s->ell[c][e]);",
     "wj += O_MU0 * (s->J[c][e] * s->J[c][e] - hj * hj) / 2.0;"),
    ("edge rule: eps divided by four", "s->eps[c][e] = O_EPS0 * se / (double)cnt;", "s->eps[c][e] = O_EPS0 * se / 4.0;"),
]

# mistakes in the oracle's adjoint, run against tests/test_oracle_adjoint.py (central differences of the
# oracle's forward, the dot-product test)
ADJOINT_MUTANTS = [
    ("objective weight sign", "double gn = 2.0 * dt * (Fr * cos(ph) - Fi * sin(ph));",
     "double gn = 2.0 * dt * (Fr * cos(ph) + Fi * sin(ph));"),
    ("ell gradient of step 4 from E^m", "gl[c][e] += 0.5 * dt * X1->E[c][e] / O_MU0 * aJ[c][e];",
     "gl[c][e] += 0.5 * dt * X0->E[c][e] / O_MU0 * aJ[c][e];"),
    ("sigma gradient theta weights swapped", "(-(1.0 - th) * X0->E[c][e] - th * Epre[c][e])",
     "(-th * X0->E[c][e] - (1.0 - th) * Epre[c][e])"),
    ("transposed forward difference sign", "aE[ec[t]][e] -= w / s->d[a];", "aE[ec[t]][e] += w / s->d[a];"),
    ("adjoint of Js in the E update sign", "aJ[c][e] -= alpha * (dt / eps) * aEp;", "aJ[c][e] += alpha * (dt / eps) * aEp;"),
    ("adjoint E-side CPML variable without decay", "apsiE[c][a][e] = s->bn[a][ia] * tot;", "apsiE[c][a][e] = tot;"),
    ("normal-edge gradient spread over three cells", "grad_sig[cells[t]] += gs[c][e] / 4.0;",
     "grad_sig[cells[t]] += gs[c][e] / 3.0;"),
]


def build(tmp, name, text):
    src = os.path.join(tmp, name + ".c")
    lib = os.path.join(tmp, "lib" + name + ".so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", lib,
                           src, "-lm"])
    return lib


def run_pins(job):
    lib, pins = job
    env = dict(os.environ, TFL_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", pins), "-x", "-q", "-p", "no:cacheprovider"]
    if pins == "test_oracle_pins.py":
        cmd += ["-k", FAST]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-1500:]


def test_planted_mistakes_fail_the_pins(tmp_path):
    text = open(SRC).read()
    unaltered = build(str(tmp_path), "unaltered", text)
    jobs = {"unaltered (forward pins)": (unaltered, "test_oracle_pins.py"),
            "unaltered (adjoint pins)": (unaltered, "test_oracle_adjoint.py")}
    cases = [(m, "test_oracle_pins.py") for m in MUTANTS] + [(m, "test_oracle_adjoint.py") for m in ADJOINT_MUTANTS]
    for q, ((name, old, new), pins) in enumerate(cases):
        assert text.count(old) == 1, f"mutant {name!r}: the text to replace must occur once"
        jobs[name] = (build(str(tmp_path), f"mutant{q}", text.replace(old, new)), pins)
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        res = dict(zip(jobs, ex.map(run_pins, jobs.values())))
    for name in ("unaltered (forward pins)", "unaltered (adjoint pins)"):
        rc, out = res.pop(name)
        assert rc == 0, f"the unaltered copy must pass the pins ({name}):\n" + out
    survived = [name for name, (rc, _) in res.items() if rc == 0]
    for name, (rc, out) in res.items():
        last = [ln for ln in out.splitlines() if ln.startswith("FAILED")]
        print(f"{name}: {'caught' if rc else 'SURVIVED'} {last[:1]}", flush=True)
    assert not survived, f"mistakes the pins do not catch: {survived}"
