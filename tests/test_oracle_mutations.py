"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks that its pins catch
each one: a pinned oracle must fail when a term is dropped, a sign flipped, an index or an
operand order changed.  Each mutant of the C oracle is compiled to a temporary library, each
mutant of the numpy surrogate oracle is loaded in place of oracle.surrogate, and the relevant pin
file is run against it in a subprocess."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rcell_oracle.c")

MUTANTS = [
    ("FENE force sign", "double g = K * r / (1.0 - t);", "double g = -K * r / (1.0 - t);", "forces"),
    ("LJ energy shift dropped", "*pe += 4.0 * e * (sr6 * sr6 - sr6) - shift;",
     "*pe += 4.0 * e * (sr6 * sr6 - sr6);", "forces"),
    ("EAM embedding of j replaced by i", "(rho[q->i] + rho[q->j]) * drho", "(rho[q->i] + rho[q->i]) * drho", "forces"),
    ("virial index", "W[3 * a + b] += g * d[a] * d[b] / r;", "W[3 * a + b] += g * d[a] * d[a] / r;", "forces"),
    ("EAM density shift dropped", "double rr = pow(a / q->r, p->sc_m) - rhoc;", "double rr = pow(a / q->r, p->sc_m);", "forces"),
    ("rotation reversed", "mul3(Q, s, t);\n  mul3(t, Qt, sf);", "mul3(Qt, s, t);\n  mul3(t, Q, sf);", "coupling"),
    ("F^-1 instead of F^-T", "mul3(sf, FiT, pm);", "mul3(sf, Fi, pm);", "coupling"),
    ("Delta R operand order", "mul3(R + 9 * k, Ri, dR + 9 * k);", "mul3(Ri, R + 9 * k, dR + 9 * k);", "coupling"),
    ("tilt reduction drops the xy part of c", "H[2] -= k * H[1]; H[5] -= k * H[4];", "H[5] -= k * H[4];", "coupling"),
    ("Gram-Schmidt projection sign", "v[0] -= s * q[i][0]; v[1] -= s * q[i][1];", "v[0] += s * q[i][0]; v[1] -= s * q[i][1];", "coupling"),
    ("noise variance halved", "double c24 = sqrt(24.0 *", "double c24 = sqrt(12.0 *", "dynamics"),
    ("drag sign", "double drag = -(p->gamma", "double drag = (p->gamma", "dynamics"),
    ("kinetic stress sign", "(W[3 * ia[k] + ib[k]] - K[3 * ia[k] + ib[k]]) / V",
     "(W[3 * ia[k] + ib[k]] + K[3 * ia[k] + ib[k]]) / V", "dynamics"),
    ("full kick instead of half kick", "double h = p->dt / (2.0 * p->mass * p->mvv2e);",
     "double h = p->dt / (p->mass * p->mvv2e);", "dynamics"),
    ("Philox Weyl constant", "k0 += 0x9E3779B9u;", "k0 += 0x9E3779B7u;", "philox"),
    # the Maxwell-Boltzmann initial velocities
    ("Box-Muller cosine for two components", "c->v[3 * i + 1] = sd * r0 * sin(two_pi * u[1]);",
     "c->v[3 * i + 1] = sd * r0 * cos(two_pi * u[1]);", "dynamics"),
    ("centre-of-mass velocity kept", "c->v[3 * i + q] -= mean[q];", "c->v[3 * i + q] -= 0.0 * mean[q];", "dynamics"),
    ("3N degrees of freedom", "sqrt(kt_m * (3.0 * c->n - 3.0) / sum2)", "sqrt(kt_m * (3.0 * c->n) / sum2)", "dynamics"),
    ("window average over one step too many",
     "sv[q] = c->wcount > 0 ? c->wsum[q] / (double)c->wcount : c->last[q];",
     "sv[q] = c->wcount > 0 ? c->wsum[q] / (double)(c->wcount + 1) : c->last[q];", "dynamics"),
    ("window kept across a deformation",
     "    memset(c->wsum, 0, sizeof c->wsum); c->wcount = 0;\n    wrap_positions(c);\n    int st = prime(&C->p, c);",
     "    wrap_positions(c);\n    int st = prime(&C->p, c);", "dynamics"),
    ("drift before the first half kick",
     "  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->v[k] += h * c->f[k];\n"
     "  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->x[k] += p->dt * c->v[k];\n  wrap_positions(c);\n  double W[9];",
     "  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->x[k] += p->dt * c->v[k];\n"
     "  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->v[k] += h * c->f[k];\n  wrap_positions(c);\n  double W[9];",
     "dynamics"),
    ("kinetic tensor without the metal-units factor",
     "K[3 * a + b] += p->mass * p->mvv2e * c->v[3 * i + a] * c->v[3 * i + b];",
     "K[3 * a + b] += p->mass * c->v[3 * i + a] * c->v[3 * i + b];", "dynamics"),
    ("previous stretch not updated by a deformation", "    memcpy(c->Rprev, R + 9 * k, sizeof c->Rprev);\n", "", "coupling"),
    ("statics returns the stress of the unrelaxed start", "    if (st == OK) sample_stress(p, c, W, c->last);\n", "",
     "statics"),
    ("statics leaves the minimiser's velocities",
     "    memset(c->v, 0, (size_t)n3 * sizeof(double));\n    if (st == OK) sample_stress",
     "    if (st == OK) sample_stress", "statics"),
    ("statics converges on the summed force", "if (fmax2 <= ftol * ftol || it >= max_iter) break;",
     "if (F2 <= ftol * ftol * 1e6 || it >= max_iter) break;", "statics"),
    ("noise mean not removed", "double xi = c24 * ((double)kk[3 * i + a] - mean[a]);",
     "double xi = c24 * (double)kk[3 * i + a];", "dynamics"),
    ("drag omitted", "c->f[3 * i + a] = (c->f[3 * i + a] + drag * c->v[3 * i + a]) + xi;",
     "c->f[3 * i + a] = c->f[3 * i + a] + xi;", "dynamics"),
    ("FENE energy and force both without R0^2",
     "*pe += -0.5 * K * R0 * R0 * log(1.0 - t);\n      double g = K * r / (1.0 - t);",
     "*pe += -0.5 * K * log(1.0 - t);\n      double g = K * r / (1.0 - t) / (R0 * R0);", "forces"),
    ("embedding linear in rho (energy and force alike)",
     "      *pe += -e * c * sqrt(rho[i]);\n      rho[i] = rho[i] > 0.0 ? -e * c / (2.0 * sqrt(rho[i])) : 0.0;",
     "      *pe += -e * c * rho[i];\n      rho[i] = -e * c;", "forces"),
    ("J left at 1 after a deformation", "c->J = c->R[0] * c->R[4] * c->R[8];", "c->J = 1.0;", "coupling"),
    ("positions not remapped by Delta R",
     "for (int32_t i = 0; i < c->n; ++i) matvec(dR + 9 * k, &c->x[3 * i], &c->x[3 * i]);", "", "coupling"),
    # the cell-list branch of the pair search: bins narrower than the cutoff in a skewed box, and a
    # stencil that misses the neighbouring bin below
    ("bin count from the box edge instead of the perpendicular width",
     "for (int k = 0; k < 3; ++k) nb[k] = (int)floor(w[k] / rc);",
     "for (int k = 0; k < 3; ++k) nb[k] = (int)floor(H[4 * k] / rc);", "forces"),
    ("stencil skips the lower z bin", "for (int o2 = -1; o2 <= 1; ++o2) {", "for (int o2 = 0; o2 <= 1; ++o2) {",
     "forces"),
]

SUR_SRC = os.path.join(ROOT, "oracle", "surrogate.py")
SUR_MUTANTS = [
    ("ensemble variance scaled by y_sd instead of y_sd^2",
     "    outs = np.stack([forward(p, dims, Xn)[0] * y_sd + y_mu for p in params])\n"
     "    return outs.mean(0), outs.var(0)",
     "    outs = np.stack([forward(p, dims, Xn)[0] for p in params])\n"
     "    return outs.mean(0) * y_sd + y_mu, outs.var(0) * y_sd"),
    ("ensemble variance with K - 1 in the denominator", "return outs.mean(0), outs.var(0)",
     "return outs.mean(0), outs.var(0, ddof=1)"),
    ("input normalisation multiplies by the spread", "return (X - mu) / sd", "return (X - mu) * sd"),
    ("SiLU derivative drops a factor", "return s * (1.0 + z * (1.0 - s))", "return s * (1.0 + z * s)"),
    ("weight gradient of the wrong layer input", "gW[l] = acts[l].T @ dz", "gW[l] = acts[l + 1].T @ dz"),
    ("Adam without bias correction", "mh = m / (1 - b1 ** t)", "mh = m"),
    ("Adam epsilon inside the root", "return p - lr * mh / (np.sqrt(vh) + eps), m, v",
     "return p - lr * mh / np.sqrt(vh + eps), m, v"),
    ("bias gradient averaged instead of summed", "gb[l] = dz.sum(0)", "gb[l] = dz.mean(0)"),
    ("loss gradient without its factor 2", "return float((d * d).mean()), 2.0 * d / d.size",
     "return float((d * d).mean()), d / d.size"),
    ("back-propagation through the wrong pre-activation", "dz = (dz @ Ws[l].T) * silu_grad(zs[l - 1])",
     "dz = (dz @ Ws[l].T) * silu_grad(zs[l])"),
]

# loads the mutated file as oracle.surrogate, then runs the surrogate pins
_SUR_BOOT = (
    "import importlib.util, sys; import oracle; "
    "spec = importlib.util.spec_from_file_location('oracle.surrogate', sys.argv[1]); "
    "m = importlib.util.module_from_spec(spec); sys.modules['oracle.surrogate'] = m; "
    "spec.loader.exec_module(m); oracle.surrogate = m; import pytest; "
    "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', sys.argv[2]]))")


def _run_sur_mutant(m, tmp):
    name, old, new = m
    src = open(SUR_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique or missing: {name}"
    path = os.path.join(tmp, f"sur_{abs(hash(name))}.py")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    r = subprocess.run([sys.executable, "-c", _SUR_BOOT, path,
                        os.path.join(ROOT, "tests", "test_oracle_surrogate.py")],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def _run_mutant(m, tmp):
    name, old, new, target = m
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique or missing: {name}"
    mdir = os.path.join(tmp, f"{abs(hash(name))}_{target}")
    os.makedirs(mdir, exist_ok=True)
    csrc = os.path.join(mdir, "m.c")
    with open(csrc, "w") as fh:
        fh.write(src.replace(old, new))
    for h in ("rcell_oracle.h",):
        with open(os.path.join(mdir, h), "w") as fh:
            fh.write(open(os.path.join(ROOT, "oracle", h)).read())
    lib = os.path.join(mdir, "libm_oracle.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", csrc, "-o", lib, "-lm"])
    env = dict(os.environ, RCELL_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    # the statics pins without their slowest case (two relaxations beyond stability, ~45 s)
    sel = ["-k", "not beyond_stability"] if target == "statics" else []
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *sel,
                        os.path.join(ROOT, "tests", f"test_oracle_{target}.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


CONTROLS = [("unmutated copy", "int orc_threads(int32_t n) {", "int orc_threads(int32_t n) {", t)
            for t in ("forces", "coupling", "dynamics", "philox", "statics")]


def test_surrogate_pins_catch_planted_mistakes():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
            results = list(ex.map(lambda m: _run_sur_mutant(m, tmp), SUR_MUTANTS + [("unmutated copy", "import numpy as np",
                                                                                      "import numpy as np")]))
    control = results[-1]
    assert control[1] == 0, f"the harness fails on the unmutated surrogate oracle: {control}"
    survivors = [name for name, rc in results[:-1] if rc == 0]
    assert not survivors, f"mutants not caught by the pins: {survivors}"


def test_pins_catch_planted_mistakes():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
            results = list(ex.map(lambda m: _run_mutant(m, tmp), MUTANTS + CONTROLS))
    controls = results[len(MUTANTS):]
    results = results[:len(MUTANTS)]
    assert all(rc == 0 for _, rc in controls), f"the harness fails on the unmutated oracle: {controls}"
    survivors = [name for name, rc in results if rc == 0]
    assert not survivors, f"mutants not caught by the pins: {survivors}"
