"""The oracle's pins have teeth: each plausible mistake below (a dropped
term, a wrong sign, index or operand), planted in a private copy of the
oracle source on the CPU, must make at least one pin fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (description, text in hydro_oracle.c, replacement)
MUTATIONS = [
    ("drop the central-upwind diffusion term", "ap * am * (Up[f] - Um[f])", "0.0 * (Up[f] - Um[f])"),
    ("wrong sign of the update", "sg->u_in[g] - lambda * s", "sg->u_in[g] + lambda * s"),
    ("pressure missing from the normal momentum flux", "F[1 + d] = F[1 + d] + p;", "F[1 + d] = F[1 + d];"),
    ("left and right edge swapped at a face", "const double *Wm = &qR[i * nf];", "const double *Wm = &qL[i * nf];"),
    ("wrong interface weight", "dm[i * nf + f]) / 6.0;", "dm[i * nf + f]) / 3.0;"),
    ("overshoot fix applied to the wrong edge", "l = 3.0 * qc - 2.0 * r;", "r = 3.0 * qc - 2.0 * l;"),
    ("transposed momentum component", "double vx = U[1] / rho;", "double vx = U[2] / rho;"),
    ("one-sided speed not clipped at zero", "fmax(fmax(vm + cm, vp + cp), 0.0)", "fmax(vm + cm, vp + cp)"),
    ("pressure work missing from the energy flux", "F[4] = (U[4] + p) * vd;", "F[4] = U[4] * vd;"),
    ("central slope not halved", "double dq = 0.5 * (qp - qm);", "double dq = (qp - qm);"),
    ("slope limit without the factor 2", "2.0 * fabs(q0 - qm), 2.0 * fabs(qp - q0)", "fabs(q0 - qm), fabs(qp - q0)"),
    ("first face of each line skipped", "for (int i = 2; i <= M - 4; ++i) {", "for (int i = 3; i <= M - 4; ++i) {"),
    ("z flux difference replaced by y", "s = s + dF[(2 * nint + c) * nf + f];", "s = s + dF[(1 * nint + c) * nf + f];"),
    ("level refines the wrong way", "ldexp(dx, -sg->level)", "ldexp(dx, sg->level)"),
    ("extrema never flattened", "if ((r - qc) * (qc - l) <= 0.0) {", "if ((r - qc) * (qc - l) < -1.0) {"),
    ("wrong internal energy factor", "U[4] = W[4] / (GAMMA - 1.0) +", "U[4] = W[4] / (GAMMA) +"),
]

# mistakes in the 26-point form, caught by its own pins
MUTATIONS26 = [
    ("Simpson weights of edge midpoints and vertices swapped",
     "(s1 == 0 || s2 == 0) ? 4.0 : 1.0", "(s1 == 0 || s2 == 0) ? 1.0 : 4.0"),
    ("face quadrature not normalised", "Fh[i * nf + f] = acc[f] / 36.0;", "Fh[i * nf + f] = acc[f] / 32.0;"),
    ("high cell's point direction flipped", "ep[d] = -1;", "ep[d] = 1;"),
    ("high cell's transverse offset mirrored", "em[t1] = ep[t1] = s1;", "em[t1] = s1;\n              ep[t1] = -s1;"),
    ("value taken toward -e", "memcpy(out, &qR[2 * nf], sizeof(double) * nf);",
     "memcpy(out, &qL[2 * nf], sizeof(double) * nf);"),
]

PINS = ["tests/test_oracle_pins.py"]


@pytest.mark.slow
@pytest.mark.parametrize("desc,old,new", MUTATIONS26, ids=[m[0] for m in MUTATIONS26])
def test_planted_mistake_in_the_26_point_form_is_caught(tmp_path, desc, old, new):
    _planted(tmp_path, desc, old, new, ["tests/test_oracle26.py"])


@pytest.mark.slow
@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, desc, old, new):
    _planted(tmp_path, desc, old, new, PINS)


def _planted(tmp_path, desc, old, new, pins):
    for d in ("oracle", "tests", "paper_2210_06438_amd"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path / "pytest.ini")
    src = tmp_path / "oracle" / "hydro_oracle.c"
    text = src.read_text()
    assert text.count(old) == 1, f"mutation site not unique: {old!r}"
    src.write_text(text.replace(old, new))
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", *pins],
                       cwd=tmp_path, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch: {desc}\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout, r.stdout[-2000:]
