"""The oracle's pins catch plausible mistakes: each case copies the oracle (and the seeded input
generator) into a scratch folder, plants one slip in one line of the copy, and runs the pin
tests there, which must fail; the unchanged copy must pass.  Nothing outside the scratch folder
is touched, and the GPU path is not involved."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (label, oracle file, line as written, planted slip, pin file)
MUTATIONS = [
    ("Naik hop of length 1", "oracle/dslash.py",
     "w += _matvec(n_mu, np.roll(vf, -3, ax))", "w += _matvec(n_mu, np.roll(vf, -1, ax))",
     "test_oracle_pins.py"),
    ("backward fat link taken at x", "oracle/dslash.py",
     "w -= _matvec(_dag(np.roll(x_mu, 1, ax)), np.roll(vf, 1, ax))",
     "w -= _matvec(_dag(x_mu), np.roll(vf, 1, ax))", "test_oracle_pins.py"),
    ("backward Naik link without dagger", "oracle/dslash.py",
     "w -= _matvec(_dag(np.roll(n_mu, 3, ax)), np.roll(vf, 3, ax))",
     "w -= _matvec(np.roll(n_mu, 3, ax), np.roll(vf, 3, ax))", "test_oracle_pins.py"),
    ("backward Naik link taken at x - mu", "oracle/dslash.py",
     "w -= _matvec(_dag(np.roll(n_mu, 3, ax)), np.roll(vf, 3, ax))",
     "w -= _matvec(_dag(np.roll(n_mu, 1, ax)), np.roll(vf, 3, ax))", "test_oracle_pins.py"),
    ("backward hop sign flipped", "oracle/dslash.py",
     "w -= _matvec(_dag(np.roll(x_mu, 1, ax)), np.roll(vf, 1, ax))",
     "w += _matvec(_dag(np.roll(x_mu, 1, ax)), np.roll(vf, 1, ax))", "test_oracle_pins.py"),
    ("x and y axes swapped", "oracle/dslash.py",
     "_AXIS = (3, 2, 1, 0)", "_AXIS = (2, 3, 1, 0)", "test_oracle_pins.py"),
    ("links applied transposed", "oracle/dslash.py",
     'return np.einsum("...ab,...b->...a", a, v)', 'return np.einsum("...ba,...b->...a", a, v)',
     "test_oracle_pins.py"),
    ("Naik term dropped", "oracle/dslash.py",
     "w += _matvec(n_mu, np.roll(vf, -3, ax))", "pass", "test_oracle_pins.py"),
    ("mass squared taken as mass", "oracle/dslash.py",
     "return mass * mass * np.asarray(v) - dslash_half(fat, naik, t, dims, 0)",
     "return mass * np.asarray(v) - dslash_half(fat, naik, t, dims, 0)", "test_oracle_pins.py"),
    ("CG beta inverted", "oracle/cg.py",
     "beta = rho_new / rho", "beta = rho / rho_new", "test_oracle_pins.py"),
    ("flexible CG beta sign flipped", "oracle/cg.py",
     "beta = -_dot(q, z) / pq", "beta = _dot(q, z) / pq", "test_oracle_fcg.py"),
    ("flexible CG step with swapped inner product", "oracle/cg.py",
     "alpha = _dot(p, r) / pq", "alpha = _dot(r, p) / pq", "test_oracle_fcg.py"),
    ("flexible CG truncation dropped", "oracle/cg.py",
     "p = z + beta * p", "p = z", "test_oracle_fcg.py"),
    ("Adam without bias correction", "oracle/nn.py",
     "mhat = m / (1 - b1 ** t)", "mhat = m", "test_oracle_nn.py"),
    ("Adam second moment on the complex modulus", "oracle/nn.py",
     "v = b2 * v + (1 - b2) * gr * gr",
     "v = b2 * v + (1 - b2) * np.concatenate([np.abs(g) ** 2, np.abs(g) ** 2])", "test_oracle_nn.py"),
    ("Adam betas swapped", "oracle/nn.py",
     "m = b1 * m + (1 - b1) * gr", "m = b2 * m + (1 - b2) * gr", "test_oracle_nn.py"),
]


def _scratch(tmp_path, pin_file):
    shutil.copytree(os.path.join(ROOT, "oracle"), tmp_path / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "synth"), tmp_path / "synth",
                    ignore=shutil.ignore_patterns("__pycache__"))
    (tmp_path / "tests").mkdir()
    for f in ("conftest.py", pin_file):
        shutil.copy(os.path.join(ROOT, "tests", f), tmp_path / "tests" / f)
    if os.path.isdir(os.path.join(ROOT, "tests", "golden")):
        shutil.copytree(os.path.join(ROOT, "tests", "golden"), tmp_path / "tests" / "golden")


def _run(tmp_path, pin_file):
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    # a slip that stops a solver from converging shows up as a pin running out of time
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           "--timeout", "20", "-m", "not gpu", os.path.join("tests", pin_file)],
                          cwd=tmp_path, env=env, capture_output=True, text=True, timeout=900)


@pytest.mark.parametrize("pin_file", ["test_oracle_pins.py", "test_oracle_fcg.py", "test_oracle_nn.py"])
def test_unchanged_copy_passes(tmp_path, pin_file):
    _scratch(tmp_path, pin_file)
    res = _run(tmp_path, pin_file)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]


@pytest.mark.parametrize("label,path,line,slip,pin_file", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_slip_fails_a_pin(tmp_path, label, path, line, slip, pin_file):
    _scratch(tmp_path, pin_file)
    target = tmp_path / path
    src = target.read_text()
    assert src.count(line) == 1, f"{label}: the line to change is not unique in {path}"
    target.write_text(src.replace(line, slip))
    res = _run(tmp_path, pin_file)
    assert res.returncode != 0, f"{label}: the pins did not notice\n" + res.stdout[-2000:]
