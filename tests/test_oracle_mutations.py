"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in a copy of the oracle (a transposed rotation, a dropped factor, a flipped
sign, a loosened inequality, a wrong constant of the paper's formulas) and
runs the pin tests against that copy in a separate process: the run must
fail.  The repository's own oracle is never modified."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FWD_BWD = ["tests/test_oracle_forward.py", "tests/test_oracle_backward.py"]

# (name, oracle file, text, planted text, pin test files)
MUTATIONS = [
    ("rotation transposed (eq. 3-6 / quaternion R)", "oracle/erbf.py",
     "    return R\n\n\ndef quat_rot_jacobian", "    return np.transpose(R, (0, 2, 1))\n\n\ndef quat_rot_jacobian",
     FWD_BWD),
    ("offset rotated by R^T instead of R", "oracle/erbf.py",
     "u = [R[k, 0] * dx + R[k, 1] * dy + R[k, 2] * dz for k in range(3)]",
     "u = [R[0, k] * dx + R[1, k] * dy + R[2, k] * dz for k in range(3)]", FWD_BWD),
    ("centre gradient loses its factor 2", "oracle/erbf.py",
     "gc = 2.0 * a[:, None]", "gc = 1.0 * a[:, None]", FWD_BWD),
    ("scale gradient sign flipped", "oracle/erbf.py", "gs = -2.0 * a", "gs = 2.0 * a", FWD_BWD),
    ("quaternion Jacobian sign flipped", "oracle/erbf.py",
     "J[:, 0] = np.stack([np.stack([o, -2 * z, 2 * y], -1),",
     "J[:, 0] = np.stack([np.stack([o, 2 * z, 2 * y], -1),", FWD_BWD),
    ("id1 mask inequality loosened (eq. 3-18)", "oracle/erbf.py",
     "id1 = (t <= tau1) & (fl > tau1)", "id1 = (t < tau1) & (fl > tau1)", FWD_BWD),
    ("eq. 3-21 terms swapped", "oracle/erbf.py",
     "num = float(np.sum((g1 - g2) * g1))", "num = float(np.sum((g2 - g1) * g2))", FWD_BWD),
    ("seeded scale halved (eq. 3-24)", "oracle/erbf.py",
     "d = np.sqrt(np.log(np.abs(ev) / eps)) / dbar", "d = np.sqrt(np.log(np.abs(ev) / eps)) / dbar / 2", FWD_BWD),
    ("target width h uses |m| (eq. 3-10)", "oracle/erbf.py",
     "h = math.log(2.0) / (m * m)", "h = math.log(2.0) / abs(m)", FWD_BWD),
    ("cull radius widened by 1% (eq. 3-15-1)", "oracle/erbf.py",
     "phi = np.where(dx * dx + dy * dy + dz * dz < r2, phi, 0.0)\n            f[",
     "phi = np.where(dx * dx + dy * dy + dz * dz < 1.01*r2, phi, 0.0)\n            f[", FWD_BWD),
    ("octree threshold halved", "oracle/erbf.py",
     "<= math.sqrt(3.0) / n", "<= math.sqrt(3.0) / (2 * n)", ["tests/test_oracle_forward.py"]),
    ("sample label 0.9 instead of 1", "oracle/erbf.py",
     "        return np.ones(self.cap)", "        return np.full(self.cap, 0.9)", ["tests/test_oracle_samples.py"]),
    ("Hausdorff distance from a mean", "oracle/metrics.py",
     "hd = max(d_tr.max(), d_rt.max())", "hd = max(d_tr.mean(), d_rt.max())", ["tests/test_oracle_metrics.py"]),
    ("Chamfer distance weights", "oracle/metrics.py",
     "cd = 0.5 * d_tr.mean() + 0.5 * d_rt.mean()", "cd = d_tr.mean() + 0.5 * d_rt.mean()",
     ["tests/test_oracle_metrics.py"]),
    ("area sampling without the square root", "oracle/metrics.py",
     "r1 = np.sqrt(u[:, 1])[:, None]", "r1 = u[:, 1][:, None]", ["tests/test_oracle_metrics.py"]),
    ("edge interpolation from the wrong corner", "oracle/metrics.py",
     "t = (iso - v[a]) / (v[b] - v[a])", "t = (iso - v[b]) / (v[a] - v[b])", ["tests/test_oracle_metrics.py"]),
    ("inscribed-sphere scale loses its factor 2 (eq. 3-12)", "oracle/erbf.py",
     "d = 2.0 * np.sqrt(-np.log(gamma / (w * w))) / dhat", "d = np.sqrt(-np.log(gamma / (w * w))) / dhat",
     ["tests/test_oracle_forward.py"]),
    ("covered points kept by the greedy init (Algorithm 1)", "oracle/erbf.py",
     "alive[cand[d2 <= R2[k]]] = False", "alive[cand[d2 < 0.25 * R2[k]]] = False", ["tests/test_oracle_forward.py"]),
    ("effective basis count uses > (eq. add_activate)", "oracle/schedule.py",
     "np.abs(np.asarray(w, np.float64)) >= tau_d", "np.abs(np.asarray(w, np.float64)) > tau_d",
     ["tests/test_oracle_schedule.py"]),
    ("L1 switched on by a rising spread (Algorithm 3)", "oracle/schedule.py",
     "float(np.std(s.l2_hist)) < cfg.tau_l2", "float(np.std(s.l2_hist)) > cfg.tau_l2",
     ["tests/test_oracle_schedule.py"]),
    ("final-phase cosine with the wrong sign", "oracle/schedule.py",
     "(1.0 + math.cos(math.pi * frac))", "(1.0 - math.cos(math.pi * frac))", ["tests/test_oracle_schedule.py"]),
    ("Euler angles composed in the reverse order (eq. 3-6)", "oracle/erbf.py",
     "    return Rz @ Ry @ Rx\n", "    return Rx @ Ry @ Rz\n", FWD_BWD),
    ("seeding keeps points that are not local maxima (Algorithm 2)", "oracle/erbf.py",
     "if sel.any() and absE[g] < absE[gl[sel]].max():", "if sel.any() and absE[g] < absE[gl[sel]].max() and False:",
     FWD_BWD),
    ("m taken over the first level only (eq. 3-10)", "oracle/erbf.py",
     "return float(min(np.min(np.asarray(S, dtype=np.float64)) for S in S_levels))",
     "return float(np.min(np.asarray(S_levels[0], dtype=np.float64)))", FWD_BWD),
    ("targets lose their factor 2 (eq. 3-10)", "oracle/erbf.py",
     "return 2.0 * np.exp(-h * (S - m) ** 2)", "return np.exp(-h * (S - m) ** 2)", FWD_BWD),
    ("L1 of signed weights (eq. 3-14_2)", "oracle/erbf.py",
     "L1 = float(np.sum(np.abs(K.w)))", "L1 = float(np.sum(K.w))", FWD_BWD),
    ("Adam bias correction off by one step", "oracle/erbf.py",
     "mhat = m1 / (1 - b1 ** t)", "mhat = m1 / (1 - b1 ** (t + 1))", FWD_BWD),
    ("quaternion gradient without the tangent projection", "oracle/erbf.py",
     "proj = gqhat - K.qhat * np.sum(K.qhat * gqhat, axis=1, keepdims=True)", "proj = gqhat", FWD_BWD),
    ("a tetrahedron of the cube split replaced", "oracle/metrics.py",
     "(0, 4, 5, 7), (0, 5, 1, 7))", "(0, 4, 5, 7), (0, 5, 4, 7))", ["tests/test_oracle_metrics.py"]),
    ("mini-batch mask offset by one level's base", "oracle/erbf.py",
     "sel = batch[(batch >= base) & (batch < base + lv.npts)] - base",
     "sel = batch[(batch >= base) & (batch < base + lv.npts)] - base // 2", FWD_BWD),
    ("L1 gradient beta * w in place of beta * sign(w) (eq. 3-15-2)", "oracle/erbf.py",
     "alpha * gr.w + beta * sign(w)", "alpha * gr.w + beta * w", FWD_BWD),
    ("centre gradient without alpha (eq. 3-15-2)", "oracle/erbf.py",
     "alpha * gr.c, alpha * gr.s", "gr.c, alpha * gr.s", FWD_BWD),
    ("samples do not suppress in the extreme-point test (Algorithm 2)", "oracle/erbf.py",
     "if ok and P_ida.shape[0]:", "if ok and P_ida.shape[0] and False:", ["tests/test_oracle_samples.py"]),
    ("dbar from |S| although samples are registered (eq. 3-24)", "oracle/erbf.py",
     "        if P_all.shape[0]:\n            dist =", "        if False:\n            dist =",
     ["tests/test_oracle_samples.py"]),
    ("samples taken as seeding candidates (Algorithm 2)", "oracle/erbf.py",
     "gcand = gid[is_grid[gid]]", "gcand = gid", ["tests/test_oracle_samples.py"]),
]


def _copy_tree(dst):
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("__pycache__", "*.pyc", "test_oracle_mutations.py"))


def _run(dst, files):
    env = dict(os.environ)
    env["PYTHONDONTWRITEBYTECODE"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *files], cwd=dst, capture_output=True, text=True, env=env, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def pristine(tmp_path_factory):
    dst = str(tmp_path_factory.mktemp("oracle_copy"))
    _copy_tree(dst)
    files = sorted({f for m in MUTATIONS for f in m[4]})
    rc, out = _run(dst, files)
    assert rc == 0, "the unmodified copy must pass its pins:\n" + out
    return dst


@pytest.mark.parametrize("name,path,text,planted,files", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(pristine, tmp_path, name, path, text, planted, files):
    dst = str(tmp_path / "copy")
    shutil.copytree(pristine, dst)
    target = os.path.join(dst, path)
    src = open(target).read()
    assert src.count(text) >= 1, f"{name}: the text to replace is gone from {path}"
    open(target, "w").write(src.replace(text, planted, 1))
    rc, out = _run(dst, files)
    assert rc != 0, f"{name}: no pin failed\n{out}"
