"""Planted mistakes in the oracle (CPU only).

Each mutant below is oracle.c (or oracle/roadmap.py) with one plausible slip: a sign, a dropped term, a transposed
operand, a wrong index, an off-by-one or a non-strict comparison.  Every mutant must make at
least one of the oracle's pin tests fail (hand values, closed forms, brute force, invariants,
finite differences).  A mutant that passes all of them would mean the pins do not bind that
part of the oracle to the paper and the mathematics.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = [os.path.join(ROOT, "tests", f) for f in
        ("test_oracle_fk.py", "test_oracle_clearance.py", "test_oracle_validity.py",
         "test_oracle_cost.py")]

# (name, text of oracle.c, replacement); the text must occur exactly once.
MUTANTS = [
    # forward kinematics (Sec. III-B)
    ("dh_rotation_sign", "m[1] = -st * ca;", "m[1] = st * ca;"),
    ("dh_offset_d_dropped", "m[11] = d;", "m[11] = 0.0;"),
    ("dh_length_a_wrong_axis", "m[7] = a * st;", "m[7] = a * ct;"),
    ("dh_twist_sin_sign", "m[9] = sa;", "m[9] = -sa;"),
    ("mount_after_parent_swapped", "mat_mul(T[rb->parent_link[j]], M, P);",
     "mat_mul(M, T[rb->parent_link[j]], P);"),
    ("theta_offset_dropped", "dh_matrix(dh[0], dh[1], dh[2], dh[3], q[j] + dh[4], A);",
     "dh_matrix(dh[0], dh[1], dh[2], dh[3], q[j], A);"),
    ("prismatic_slides_along_x", "dh_matrix(dh[0], dh[1] + q[j], dh[2], dh[3], dh[4], A);",
     "dh_matrix(dh[0] + q[j], dh[1], dh[2], dh[3], dh[4], A);"),
    ("sphere_offset_rotated_by_transpose",
     "out[3 * s + i] = m[4 * i] * l[0] + m[4 * i + 1] * l[1] + m[4 * i + 2] * l[2] +",
     "out[3 * s + i] = m[i] * l[0] + m[4 + i] * l[1] + m[8 + i] * l[2] +"),
    # clearance to the primitives (Sec. III-C)
    ("sphere_radius_dropped", "return norm3(d) - prim[3];", "return norm3(d);"),
    ("capsule_parameter_unclamped",
     "    double t = uu > 0.0 ? dot3(w, u) / uu : 0.0;\n    if (t < 0.0) t = 0.0;\n"
     "    if (t > 1.0) t = 1.0;\n    double d[3]",
     "    double t = uu > 0.0 ? dot3(w, u) / uu : 0.0;\n    double d[3]"),
    ("cylinder_inside_sign", "return -(a < b ? a : b);", "return (a < b ? a : b);"),
    ("cylinder_height_radius_swapped",
     "const double *o = prim, *w = prim + 3;\n    double H = prim[6], R = prim[7];\n"
     "    double v[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};\n    double h = dot3(v, w);\n"
     "    double rad[3] = {v[0] - h * w[0], v[1] - h * w[1], v[2] - h * w[2]};\n"
     "    double rho = norm3(rad);\n    double ah",
     "const double *o = prim, *w = prim + 3;\n    double H = prim[7], R = prim[6];\n"
     "    double v[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};\n    double h = dot3(v, w);\n"
     "    double rad[3] = {v[0] - h * w[0], v[1] - h * w[1], v[2] - h * w[2]};\n"
     "    double rho = norm3(rad);\n    double ah"),
    ("box_rotation_not_transposed",
     "double pk = R[0 + k] * v[0] + R[3 + k] * v[1] + R[6 + k] * v[2];",
     "double pk = R[3 * k] * v[0] + R[3 * k + 1] * v[1] + R[3 * k + 2] * v[2];"),
    ("box_inside_term_dropped", "return sqrt(out2) + (mx < 0.0 ? mx : 0.0);",
     "return sqrt(out2);"),
    ("self_pair_one_radius_twice",
     "double cl = norm3(d) - rb->sphere_xyzr[4 * s + 3] - rb->sphere_xyzr[4 * t + 3];",
     "double cl = norm3(d) - 2.0 * rb->sphere_xyzr[4 * s + 3];"),
    ("self_pairs_skipped", "for (int p = 0; p < rb->n_pairs; ++p) {",
     "for (int p = 0; p < 0; ++p) {"),
    ("touching_counts_as_collision", "return isnan(cm) ? 1 : (cm < 0.0);",
     "return isnan(cm) ? 1 : (cm <= 0.0);"),
    ("touching_collides_in_batches", "if (jb->flag) jb->flag[i] = isnan(cm) ? 1 : (cm < 0.0);",
     "if (jb->flag) jb->flag[i] = isnan(cm) ? 1 : (cm <= 0.0);"),
    ("touching_collides_on_edges", "if (cm < 0.0) hit = 1;", "if (cm <= 0.0) hit = 1;"),
    ("non_finite_state_is_free",
     "const double *q) {\n    if (!all_finite(q, rb->dof)) return NAN;\n    double *c = (double *)"
     "malloc(sizeof(double) * 3 * (rb->n_spheres + 1));\n    orc_sphere_centres(rb, q, c);\n"
     "    double cmin",
     "const double *q) {\n    double *c = (double *)"
     "malloc(sizeof(double) * 3 * (rb->n_spheres + 1));\n    orc_sphere_centres(rb, q, c);\n"
     "    double cmin"),
    # edge discretisation and edge validity (Sec. III-D)
    ("edge_count_without_endpoint", "double n = ceil(L / res) + 1.0;",
     "double n = ceil(L / res);"),
    ("edge_length_sum_not_max", "if (d > L) L = d;", "L += d;"),
    ("edge_spacing_off_by_one", "double t = (double)k / (double)(n - 1);",
     "double t = (double)k / (double)n;"),
    ("non_finite_edge_is_free", "                jb->flag[i] = 1;\n",
     "                jb->flag[i] = 0;\n"),
    # squared-penetration cost and its gradient
    ("cost_penetration_not_squared",
     "double p = -orc_clearance(kind, c + 3 * s, r, prim_row(env, kind, i));\n"
     "                if (p > 0.0) C += p * p;",
     "double p = -orc_clearance(kind, c + 3 * s, r, prim_row(env, kind, i));\n"
     "                if (p > 0.0) C += p;"),
    ("cost_self_pairs_dropped", "        if (p > 0.0) C += p * p;\n    }\n    free(c);\n    return C;",
     "    }\n    free(c);\n    return C;"),
    ("gradient_env_force_sign", "f[3 * s + a] += -2.0 * p * g[a];",
     "f[3 * s + a] += 2.0 * p * g[a];"),
    ("gradient_self_force_sign", "f[3 * t + a] += 2.0 * p * d[a] / n;",
     "f[3 * t + a] += -2.0 * p * d[a] / n;"),
    ("jacobian_cross_product_reversed",
     "double jc[3] = {z[1] * v[2] - z[2] * v[1], z[2] * v[0] - z[0] * v[2],\n"
     "                            z[0] * v[1] - z[1] * v[0]};",
     "double jc[3] = {v[1] * z[2] - v[2] * z[1], v[2] * z[0] - v[0] * z[2],\n"
     "                            v[0] * z[1] - v[1] * z[0]};"),
    ("jacobian_moved_by_off_by_one", "if (lk == j + 1) return 1;", "if (lk == j) return 1;"),
    ("gradient_box_face_sign", "local[kmax] = p[kmax] >= 0.0 ? 1.0 : -1.0;",
     "local[kmax] = p[kmax] >= 0.0 ? -1.0 : 1.0;"),
]


# Planted mistakes in the Python half of the oracle (oracle/roadmap.py), checked against the
# roadmap pins.
ROADMAP = os.path.join(ROOT, "oracle", "roadmap.py")
ROADMAP_PINS = [os.path.join(ROOT, "tests", "test_oracle_roadmap.py")]
ROADMAP_MUTANTS = [
    ("knn_self_is_a_neighbour", "            s[np.arange(len(qb)), qb] = np.inf",
     "            pass"),
    ("knn_ties_to_higher_index", "np.lexsort((np.broadcast_to(np.arange(n), s.shape), s), axis=1)",
     "np.lexsort((np.broadcast_to(-np.arange(n), s.shape), s), axis=1)"),
    ("knn_non_finite_kept", "            order = np.where(np.isfinite(dd), order, -1)\n",
     ""),
    ("dist_abs_not_squared", "s = (s + (d * d).astype(np.float32)).astype(np.float32)",
     "s = (s + np.abs(d)).astype(np.float32)"),
    ("pairs_both_directions", "if i < j or i not in idx[j]:", "if True:"),
    ("pairs_mutual_dropped", "if i < j or i not in idx[j]:", "if i < j:"),
    # the FP64 definition
    ("exact_self_is_a_neighbour", "        s[i] = np.inf                               # a sample",
     "        pass                                        # a sample"),
    ("exact_ties_to_higher_index", "order = np.lexsort((np.arange(n), s))",
     "order = np.lexsort((-np.arange(n), s))"),
    ("exact_last_coordinate_dropped", "    for j in range(x.shape[1]):\n        d = x[:, j][:, None] - y[:, j][None, :]\n        s += d * d",
     "    for j in range(x.shape[1] - 1):\n        d = x[:, j][:, None] - y[:, j][None, :]\n        s += d * d"),
    ("exact_abs_not_squared", "        s += d * d\n", "        s += np.abs(d)\n"),
    ("exact_next_off_by_one", "            d2_next[r] = s[take[k]]", "            d2_next[r] = s[take[k - 1]]"),
    ("bound_too_tight", "return (1.0 + U32) ** (dim + 2) - 1.0", "return (1.0 + U32) ** dim - 1.0"),
]

# Loads a mutated roadmap.py in place of oracle.roadmap, then runs the given pin tests.
_ROADMAP_RUNNER = """
import importlib.util, sys
import pytest
sys.path.insert(0, {root!r})
import oracle
spec = importlib.util.spec_from_file_location("oracle.roadmap", {path!r})
mod = importlib.util.module_from_spec(spec)
spec.loader.exec_module(mod)
sys.modules["oracle.roadmap"] = mod
oracle.roadmap = mod
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *{pins!r}]))
"""


def _run_roadmap_mutant(tmp, name, old, new):
    src = open(ROADMAP).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur once in roadmap.py"
    path = os.path.join(tmp, f"roadmap_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    code = _ROADMAP_RUNNER.format(root=ROOT, path=path, pins=ROADMAP_PINS)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-1500:]


def _run_mutant(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur once in oracle.c"
    mdir = os.path.join(tmp, name)
    os.makedirs(mdir, exist_ok=True)
    csrc, lib = os.path.join(mdir, "oracle.c"), os.path.join(mdir, "liboracle.so")
    with open(csrc, "w") as f:
        f.write(src.replace(old, new))
    from oracle import oracle as O
    subprocess.check_call(["gcc", *O.CFLAGS, "-o", lib, csrc, "-lm"])
    env = dict(os.environ, VK_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-1500:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("mutants"))
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {m[0]: ex.submit(_run_mutant, tmp, *m) for m in MUTANTS}
        futs.update({m[0]: ex.submit(_run_roadmap_mutant, tmp, *m) for m in ROADMAP_MUTANTS})
        return {k: f.result() for k, f in futs.items()}


def test_unmutated_oracle_passes_its_pins(tmp_path):
    from oracle import oracle as O
    O.build(force=False)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-1500:]
    # the runner that swaps in a roadmap module passes with the module unchanged
    rc, tail = _run_roadmap_mutant(str(tmp_path), "none", "import numpy as np", "import numpy as np")
    assert rc == 0, tail


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS + ROADMAP_MUTANTS])
def test_pins_catch_planted_mistake(outcomes, name):
    rc, tail = outcomes[name]
    assert rc == 1, f"mutant {name} was not caught (pytest exit {rc}):\n{tail}"
