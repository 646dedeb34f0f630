"""Mutation check of the oracles' pins (CPU, no GPU).

Each entry below plants one plausible mistake (a dropped term, a wrong sign,
index, factor or rounding direction, a transposed operand) in a temporary copy
of the oracle outside the source tree, then runs the pin suites against that
copy: at least one pin must fail.  An unmodified copy must pass, so a failure
comes from the planted mistake and not from the harness.  The tree's own
oracle is never modified.
"""
import os
import re
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = "tests/test_oracle_pins.py"
SURR = "tests/test_oracle_surrogate.py"
CPP = "oracle/oracle.cpp"
PY = "oracle/__init__.py"
SPY = "oracle/surrogate.py"

# (name, file, original text, planted text, pin suite)
MUTANTS = [
    # O1 / O4: condensation
    ("cell_merge_drops_A_mass", CPP, "o.cells.back().cA += c.cA;", "o.cells.back().cA += 0;", PINS),
    ("snap_rounds_to_nearest", CPP, "I[k] = (int64_t)std::floor(x);", "I[k] = (int64_t)std::nearbyint(x);", PINS),
    # O2: RWMD
    ("rwmd_without_diagonal_arc", CPP, "double best = 0.5 * (d - b);  // arc to the diagonal node",
     "double best = 1e300;", PINS),
    ("rwmd_min_of_the_sides", CPP, "o.L = std::max(o.LA, o.LB);", "o.L = std::min(o.LA, o.LB);", PINS),
    ("rwmd_fixed_point_rounds_up", CPP, "S += (int64_t)std::floor(std::ldexp(x, F));",
     "S += (int64_t)std::ceil(std::ldexp(x, F));", PINS),
    ("rwmd_scan_stops_early", CPP, "for (size_t r = k; r < other.size() && other[r].b - b < best; ++r)",
     "for (size_t r = k; r < other.size() && other[r].b - b < 0.5 * best; ++r)", PINS),
    # O3: error budget
    ("grid_twice_too_coarse", CPP, "double gmax = ((2.0 * eps_c) * L) / (double)n;",
     "double gmax = ((4.0 * eps_c) * L) / (double)n;", PINS),
    # (a start below the smallest valid s is repaired by the search upwards,
    # so the mistake that matters is a start above it)
    ("s_from_a_different_stretch", CPP, "int s = (int)std::ceil(2.0 + 4.0 / tau);",
     "int s = (int)std::ceil(4.0 + 8.0 / tau);", PINS),
    ("paper_grid_from_s_minus_2", CPP, "o.eps_c = s_override >= 12 ? 8.0 / (double)(s_override - 4) : 1.0;",
     "o.eps_c = s_override >= 12 ? 8.0 / (double)(s_override - 2) : 1.0;", PINS),
    # O6 / O7: tree and WSPD
    ("tree_box_from_left_child", CPP, "nd.maxj = std::max(o.nodes[l].maxj, o.nodes[r].maxj);",
     "nd.maxj = o.nodes[l].maxj;", PINS),
    ("separation_by_s_minus_one", CPP, "if (dist >= (int64_t)o.s * dmax) {",
     "if (dist >= (int64_t)(o.s - 1) * dmax) {", PINS),
    # O8: network
    ("cell_cost_without_factor_two", CPP, ": 2 * std::max(std::llabs(o.cells[u].i",
     ": std::max(std::llabs(o.cells[u].i", PINS),
    ("diagonal_cost_off_by_one", CPP, "int64_t dd = o.cells[(size_t)c].j - o.cells[(size_t)c].i;",
     "int64_t dd = o.cells[(size_t)c].j - o.cells[(size_t)c].i + 1;", PINS),
    ("B_to_A_arc_costs_one", CPP, "arcs->push_back({N + 1, N, 0});", "arcs->push_back({N + 1, N, 1});", PINS),
    # O9 / O10: flow and output
    ("residual_cost_sign", CPP, "E.push_back({a, 0, -cost});", "E.push_back({a, 0, cost});", PINS),
    ("w1_without_condensation_term", CPP, "o.W1 = std::ldexp((double)(o.flow_cost + o.n), o.e - 1);",
     "o.W1 = std::ldexp((double)(o.flow_cost), o.e - 1);", PINS),
    # O7': pruning
    ("prune_half_the_distance", CPP, "return 2 * dist >= (a.maxj - a.mini) + (b.maxj - b.mini);",
     "return 4 * dist >= (a.maxj - a.mini) + (b.maxj - b.mini);", PINS),
    # Euclidean metric
    ("l2_rwmd_squared_distance", CPP, "return std::min(std::sqrt(q), (d - b) * R_SQRT1_2);",
     "return std::min(q, (d - b) * R_SQRT1_2);", PINS),
    ("l2_grid_without_sqrt2", CPP, "if (l2) gmax = gmax * R_SQRT1_2;", "if (l2) gmax = gmax * 1.0;", PINS),
    ("l2_separation_by_s_not_s2", CPP, "if (dist2 >= (__int128)o.s * o.s * std::max(da, db)) {",
     "if (dist2 >= (__int128)o.s * std::max(da, db)) {", PINS),
    ("l2_cost_rounded_down", CPP,
     "return (int64_t)std::ceil(std::ldexp(std::sqrt((double)(di * di + dj * dj)), K));",
     "return (int64_t)std::floor(std::ldexp(std::sqrt((double)(di * di + dj * dj)), K));", PINS),
    ("l2_diagonal_cost_without_sqrt2", CPP,
     "return (int64_t)std::ceil(std::ldexp((double)di_dj * R_SQRT1_2, K));",
     "return (int64_t)std::ceil(std::ldexp((double)di_dj * 0.5, K));", PINS),
    ("l2_w1_linf_condensation_term", CPP, "o.W1 = o.W1_paper + (double)o.n * std::ldexp(R_SQRT1_2, o.e);",
     "o.W1 = o.W1_paper + (double)o.n * std::ldexp(0.5, o.e);", PINS),
    # exact W1 by Hungarian matching (Python side)
    ("hungarian_full_persistence_to_diagonal", PY, "else 0.5 * (P[:, 1] - P[:, 0])",
     "else (P[:, 1] - P[:, 0])", PINS),
    ("hungarian_l1_ground_metric", PY, "np.maximum(np.abs(db), np.abs(dd))", "(np.abs(db) + np.abs(dd))", PINS),
    # learned form: forward, loss gradient and backward
    ("surrogate_grad_without_factor_two", SPY, "g = 2.0 * rel / (w[j] * nP) / pred * diff",
     "g = rel / (w[j] * nP) / pred * diff", SURR),
    ("surrogate_grad_sign_of_second", SPY, "demb[pb[j]] -= g", "demb[pb[j]] += g", SURR),
    ("surrogate_backward_W2_transposed", SPY, "dh1 = dz2 @ W2", "dh1 = dz2 @ W2.T", SURR),
    ("surrogate_backward_no_relu_mask", SPY, "dz1 = dh1 * (h1 > 0.0)", "dz1 = dh1", SURR),
    # the WCD lower bound
    ("wcd_not_halved", SPY, "return 0.5 * float(np.hypot(d[0], d[1]) if l2 else np.abs(d).max())",
     "return float(np.hypot(d[0], d[1]) if l2 else np.abs(d).max())", SURR),
    ("wcd_projection_to_birth", SPY, "proj = lambda X: np.repeat(((X[:, 0] + X[:, 1]) * 0.5)[:, None], 2, axis=1)",
     "proj = lambda X: np.repeat(X[:, :1], 2, axis=1)", SURR),
]


def _copy_tree(dst):
    def ignore(_d, names):
        return [n for n in names if n == "__pycache__" or n.endswith(".so") or n.startswith(".")]

    for d in ("oracle", "pdsynth"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d), ignore=ignore)
    os.makedirs(os.path.join(dst, "tests", "golden"))
    for f in ("conftest.py", os.path.basename(PINS), os.path.basename(SURR)):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))
    g = os.path.join(ROOT, "tests", "golden")
    for f in os.listdir(g):
        if f.endswith(".json"):
            shutil.copy(os.path.join(g, f), os.path.join(dst, "tests", "golden", f))


def _run(mutant, workdir):
    name, path, old, new, suite = mutant
    d = os.path.join(workdir, name)
    _copy_tree(d)
    if old is not None:
        p = os.path.join(d, path)
        src = open(p).read()
        assert src.count(old) == 1, f"{name}: the original text must occur once in {path}"
        with open(p, "w") as f:
            f.write(src.replace(old, new))
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", suite],
                       cwd=d, env=env, capture_output=True, text=True, timeout=600)
    failed = re.findall(r"^FAILED (\S+)", r.stdout, flags=re.M)
    return name, r.returncode, failed, r.stdout[-3000:] + r.stderr[-2000:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    for name, path, old, _new, _suite in MUTANTS:
        assert open(os.path.join(ROOT, path)).read().count(old) == 1, name
    controls = [("control_pins", CPP, None, None, PINS), ("control_surrogate", SPY, None, None, SURR)]
    with tempfile.TemporaryDirectory() as work:
        with ThreadPoolExecutor(max_workers=max(1, min(8, (os.cpu_count() or 2) - 1))) as ex:
            results = list(ex.map(lambda m: _run(m, work), controls + MUTANTS))
    report, missed = {}, []
    for name, rc, failed, tail in results:
        if name.startswith("control"):
            assert rc == 0, f"{name} should pass unmodified:\n{tail}"
        elif rc == 1 and failed:
            # exit status 1: tests ran and at least one pin failed (not an
            # import error, a crash or a usage error)
            report[name] = failed[0]
        else:
            missed.append(f"{name} (rc {rc}):\n{tail}")
    assert not missed, "planted mistakes not caught:\n" + "\n".join(missed)
    assert len(report) == len(MUTANTS)
    print("\n".join(f"{k}: {v}" for k, v in report.items()))
