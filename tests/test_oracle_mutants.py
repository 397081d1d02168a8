"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of oracle/oracle.c (a
dropped term, a wrong index or operand, an off-by-one, a non-strict
comparison), builds that copy,
and runs the pin suites (tests/test_oracle_pins.py, tests/test_oracle_dynamic.py)
against it in a child
process; at least one pin must fail. The oracle itself is never modified.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# name: (text of oracle.c, its replacement)
MUTANTS = {
    # Alg. 2 GG-Apply without the dangling-mass term
    "pr_apply_drops_dangling": ("xn = (1.0 - d) / n + d * (sum + D / n);", "xn = (1.0 - d) / n + d * (sum);"),
    # Alg. 2 GG-Gather without the division by the out-degree
    "pr_gather_no_outdeg": ("sum += r->pr_x[v] / deg[v];", "sum += r->pr_x[v];"),
    # PREFIX influence over the running sum before the edge's own contribution
    "pr_prefix_exclusive": ("        P += c;\n        double influence;",
                            "        double influence;\n        P += 0.0;"),
    # SSSP relaxation with an off-by-one weight
    "sssp_weight_off_by_one": ("const uint64_t cand = (uint64_t)xv + (uint64_t)g->weight[e];\n      if (cand < best)",
                               "const uint64_t cand = (uint64_t)xv + (uint64_t)g->weight[e] + 1u;\n      if (cand < best)"),
    # CC gather reading the destination's label instead of the source's
    "cc_reads_destination": ("      const int32_t xv = r->l_x[g->col[e]];\n      if (xv < best) best = xv;",
                             "      const int32_t xv = r->l_x[u];\n      if (xv < best) best = xv;"),
    # GG schedule with the wrong period
    "gg_period_off_by_one": ("if (!p->decoupled) return i % (p->alpha + 1) == 0;",
                             "if (!p->decoupled) return i % (p->alpha + 2) == 0;"),
    # the NONE dangling reading still spreading the dangling mass
    "dangling_none_ignored": ("  if (r->app.dangling == GGO_DANGLING_UNIFORM)\n    for (int32_t v = 0; v < n; ++v)\n      if (deg[v] == 0)",
                              "  if (1)\n    for (int32_t v = 0; v < n; ++v)\n      if (deg[v] == 0)"),
    # TOTAL influence taken over the running sum (the PREFIX reading)
    "total_uses_running_sum": ("influence = rowsum32 > 0.0 ? c / rowsum32 : 0.0;",
                               "influence = P > 0.0 ? c / P : 0.0;"),
    # ACTIVE degree with the dangling set of the full graph
    "active_degree_full_dangling_set": ("      if (deg[v] == 0) D += r->pr_x[v];",
                                        "      if (r->outdeg[v] == 0) D += r->pr_x[v];"),
    # ACTIVE degree counted over every out-edge instead of the active ones
    "active_degree_counts_all_edges": ("        if (r->active[e]) r->odeg_act[r->g.col[e]]++;",
                                       "        r->odeg_act[r->g.col[e]]++;"),
    # decoupled schedule: first superstep one iteration early
    "decoupled_first_off_by_one": ("  const int32_t first = p->alpha0 + 1;", "  const int32_t first = p->alpha0;"),
    # decoupled schedule: theta0 never used
    "decoupled_theta0_ignored": ("return (p->decoupled && i == p->alpha0 + 1) ? p->theta0 : p->theta;",
                                 "return p->theta;"),
    # GG-VStatus: the destination's status instead of the source's
    "vstatus_reads_destination": ("any = r->active[e] && r->vact[r->g.col[e]];", "any = r->active[e] && r->vact[u];"),
    # GG-VStatus: non-strict comparison with epsilon
    "vstatus_not_strict": ("r->vact[u] = (uint8_t)(delta > bound);", "r->vact[u] = (uint8_t)(delta >= bound);"),
    # SSSP EStatus: improvement measured against the new minimum instead of the old one
    "sssp_estatus_wrong_denominator": ("flag = ((run - nw) << 16) > theta_q * run;",
                                       "flag = ((run - nw) << 16) > theta_q * nw;"),
    # SSSP EStatus deactivating the arcs of unreached sources
    "sssp_unreached_deactivated": ("if (xv == GGO_INF_U32) continue; /* not assessable: keeps its flag */",
                                   "if (xv == GGO_INF_U32) { r->active[e] = 0; continue; }"),
    # EStatus with >= instead of the strict > of Alg. 2
    "estatus_not_strict": ("const int flag = r->infl[e] > r->theta_now;",
                           "const int flag = r->infl[e] >= r->theta_now;"),
    # PPR teleporting to every vertex instead of the source
    "ppr_teleport_everywhere": ("xn = (u == s ? (1.0 - d) : 0.0) + d * (sum + (u == s ? D : 0.0));",
                                "xn = (1.0 - d) / n + d * (sum + (u == s ? D : 0.0));"),
    # CC influence relative to the row's first label only (running minimum never updated)
    "cc_influence_no_running_min": ("        r->infl[e] = xv < run ? 1.0 : 0.0;\n        if (xv < run) run = xv;",
                                    "        r->infl[e] = xv < run ? 1.0 : 0.0;"),
    # BP message without the factor of the log-ratio (half the log-ratio)
    "bp_message_half": ("  return log(m1) - log(m0);", "  return 0.5 * (log(m1) - log(m0));"),
    # BP message with the potential's two entries swapped (anti-ferromagnetic)
    "bp_psi_swapped": ("const double m1 = same * b1 + diff * b0;", "const double m1 = diff * b1 + same * b0;"),
    # BP update without the vertex's own prior
    "bp_prior_dropped": ("const double xn = r->app.prior[u] + sum;", "const double xn = sum;"),
    # BP influence on signed values instead of magnitudes
    "bp_influence_signed": ("r->infl[e] = fabs(P) > 0.0 ? fabs(c) / fabs(P) : 0.0;",
                            "r->infl[e] = P > 0.0 ? c / P : 0.0;"),
    # SSSP push-order influence starting at INF (the PREFIX reading) in EStatus
    "push_sssp_starts_at_inf": ("    if (r->mode[u] != ROW_SUPER) continue;\n"
                                "    uint64_t run = r->pol.influence == GGO_INFL_PUSH ? r->d_x[u] : GGO_INF_U32;",
                                "    if (r->mode[u] != ROW_SUPER) continue;\n    uint64_t run = GGO_INF_U32;"),
    # CC push-order influence starting at INF
    "push_cc_starts_at_inf": ("int64_t run = r->pol.influence == GGO_INFL_PUSH ? (int64_t)r->l_x[u] : INT64_MAX;",
                              "int64_t run = INT64_MAX;"),
    # dynamic update: the taint closure never grows beyond its seeds
    "update_no_closure": ("      int grew = 1;\n      while (grew) {", "      int grew = 0;\n      while (grew) {"),
    # dynamic update: every deleted arc seeds, supporting or not
    "update_seed_ignores_support": ("if (deleted_old[e] && supports(r, r->g.col[e], u, r->g.weight ? r->g.weight[e] : 0))",
                                    "if (deleted_old[e])"),
    # dynamic update: inserted arcs start inactive
    "update_inserted_inactive": ("act[e] = old_of_new[e] >= 0 ? r->active[old_of_new[e]] : 1;",
                                 "act[e] = old_of_new[e] >= 0 ? r->active[old_of_new[e]] : 0;"),
    # dynamic update: out-degrees of the old graph kept
    "update_stale_outdeg": ("  memset(r->outdeg, 0, sizeof(int32_t) * ((size_t)n + 1));\n"
                            "  for (int64_t e = 0; e < m1; ++e) r->outdeg[gn->col[e]]++;", ""),
}


def run_pins_against(tmp_path, src):
    """Build `src` as an oracle library in tmp_path and run the pin suite
    against it in a child process; returns pytest's exit code."""
    with open(tmp_path / "oracle.c", "w") as f:
        f.write(src)
    shutil.copy(os.path.join(ORACLE, "oracle.h"), tmp_path / "oracle.h")
    lib = str(tmp_path / "liboracle_copy.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", lib, str(tmp_path / "oracle.c"), "-lm"])
    env = dict(os.environ, GGO_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_dynamic.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout


def oracle_source():
    with open(os.path.join(ORACLE, "oracle.c")) as f:
        return f.read()


def test_unmodified_copy_passes_the_pins(tmp_path):
    code, out = run_pins_against(tmp_path, oracle_source())
    assert code == 0, out[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle_source()
    assert src.count(old) == 1, "the mutant's target text must occur exactly once"
    code, out = run_pins_against(tmp_path, src.replace(old, new))
    # exit code 1: tests ran and at least one failed (not a crash or an error)
    assert code == 1, "no pin failed for mutant %s:\n%s" % (name, out[-2000:])
