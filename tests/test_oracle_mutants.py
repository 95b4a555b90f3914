"""Mutation check of the oracle's pins (CPU only, no GPU).

Each mutant is a copy of the oracle's C sources with ONE plausible mistake
planted -- a dropped term, a wrong sign, index or height, a transposed
operand, a wrong neighbour -- built into a library of its own.  The pin tests
of test_oracle.py (brute force, the row DP, closed forms, library max-flow,
the certificate's acceptance of an independent preflow and its rejection of
planted mistakes) then run against it in a child process, and at least one
of them must fail.  The unmodified sources, built the same way, must pass.
So a mistake of any of these kinds in the graph of Section 1.2, in Dinic's
method (Section 2), in the cut and surface extraction (Eq. 6, Theorem 1.1),
in the soft smoothness term or in the certificate would not go unnoticed.

Mutants that cannot change any result (an arc whose capacity is zero, a
constraint that another arc already implies) are left out: no pin can tell
them apart from the oracle.  Each one that is left out is named at the end of
this file with the reason.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")
SOURCES = ("oracle.c", "certify.c")
PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle.py"),
             os.path.join(ROOT, "tests", "test_oracle_band.py")]

# (name, file, text in the source, its replacement); the text must occur
# exactly once in that file.
MUTANTS = [
    # --- graph of the cost volume (Section 1.2) ---------------------------
    ("base_offset_dropped", "oracle.c", "B += 1;", "B += 0;"),
    ("weight_operands_transposed", "oracle.c",
     "(int64_t)c[v] - (int64_t)c[v - 1]", "(int64_t)c[v - 1] - (int64_t)c[v]"),
    ("source_capacity_sign", "oracle.c",
     "if (w < 0) fn(ctx, s, v, -w);", "if (w < 0) fn(ctx, s, v, w);"),
    ("sink_arcs_from_wrong_node", "oracle.c",
     "if (w > 0) fn(ctx, v, t, w);", "if (w > 0) fn(ctx, v - (z > 0), t, w);"),
    ("down_arc_reversed", "oracle.c",
     "if (z >= 1) fn(ctx, v, v - 1, OR_INF);", "if (z >= 1) fn(ctx, v - 1, v, OR_INF);"),
    ("lateral_height_off_by_one", "oracle.c",
     "int64_t zt = z - delta < 0 ? 0 : z - delta;",
     "int64_t zt = z - delta - 1 < 0 ? 0 : z - delta - 1;"),
    ("neighbour_minus_y_missing", "oracle.c",
     "dy[4] = {0, 0, 1, -1};", "dy[4] = {0, 0, 1, 1};"),
    ("soft_arc_wrong_height", "oracle.c",
     "fn(ctx, v, node_id(qx, qy, z, ny, K), alpha);",
     "fn(ctx, v, node_id(qx, qy, z - 1, ny, K), alpha);"),
    ("soft_arc_double_capacity", "oracle.c",
     "fn(ctx, v, node_id(qx, qy, z, ny, K), alpha);",
     "fn(ctx, v, node_id(qx, qy, z, ny, K), 2 * alpha);"),
    # --- Dinic's method (Section 2) ----------------------------------------
    ("blocking_flow_keeps_reverse", "oracle.c",
     "g->res[g->rev[a]] += push;", "g->res[g->rev[a]] += 0 * push;"),
    ("flow_total_keeps_last_phase", "oracle.c",
     "out->flow += blocking_flow(g, s, t, level, cur, buf);",
     "out->flow = blocking_flow(g, s, t, level, cur, buf);"),
    # --- cuts, surfaces and energies (Eq. 6, Theorem 1.1, Eq. 1) -----------
    ("sink_side_search_forward", "oracle.c",
     "if (g->res[g->rev[a]] > 0 && !mark[u])", "if (g->res[a] > 0 && !mark[u])"),
    ("hmin_lowest_instead_of_highest", "oracle.c",
     "if (sreach[v]) lo = z;", "if (sreach[v] && lo < 0) lo = z;"),
    ("hmax_from_sink_side", "oracle.c",
     "if (!treach[v]) hi = z;", "if (treach[v]) hi = z;"),
    ("cut_counts_inner_arcs", "oracle.c",
     "if (g->fwd[a] && !sreach[g->head[a]]) {", "if (g->fwd[a] && sreach[g->head[a]]) {"),
    ("smooth_term_y_pairs_dropped", "oracle.c",
     "if (y + 1 < ny) sum += llabs(a - h[x * ny + y + 1]);",
     "if (y + 1 < ny) sum += 0 * llabs(a - h[x * ny + y + 1]);"),
    ("smooth_term_wrong_neighbour", "oracle.c",
     "if (x + 1 < nx) sum += llabs(a - h[(x + 1) * ny + y]);",
     "if (x + 1 < nx) sum += llabs(a - h[x * ny + y]);"),
    # --- certificate ---------------------------------------------------------
    ("cert_base_offset_dropped", "certify.c", "B += 1;", "B += 0;"),
    ("cert_sink_residual_sign", "certify.c",
     "if (e != src - (snk - r) + net[v])", "if (e != src - (snk + r) + net[v])"),
    ("cert_down_flow_direction", "certify.c",
     "if (z > 0) { net[v] -= fd; net[v - 1] += fd; }",
     "if (z > 0) { net[v] += fd; net[v - 1] -= fd; }"),
    ("cert_neighbour_order", "certify.c",
     "static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};",
     "static const int dx[4] = {0, 0, 1, -1}, dy[4] = {1, -1, 0, 0};"),
    ("cert_soft_capacity_unchecked", "certify.c",
     "if (f < 0 || f > alpha) out->bad_capacity++;", "if (f < 0) out->bad_capacity++;"),
    ("cert_soft_flow_ignored", "certify.c",
     "net[v] -= f; net[u] += f;\n                }\n            }",
     "(void)u;\n                }\n            }"),
    ("cert_cut_top_node_dropped", "certify.c",
     "if (z <= h && w > 0) out->cut += w;", "if (z < h && w > 0) out->cut += w;"),
    ("cert_soft_cut_dropped", "certify.c",
     "if (h > hq) out->cut += alpha * (h - hq);", "if (h > hq) out->cut += 0 * alpha * (h - hq);"),
    ("cert_soft_energy_wrong_pairs", "certify.c",
     "if (k == 0 || k == 2) out->energy", "if (k == 0 || k == 1) out->energy"),
    ("cert_reverse_down_residual_dropped", "certify.c",
     "if (z + 1 < K && flow_down[v + 1] > 0) VISIT(v + 1);",
     "if (z + 1 < K && flow_down[v + 1] < 0) VISIT(v + 1);"),
    ("cert_reverse_lateral_tail_height", "certify.c",
     "int64_t zt = z == 0 ? 0 : z + delta;", "int64_t zt = z == 0 ? 0 : z + delta + 1;"),
    ("cert_soft_residual_transposed", "certify.c",
     "alpha - flow_soft[(int64_t)k * N + v] + flow_soft[(int64_t)kk * N + u] > 0",
     "alpha + flow_soft[(int64_t)k * N + v] - flow_soft[(int64_t)kk * N + u] > 0"),
    ("cert_sink_reach_ignored", "certify.c",
     "if (sink_res[v] > 0) reached_sink = 1;", "if (sink_res[v] < 0) reached_sink = 1;"),
    ("cert_hmax_reverse_down_dropped", "certify.c",
     "if (z > 0 && flow_down[v] > 0) BACK(v - 1);", "if (0 && flow_down[v] > 0) BACK(v - 1);"),
    ("cert_hmax_lateral_tail_height", "certify.c",
     "const int64_t zq = z == 0 ? 0 : z + delta;", "const int64_t zq = z == 0 ? 0 : z + delta + 1;"),
    # --- narrow-band graphs (Section 3.4) --------------------------------------
    ("band_lower_rule_wrong_sign", "oracle.c",
     "if (lo[p] - delta > lo[q]) { lo[q] = lo[p] - delta; changed = 1; }",
     "if (lo[p] + delta > lo[q]) { lo[q] = lo[p] + delta; changed = 1; }"),
    ("band_upper_rule_dropped", "oracle.c",
     "if (hi[q] + delta < hi[p]) { hi[p] = hi[q] + delta; changed = 1; }",
     "if (0 && hi[q] + delta < hi[p]) { hi[p] = hi[q] + delta; changed = 1; }"),
    ("band_lateral_head_off_by_one", "oracle.c",
     "int64_t zq = z - b->delta < b->lo[q] ? b->lo[q] : z - b->delta;",
     "int64_t zq = z - b->delta + 1 < b->lo[q] ? b->lo[q] : z - b->delta + 1;"),
    ("band_cost_from_effective_bottom", "oracle.c",
     "const int32_t *cp = b->cost + p * b->K - b->off[p];",
     "const int32_t *cp = b->cost + p * b->K - b->lo[p];"),
    ("band_base_from_band_bottom", "oracle.c",
     "int64_t c0 = b->cost[p * b->K + b->lo[p] - b->off[p]];",
     "int64_t c0 = b->cost[p * b->K];"),
    ("band_hmin_lowest_instead_of_highest", "oracle.c",
     "if (sreach[v]) hl = z;", "if (sreach[v] && hl < 0) hl = z;"),
    ("band_energy_wrong_height", "oracle.c",
     "if (hl >= 0) out->energy += cost[p * K + hl - off[p]];",
     "if (hl >= 0) out->energy += cost[p * K + hl - lo[p]];"),
    ("cert_band_shift_reversed", "certify.c",
     "const int64_t sh = delta + lo[q] - lo[p];          /* arcs p -> q */",
     "const int64_t sh = delta + lo[p] - lo[q];          /* arcs p -> q */"),
    ("cert_band_reverse_tail_height", "certify.c",
     "const int64_t jq = j == 0 ? 0 : j + shq;", "const int64_t jq = j == 0 ? 0 : j + shq + 1;"),
    ("cert_band_base_offset_dropped", "certify.c", "Bb = Bb + 1;", "Bb = Bb + 0;"),
    ("cert_band_unused_slots_unchecked", "certify.c",
     "if (excess[v] != 0 || sink_res[v] != 0 || fdv != 0) out->bad_capacity++;",
     "if (0) out->bad_capacity++;"),
]

# The child process points the oracle package at the given library and runs
# the pin tests, stopping at the first failure.
_RUNNER = (
    "import sys\n"
    "import oracle\n"
    "oracle._LIB_PATH = sys.argv[1]\n"
    "import pytest\n"
    "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', *sys.argv[2:]]))\n"
)


def _build(dest_dir, mutant=None):
    os.makedirs(dest_dir)
    srcs = []
    for name in SOURCES:
        with open(os.path.join(ORACLE_DIR, name)) as f:
            text = f.read()
        if mutant is not None and mutant[1] == name:
            _, _, old, new = mutant
            assert text.count(old) == 1, f"{mutant[0]}: text not found exactly once in {name}"
            text = text.replace(old, new)
        path = os.path.join(dest_dir, name)
        with open(path, "w") as f:
            f.write(text)
        srcs.append(path)
    lib = os.path.join(dest_dir, "liboracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", lib, *srcs],
                   check=True, capture_output=True)
    return lib


def _pins_pass(lib):
    """True when every pin test passes against `lib`."""
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    try:
        r = subprocess.run([sys.executable, "-c", _RUNNER, lib, *PIN_TESTS], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=300)
    except subprocess.TimeoutExpired:
        return False, "pin tests did not finish within 300 s"
    return r.returncode == 0, r.stdout[-2000:]


@pytest.fixture(scope="module")
def build_root(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    return str(tmp_path_factory.mktemp("oracle_mutants"))


def test_unmodified_sources_pass_the_pins(build_root):
    ok, log = _pins_pass(_build(os.path.join(build_root, "control")))
    assert ok, log


def test_every_mutant_fails_a_pin(build_root):
    libs = [(m[0], _build(os.path.join(build_root, m[0]), m)) for m in MUTANTS]
    with ThreadPoolExecutor(max_workers=max(1, min(6, (os.cpu_count() or 2) - 1))) as pool:
        results = list(pool.map(lambda nl: (nl[0], _pins_pass(nl[1])), libs))
    survivors = [name for name, (ok, _) in results if ok]
    assert not survivors, f"mutants that every pin accepts: {survivors}"


# Mutants left out because they change no result:
#  - the down arc (p,1) -> (p,0) dropped: (p,0) has a source arc that can
#    never be saturated (no path from it reaches t without leaving its own
#    level), so it lies in every minimal cut with or without that arc;
#  - soft arcs also at z = 0: (p,0) -> (q,0) is already an infinite arc;
#  - the soft cut counted as alpha * max(0, h(q) - h(p)) instead of
#    alpha * max(0, h(p) - h(q)): the sum runs over both orders of every
#    neighbour pair, so both forms give the same total;
#  - Dinic's level check relaxed to any higher level, or the search restarted
#    from s after every augmentation: the paths found are still augmenting
#    paths and the loop still ends only when t is unreachable, so the flow is
#    still maximum (only the running time changes);
#  - the oracle's own conservation and capacity self-checks removed: they
#    report on a correct flow and change no returned value.
