"""The paper's Table tab:sweeps (tests/golden/tab_sweeps.txt) and the check of
instrumented sweep counters against it."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tab_sweeps.txt")


def table():
    """{partition type: (factorization-stage sweeps, solve-stage sweeps)}."""
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = (int(line[1]), int(line[2]))
    return out


def per_partition(counts, stage, p):
    """Full sweeps per partition, by type, from counters keyed (stage, type,
    full) for a plan with p >= 3 partitions (one first, p - 2 middle, one
    last)."""
    return {"first": counts[(stage, "first", True)],
            "last": counts[(stage, "last", True)],
            "middle": counts[(stage, "middle", True)] / (p - 2)}


def check(counts, p, stages=("factor", "solve", "solve_t")):
    """Assert the counters reproduce the table for every stage that ran."""
    tab = table()
    for stage in stages:
        col = 0 if stage == "factor" else 1
        got = per_partition(counts, stage, p)
        assert got["first"] == tab["first_last"][col], (stage, got)
        assert got["last"] == tab["first_last"][col], (stage, got)
        assert got["middle"] == tab["middle"][col], (stage, got)
        assert counts[(stage, "single", True)] == 0 and counts[(stage, "single", False)] == 0


def from_array(arr):
    """Counters in the KParams::sweeps layout -> dict keyed (stage, type, full)."""
    out = {}
    for si, stage in enumerate(("factor", "solve", "solve_t")):
        for ti, typ in enumerate(("single", "first", "middle", "last")):
            for full in (0, 1):
                out[(stage, typ, bool(full))] = int(arr[(si * 4 + ti) * 2 + full])
    return out
