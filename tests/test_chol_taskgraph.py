"""Host model of the blocked Cholesky factorisation's task graph (CPU).

The factorisation kernel splits the work on 64 x 64 tiles into tasks, handed out in ticket order to
whichever workgroup asks next; tasks hand tiles over through per-tile flags (a producer publishes a
flag after its stores, a consumer waits for the flag before its loads). Nothing else orders two
workgroups, so a task that reads a tile must be ordered, through a chain of such flags, after the
write it needs and before any later write that replaces it. This model writes down, per task and
in program order, the flags each task waits for, the tile versions it reads, the tiles it writes
and the flags it publishes, and checks those two conditions and that every wait is on a task with
a smaller ticket (so that every wait ends). The tasks, for block column c and row block i (row
block nb is the right-hand side):
  CRIT(j)    the critical chain, all steps on one workgroup: L_{j,j-1} = C_{j,j-1} Linv_{j-1}^T
             written over tile (j, j-1) (flag fin(j, j-1)), then C_jj factored and inverted
             (Linv_j, flag dinv(j)); C_jj and C_{j,j-1} are the raw blocks for j <= 1, else the
             partials of DIAGP(j) and SUBP(j)
  DIAGP(j)   C_jj = A_jj - sum_{k <= j-2} L_jk L_jk^T over tile (j, j) (flag pdiag(j))
  SUBP(j)    C_{j,j-1} = A_{j,j-1} - sum_{k <= j-2} L_jk L_{j-1,k}^T into the upper-triangle tile
             (j-1, j) (flag psub(j)); its last term uses L_{j-1,j-2}, formed from SUBP(j-1)'s tile
             and Linv_{j-2} for j >= 3, read from tile (1, 0) once final for j = 2
  FULL(i, c) L_ic = (A_ic - sum_{k < c} L_ik L_ck^T) Linv_c^T over tile (i, c) (flag fin(i, c))
"""
import itertools

import pytest

RAW = "raw"


def _writer(i, k, nb):
    """The task whose write of tile (i, k) holds L_ik."""
    return f"CRIT({i})" if (i == k + 1 and i < nb) else f"FULL({i},{k})"


def _tasks(nb, subp2_reads_raw=False):
    """[(name, events)] in ticket order. Events: ("wait", flag), ("read", tile, writer),
    ("write", tile), ("pub", flag); writer is the task whose write the read must see, or RAW for the
    assembled matrix. subp2_reads_raw plants the ordering mistake of an earlier SUBP(2)."""
    out = []
    for j in range(nb):
        if j >= 2:
            ev = [("read", ("A", j, j), RAW)]
            for k in range(j - 1):
                ev += [("wait", ("fin", j, k)), ("read", ("A", j, k), _writer(j, k, nb))]
            ev += [("write", ("A", j, j)), ("pub", ("pdiag", j))]
            out.append((f"DIAGP({j})", ev))
            c, m = j - 1, j - 2
            ev = [("read", ("A", j, c), RAW)]
            for k in range(j - 2):
                ev += [("wait", ("fin", j, k)), ("wait", ("fin", c, k)),
                       ("read", ("A", j, k), _writer(j, k, nb)), ("read", ("A", c, k), _writer(c, k, nb))]
            if c >= 2:
                ev += [("wait", ("dinv", m)), ("wait", ("psub", c)),
                       ("read", ("U", c - 1, c), f"SUBP({c})"), ("read", ("Linv", m), f"CRIT({m})")]
            elif subp2_reads_raw:
                ev += [("wait", ("dinv", 0)), ("read", ("A", 1, 0), RAW), ("read", ("Linv", 0), "CRIT(0)")]
            else:
                ev += [("wait", ("fin", 1, 0)), ("read", ("A", 1, 0), "CRIT(1)")]
            ev += [("wait", ("fin", j, m)), ("read", ("A", j, m), _writer(j, m, nb)),
                   ("write", ("U", j - 1, j)), ("pub", ("psub", j))]
            out.append((f"SUBP({j})", ev))
        ev = []
        if j >= 2:
            ev += [("wait", ("pdiag", j)), ("wait", ("psub", j)),
                   ("read", ("A", j, j), f"DIAGP({j})"), ("read", ("U", j - 1, j), f"SUBP({j})")]
        else:
            ev.append(("read", ("A", j, j), RAW))
            if j == 1:
                ev.append(("read", ("A", 1, 0), RAW))
        if j >= 1:
            ev += [("read", ("Linv", j - 1), f"CRIT({j - 1})"), ("write", ("A", j, j - 1)), ("pub", ("fin", j, j - 1))]
        ev += [("write", ("Linv", j)), ("pub", ("dinv", j))]
        out.append((f"CRIT({j})", ev))
        for i in list(range(j + 2, nb)) + [nb]:
            ev = [("read", ("A", i, j), RAW)]
            for k in range(j):
                ev += [("wait", ("fin", i, k)), ("wait", ("fin", j, k)),
                       ("read", ("A", i, k), _writer(i, k, nb)), ("read", ("A", j, k), _writer(j, k, nb))]
            ev += [("wait", ("dinv", j)), ("read", ("Linv", j), f"CRIT({j})"),
                   ("write", ("A", i, j)), ("pub", ("fin", i, j))]
            out.append((f"FULL({i},{j})", ev))
    return out


def _hazards(nb, tasks=None, **kw):
    """Violations of the three conditions, as readable strings (for the given task list, else the
    model's)."""
    tasks = _tasks(nb, **kw) if tasks is None else tasks
    ticket = {name: t for t, (name, _) in enumerate(tasks)}
    nodes = [(name, e) for name, ev in tasks for e in range(len(ev))]
    ev_of = dict(tasks)
    succ = {n: [] for n in nodes}
    publisher = {}
    for name, ev in tasks:
        for e, x in enumerate(ev):
            if e + 1 < len(ev):
                succ[(name, e)].append((name, e + 1))
            if x[0] == "pub":
                assert x[1] not in publisher, f"flag {x[1]} published twice"
                publisher[x[1]] = (name, e)
    for j in range(nb - 1):  # the chain workgroup runs CRIT(j) and then CRIT(j + 1)
        succ[(f"CRIT({j})", len(ev_of[f"CRIT({j})"]) - 1)].append((f"CRIT({j + 1})", 0))
    bad = []
    for name, ev in tasks:
        for e, x in enumerate(ev):
            if x[0] == "wait":
                if x[1] not in publisher:
                    bad.append(f"{name} waits for {x[1]}, which no task publishes")
                    continue
                succ[publisher[x[1]]].append((name, e))
                if ticket[publisher[x[1]][0]] >= ticket[name]:
                    bad.append(f"{name} waits for {x[1]} of {publisher[x[1]][0]}, a later ticket")
    reach = {}
    for n in nodes:  # events reachable from n (happens-after n)
        seen, stack = set(), [n]
        while stack:
            for s in succ[stack.pop()]:
                if s not in seen:
                    seen.add(s)
                    stack.append(s)
        reach[n] = seen
    writes = {}
    for name, ev in tasks:
        for e, x in enumerate(ev):
            if x[0] == "write":
                writes.setdefault(x[1], []).append((name, e))
    for name, ev in tasks:
        for e, x in enumerate(ev):
            if x[0] != "read":
                continue
            tile, want, r = x[1], x[2], (name, e)
            ws = writes.get(tile, [])
            src = [w for w in ws if w[0] == want]
            if want != RAW and (not src or r not in reach[src[0]]):
                bad.append(f"{name} reads {tile} of {want} without waiting for it")
            for w in ws:
                if w[0] == want:
                    continue
                if src and src[0] in reach[w]:
                    continue  # an older version, replaced before the one read
                if w not in reach[r]:  # else the read is done before this write replaces the tile
                    bad.append(f"{name} reads {tile} ({want}) unordered with the write of {w[0]}")
    return bad


@pytest.mark.parametrize("nb", range(1, 10))
def test_task_graph_orders_every_read(nb):
    assert _hazards(nb) == []


def test_model_catches_the_unordered_raw_read():
    """The earlier SUBP(2), which read the raw A_{1,0} from tile (1, 0) after waiting only for
    Linv_0, races with CRIT(1)'s write of L_{1,0} over that tile."""
    bad = _hazards(4, subp2_reads_raw=True)
    assert any("SUBP(2) reads ('A', 1, 0)" in b and "CRIT(1)" in b for b in bad), bad


def test_model_catches_a_missing_wait():
    """Dropping any one wait of any task (with its flag left published) breaks an ordering the
    model then reports, so no wait in the model is redundant."""
    nb = 5
    base = _tasks(nb)
    for name, ev in base:
        for e, x in enumerate(ev):
            if x[0] != "wait":
                continue
            cut = [(n, [y for f, y in enumerate(v) if not (n == name and f == e)]) for n, v in base]
            assert _hazards(nb, tasks=cut), f"the wait of {name} for {x[1]} is not needed"


def test_ticket_count_closed_form():
    """The task count per block column equals the closed form the kernel uses to decode tickets:
    g(j) = (2 if j >= 2 else 0) + 1 + max(nb - j - 2, 0) + 1."""
    for nb in range(1, 40):
        names = [n for n, _ in _tasks(nb)]
        for j in range(nb):
            g = (2 if j >= 2 else 0) + 1 + max(nb - j - 2, 0) + 1
            got = sum(1 for n in names if n in (f"DIAGP({j})", f"SUBP({j})", f"CRIT({j})")
                      or n.startswith("FULL(") and n.endswith(f",{j})"))
            assert got == g, (nb, j)
        assert len(set(names)) == len(names)
    assert list(itertools.islice((n for n, _ in _tasks(4)), 6)) == [
        "CRIT(0)", "FULL(2,0)", "FULL(3,0)", "FULL(4,0)", "CRIT(1)", "FULL(3,1)"]
