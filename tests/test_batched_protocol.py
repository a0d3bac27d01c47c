"""Host model of the persistent batched kernel's pass protocol (CPU only).

Between two passes a workgroup may sweep its vertex tiles and move each
vertex up its tree with a plain store (the step taken after a pass in which
some find stopped at the walk bound).  Hooks of the next pass, by other
workgroups, are atomicMin operations on roots.  A hook either joins two trees
or, when it finds the root already linked, keeps the pair still to be joined
as an edge (Section III-A.2: a partition joins its minimum neighbour and no
connection may be lost).

The model runs three workgroups on six vertices, one memory operation at a
time, over every interleaving: a sweep J of vertices 5 and 4 and two hooking
edges B = (1, 5) and C = (0, 5), on a forest where 4 hangs below 3 and 3
below 2.  If the sweep may run beside the
hooks, some interleaving erases C's link: J reads parent[5] = 1 after B's
hook, C lowers it to 0 and keeps only the displaced pair (1, 5), and J's
store then puts back 1, so vertex 0 is cut off.  With a grid barrier between
the sweep and the next pass (the kernel's protocol), every interleaving
keeps the input's connectivity.
"""

def _find(parent, x):
    while parent[x] != x:
        x = parent[x]
    return x


def hook_edge(a, c, kept):
    """One edge of a plain SV pass (one hook attempt), as a generator that
    yields before each shared-memory operation; ops act on `mem`."""
    def run(mem):
        ra = a
        while True:                       # find(a), one read per step
            yield
            p = mem[ra]
            if p == ra:
                break
            ra = p
        rc = c
        while True:
            yield
            p = mem[rc]
            if p == rc:
                break
            rc = p
        if ra == rc:
            return
        lo, hi = min(ra, rc), max(ra, rc)
        yield
        old = mem[hi]                     # atomicMin(&parent[hi], lo)
        mem[hi] = min(old, lo)
        if old == hi:
            return                        # hi was a root: joined
        kept.append((old, hi) if old > lo else (lo, hi))
    return run


def sweep(xs):
    """The deep-chain sweep: for each x, read parent[x]; if x is not a root,
    store the root reached from it (plain store)."""
    def run(mem):
        for x in xs:
            yield
            p = mem[x]
            if p == x:
                continue
            r = p
            while True:
                yield
                q = mem[r]
                if q == r:
                    break
                r = q
            yield
            mem[x] = r
    return run


def _run_schedule(agents, order, init, first=None):
    """Run agents (generator factories) on a copy of the forest `init`: agent
    `first` (if given) runs to completion alone, as across a grid barrier;
    then agent order[i] advances one operation at step i (an exhausted agent
    is skipped), and whatever is left runs to the end."""
    mem = list(init)
    gens = [a(mem) for a in agents]
    alive = [True] * len(gens)

    def step(k):
        try:
            next(gens[k])
        except StopIteration:
            alive[k] = False

    if first is not None:
        while alive[first]:
            step(first)
    for k in order:
        if alive[k]:
            step(k)
    for k in range(len(gens)):
        while alive[k]:
            step(k)
    return mem


def _components(n, pairs):
    p = list(range(n))
    for a, b in pairs:
        ra, rb = _find(p, a), _find(p, b)
        if ra != rb:
            p[max(ra, rb)] = min(ra, rb)
    return [_find(p, x) for x in range(n)]


def _interleavings(lengths):
    """All distinct orders in which agents with these step counts advance."""
    total = sum(lengths)

    def rec(left, acc):
        if len(acc) == total:
            yield tuple(acc)
            return
        for k, L in enumerate(left):
            if L:
                left[k] -= 1
                acc.append(k)
                yield from rec(left, acc)
                acc.pop()
                left[k] += 1
    yield from rec(list(lengths), [])


# forest at the barrier: vertex 4 hangs below 3, 3 below 2 (linked in an
# earlier pass); 0, 1 and 5 are roots.  The next pass hooks (1, 5) and (0, 5);
# the sweep moves 5 and 4 up.
N = 6
INIT = [0, 1, 2, 2, 3, 5]
EDGES = [(1, 5), (0, 5)]
TRUTH = _components(N, EDGES + [(x, INIT[x]) for x in range(N) if INIT[x] != x])


def _outcomes(with_barrier):
    bad = 0
    total = 0
    lengths = [5, 5] if with_barrier else [4, 4, 4]
    for order in _interleavings(lengths):
        kept = []
        agents = [sweep([5, 4]), hook_edge(*EDGES[0], kept), hook_edge(*EDGES[1], kept)]
        if with_barrier:
            mem = _run_schedule(agents, tuple(k + 1 for k in order), INIT, first=0)
        else:
            mem = _run_schedule(agents, order, INIT)
        links = [(x, mem[x]) for x in range(N) if mem[x] != x]
        total += 1
        if _components(N, links + kept) != TRUTH:
            bad += 1
    return bad, total


def test_sweep_beside_hooks_can_lose_a_connection():
    bad, total = _outcomes(with_barrier=False)
    assert total > 1000 and bad > 0


def test_sweep_then_barrier_keeps_every_connection():
    bad, total = _outcomes(with_barrier=True)
    assert total == 252 and bad == 0
