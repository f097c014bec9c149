"""The stack bound of the four-wide traversal, on a CPU model.

The four-wide descent visits, for an internal node m of the binary tree, the
up to four boxes one level below m's children: it goes on with the nearer
pair's nearer hit slot, pushes the farther pair as one entry (m's child itself
when both of its slots are hit, else the one hit slot) and then the nearer
pair's other hit slot, and pops when nothing is hit.  Leaves are set aside one
at a time (the postponed leaf) and the descent pops on.  The claim behind the
kernel's fixed stack is that the entries never exceed the internal-node depth
bound plus two.  This model replays that push/pop logic on random binary
trees of maximal depth with random hit patterns and distances, and on an
adversarial comb that pushes two entries per visit, and checks the bound,
that no leaf is reached twice, and that every leaf the binary traversal
reaches with the same box tests is reached (a popped child entry re-tests
the level below it, so the four-wide walk may also reach leaves whose
skipped ancestor box would have missed; the certified triangle tests make
that harmless)."""
import numpy as np
import pytest

DEPTH = 18              # internal-node depth bound of the builder
STACK = DEPTH + 2       # entries of the traversal stack


def random_tree(rng, max_depth, p_inner, cap=20000):
    """Nodes: dict id -> (left, right) for internal nodes; leaves are ints < 0.
    The root is internal; every internal node is at depth <= max_depth; a child
    is internal with probability p_inner (the first child of a node almost
    always, so that deep paths occur), until `cap` nodes exist."""
    children, depth = {}, {0: 0}
    todo, nxt, leaf = [0], 1, -1
    while todo:
        m = todo.pop()
        kids = []
        for k in range(2):
            p = max(0.95, p_inner) if k == 0 else p_inner
            if depth[m] + 1 <= max_depth and nxt < cap and rng.random() < p:
                c = nxt
                nxt += 1
                depth[c] = depth[m] + 1
                todo.append(c)
            else:
                c = leaf
                leaf -= 1
            kids.append(c)
        children[m] = tuple(kids)
    return children, depth


def slots(children, m):
    """The four-wide record of internal node m: (ref, pair) per slot, an empty
    slot as None."""
    out = []
    for c in children[m]:
        if c >= 0:
            out += list(children[c])
        else:
            out += [c, None]
    return out


def wide_walk(children, hit, dist):
    """Visit order of the four-wide descent; hit(ref) and dist(ref) give the
    box test of a slot.  Returns (leaves reached, largest stack height)."""
    stack, ref, leaves, peak = [], 0, [], 0
    while ref is not None:
        if ref < 0:  # a leaf (set aside and tested), then the next entry
            leaves.append(ref)
            ref = stack.pop() if stack else None
            continue
        s = slots(children, ref)
        h = [x is not None and hit(x) for x in s]
        t = [dist(x) if hh else np.inf for x, hh in zip(s, h)]

        def pair(i):
            a, b = 2 * i, 2 * i + 1
            near = a if h[a] and (not h[b] or t[a] <= t[b]) else b
            return near, (b if near == a else a), h[a] or h[b], h[a] and h[b], t[near]
        nA, oA, anyA, bothA, tA = pair(0)
        nB, oB, anyB, bothB, tB = pair(1)
        first_a = anyA and (not anyB or tA <= tB)
        near, nfar, anyN, bothN = (nA, oA, anyA, bothA) if first_a else (nB, oB, anyB, bothB)
        anyF, bothF = (anyB, bothB) if first_a else (anyA, bothA)
        fent = children[ref][1 if first_a else 0] if bothF else (s[nB] if first_a else s[nA])
        if anyF:
            stack.append(fent)
        if bothN:
            stack.append(s[nfar])
        peak = max(peak, len(stack))
        ref = s[near] if anyN else (stack.pop() if stack else None)
    return leaves, peak


def binary_walk(children, hit):
    """Leaves the binary traversal reaches with the same box tests."""
    stack, ref, leaves = [], 0, []
    while ref is not None:
        if ref < 0:
            leaves.append(ref)
            ref = stack.pop() if stack else None
            continue
        h = [c for c in children[ref] if hit(c)]
        stack += h[1:]
        ref = h[0] if h else (stack.pop() if stack else None)
    return leaves


@pytest.mark.parametrize("seed", range(40))
def test_wide_stack_bound_and_leaves(seed):
    rng = np.random.default_rng(seed)
    # deep, nearly complete trees stress the bound; sparse ones the leaf mix
    children, depth = random_tree(rng, DEPTH, p_inner=[0.9, 0.6, 0.3][seed % 3])
    assert max(depth.values()) == DEPTH or len(children) >= 20000 or seed % 3 == 2
    refs = list(children) + [c for kids in children.values() for c in kids if c < 0]
    p_hit = [0.97, 0.8, 0.5][seed % 3]
    hits = {r: bool(rng.random() < p_hit) for r in refs}
    dist = {r: float(rng.random()) for r in refs}

    # a ray reaches a node only through hit boxes; the box of a node contains
    # its children's, so a child's hit is conditioned on its parent's
    def hit(r):
        return hits[r]
    leaves, peak = wide_walk(children, hit, dist.get)
    assert peak <= STACK, (peak, max(depth.values()))
    # the wide walk re-tests nothing it skipped, so it reaches every leaf whose
    # own box and every other box on the way are hit, each once; the binary walk
    # reaches the leaves whose every ancestor box is hit: the wide walk skips the
    # box tests of the children of the root of each record it visits, so it
    # reaches a superset, and every leaf it reaches has a hit box itself
    ref_leaves = set(binary_walk(children, hit))
    assert len(leaves) == len(set(leaves))
    assert ref_leaves <= set(leaves)
    assert all(hits[x] for x in leaves)


def test_wide_stack_peak_on_complete_tree():
    """Every box hit on a complete tree of the maximal depth: the worst case."""
    rng = np.random.default_rng(0)
    children, depth = random_tree(rng, 12, p_inner=1.0)
    leaves, peak = wide_walk(children, lambda r: True, lambda r: float(abs(r) % 7))
    assert len(leaves) == 2 ** 13
    assert peak <= 12 + 2


def test_wide_stack_comb_worst_case():
    """A comb of the maximal depth: every spine node's other child has two
    leaves, every box is hit and the spine is always nearer, so every visit
    pushes two entries while descending two levels: the stack peaks at the
    bound and stays within it."""
    children, spine, nxt, leaf = {}, list(range(DEPTH + 1)), DEPTH + 1, -1
    for d in range(DEPTH + 1):
        if d < DEPTH:
            x = nxt
            nxt += 1
            children[x] = (leaf, leaf - 1)
            leaf -= 2
            children[d] = (spine[d + 1], x)
        else:
            children[d] = (leaf, leaf - 1)
            leaf -= 2
    dist = {r: (0.0 if 0 <= r <= DEPTH else 1.0) for r in list(children) + list(range(leaf, 0))}
    leaves, peak = wide_walk(children, lambda r: True, dist.get)
    assert len(leaves) == 2 * (DEPTH + 1)
    assert set(leaves) == set(range(leaf + 1, 0))
    assert DEPTH <= peak <= STACK, peak
