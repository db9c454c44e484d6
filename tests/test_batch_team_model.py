"""A host model of the batched kernel's team scheduling, checked for the
invariants the kernel and its workspace rely on.

The kernel (k_bbpgd_batch) forms teams of T0 consecutive workgroup slots in
each XCD; a team's leader takes the next queue position k; if the
position's size class t_k is smaller than the team, the team halves (the
lower half keeps k, the upper half becomes a team of its own and takes the
next position) until it has t_k members. A team is a node of its initial
team's binary tree, numbered heap-style (1 = the initial team, 2v and 2v + 1
the halves of v), and its barrier and partial sums live at index
team0 * 2 T0 + node. The model replays that logic with random instance
durations and checks: every queue position is processed exactly once, by a
team of exactly min(t_k, T0) members; every node index stays below the
2 x grid entries the workspace holds; every team eventually leaves."""
import heapq
import random

import pytest


def _run(grid, t0, tcls, seed, xcds=8):
    rnd = random.Random(seed)
    per_xcd = [0] * xcds
    for w in range(grid):  # round-robin dispatch over the XCDs
        per_xcd[w % xcds] += 1
    teams, base = [], 0
    for x in range(xcds):
        teams += [base + m for m in range(per_xcd[x] // t0)]
        base += per_xcd[x] // t0
    nnodes = 2 * grid
    ready = [(0.0, team0, 1, t0) for team0 in teams]  # (time, initial team, node, size)
    heapq.heapify(ready)
    nxt, done, left, created = 0, {}, 0, len(teams)
    while ready:
        now, team0, node, size = heapq.heappop(ready)
        k, nxt = nxt, nxt + 1
        if k >= len(tcls):
            left += 1
            continue
        tk = min(tcls[k], size)
        while size > tk:  # halve: the upper half becomes a team and goes back to the queue
            size //= 2
            upper = 2 * node + 1
            assert team0 * 2 * t0 + upper < nnodes
            heapq.heappush(ready, (now, team0, upper, size))
            created += 1
            node = 2 * node
        assert team0 * 2 * t0 + node < nnodes
        assert k not in done
        done[k] = size
        heapq.heappush(ready, (now + rnd.random() * tk, team0, node, size))
    assert left == created  # every team, initial or split off, left the loop once
    assert sorted(done) == list(range(len(tcls)))
    assert all(done[k] == min(tcls[k], t0) for k in done)


@pytest.mark.parametrize("grid,t0", [(256, 32), (256, 16), (256, 8), (256, 1), (128, 16),
                                     (248, 16), (64, 8)])
def test_team_halving_processes_every_position_once_at_its_class(grid, t0):
    for seed in range(25):
        rnd = random.Random(1000 * grid + 10 * t0 + seed)
        n = rnd.choice([0, 1, 2, 7, 100, 512])
        sizes = [s for s in (1, 2, 4, 8, 16, 32) if s <= t0]
        # classes never grow along the queue (it is ordered by nonzeros)
        tcls = sorted((rnd.choice(sizes) for _ in range(n)), reverse=True)
        _run(grid, t0, tcls, seed)
