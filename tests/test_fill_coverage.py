"""Host replay of how a fill launch covers its events (no GPU).

The fill kernel gives workgroup b the events [b * per_block, min(n, (b+1) *
per_block)); each iteration of its loop covers `threads * U` consecutive
events, event base + j * threads + tid for thread tid and j < U, first the
full iterations with no range check and then at most one partial iteration
that skips offsets past the workgroup's range.  The prefetch of the next
iteration reads through a buffer descriptor sized to the workgroup's range, so
offsets past it return zeros without touching memory.

These tests replay that arithmetic (the plan's grid formulas and the loop
bounds) on the CPU for the launch shapes the GPU tests use, including the
two-axis weighted fill with global atomics (326 workgroups of 1024 threads
and 3 events each for 1,000,003 events), and require every event to be
accumulated exactly once and every load to stay inside the descriptor or
return zero.
"""
import numpy as np
import pytest


def plan_grid(n, threads, unroll, blocks_max):
    """Workgroups and events per workgroup, as the plan computes them."""
    step = threads * unroll
    g = min(blocks_max, (n + step - 1) // step)
    g = max(g, (n + (1 << 28) - 1) >> 28, 1)
    per = (n + g - 1) // g
    per = (per + step - 1) // step * step
    g = max(1, (n + per - 1) // per)
    return g, per


def replay(n, threads, unroll, g, per):
    """Counts how often each event is accumulated, and checks each load."""
    seen = np.zeros(n, dtype=np.int64)
    step = threads * unroll
    tid = np.arange(threads, dtype=np.int64)
    for b in range(g):
        start = b * per
        end = min(start + per, n)
        ln = max(end - start, 0)
        assert ln * 8 < 2 ** 32, "a workgroup's byte offsets fit 32 bits"
        base = 0
        batches = []
        while base + step <= ln:          # full iterations
            batches.append((base, True))
            base += step
        while base < ln:                  # the partial one
            batches.append((base, False))
            base += step
        for base, full in batches:
            for j in range(unroll):
                off = base + j * threads + tid
                ok = np.ones(threads, bool) if full else off < ln
                if full:
                    assert off.max() < ln, "a full iteration stays in range"
                np.add.at(seen, start + off[ok], 1)
                # the prefetch of the next iteration: in range or zero-filled
                nxt = base + step + j * threads + tid
                assert np.all((nxt < ln) | (nxt * 8 >= ln * 8))
    return seen


@pytest.mark.parametrize("n,threads,unroll,blocks_max", [
    (1_000_003, 1024, 3, 512),     # 2D weighted, staged edges, global atomics
    (1_000_003, 1024, 3, 256),
    (3_000_017, 1024, 8, 256),     # 1D learned
    (2_000_000, 1024, 2, 512),     # 3D
    (1, 1024, 4, 512), (63, 256, 4, 512), (65, 1024, 6, 512), (1025, 512, 3, 512),
    (8193, 1024, 4, 512), (99_991, 1024, 3, 512),
])
def test_every_event_once(n, threads, unroll, blocks_max):
    g, per = plan_grid(n, threads, unroll, blocks_max)
    assert (g - 1) * per < n <= g * per
    seen = replay(n, threads, unroll, g, per)
    assert np.all(seen == 1), "events covered %s times" % np.unique(seen).tolist()


def test_global_weighted_2d_launch_shape():
    # the launch of the weighted two-axis fill with global atomics
    g, per = plan_grid(1_000_003, 1024, 3, 512)
    assert (g, per) == (326, 3072)
    assert 1_000_003 - (g - 1) * per == 1603   # the last workgroup's partial batch
