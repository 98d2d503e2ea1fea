"""The level-barrier schedule's device-wide barrier, as a counting protocol.

`ls_barrier` in kernels.hip is a combining tree: each wavefront increments its
group's arrival counter (groups of 64 wavefronts, the last one partial); the
group's last arrival increments the top counter; the last of those sets every
group's release flag to the barrier's generation; a wavefront leaves when its
group's flag has reached the generation. Counters are never reset: barrier g
is complete when a group counter reaches g times the group's size.

This test runs that counting, step by step, for every wavefront of a grid
under seeded random interleavings, and checks what the kernel relies on:

* safety: no wavefront leaves barrier g before every wavefront has arrived
  at it (so every store of level g - 1 precedes every read of level g);
* liveness: every wavefront leaves every barrier (no count is missed across
  generations, whatever the order of arrivals);
* exactly one last arrival per group and one top-level last arrival per
  barrier, so each flag is written once per generation.

Memory ordering (the fences around these atomics) is outside a counting
model; the GPU parity suite runs every case under the schedule.
"""
import random

import pytest

GROUP = 64


def run_grid(nw: int, n_barriers: int, seed: int):
    rng = random.Random(seed)
    M = (nw + GROUP - 1) // GROUP
    group_cnt = [0] * M
    top = [0]
    flag = [0] * M
    arrived = [0] * (n_barriers + 1)   # arrivals per generation
    group_last = [[0] * M for _ in range(n_barriers + 1)]
    top_last = [0] * (n_barriers + 1)

    def wave(b):
        m = b // GROUP
        gs = GROUP if m + 1 < M else nw - GROUP * m
        for gen in range(1, n_barriers + 1):
            yield  # the level's work
            old = group_cnt[m]
            group_cnt[m] += 1          # one atomic fetch_add
            arrived[gen] += 1
            yield
            if old + 1 == gs * gen:
                group_last[gen][m] += 1
                t = top[0]
                top[0] += 1            # one atomic fetch_add
                yield
                if t + 1 == M * gen:
                    top_last[gen] += 1
                    for i in range(M):
                        flag[i] = gen  # one store per flag
                        yield
            while flag[m] < gen:       # polling
                yield
            assert arrived[gen] == nw, f"left barrier {gen} with {arrived[gen]} of {nw} arrived"

    live = {b: wave(b) for b in range(nw)}
    steps = 0
    while live:
        b = rng.choice(list(live))
        try:
            next(live[b])
        except StopIteration:
            del live[b]
        steps += 1
        assert steps < 200 * nw * (n_barriers + 1) + 10_000, "the grid did not drain"
    for gen in range(1, n_barriers + 1):
        assert group_last[gen] == [1] * M
        assert top_last[gen] == 1
    for m in range(M):
        gs = GROUP if m + 1 < M else nw - GROUP * m
        assert group_cnt[m] == gs * n_barriers
    assert top[0] == M * n_barriers


@pytest.mark.parametrize("nw", [1, 2, 63, 64, 65, 127, 128, 129, 300])
def test_barrier_counting_is_safe_and_live(nw):
    for seed in range(3):
        run_grid(nw, n_barriers=4, seed=seed * 1000 + nw)


def test_barrier_counting_full_grid():
    """4,096 wavefronts (the grid on 256 CUs at four per SIMD), 3 barriers."""
    run_grid(4096, n_barriers=3, seed=7)
