"""Host logic of the batching mode: grouping of uneven problems into batch plans."""
import dataclasses

import pytest

import workloads as W
from paper_2502_21013_amd.batch import plan_groups, pow2_split, share_key


def test_pow2_split():
    assert pow2_split(1, 64) == [1]
    assert pow2_split(5, 64) == [4, 1]
    assert pow2_split(7, 4) == [4, 2, 1]
    assert pow2_split(64, 16) == [16, 16, 16, 16]
    assert pow2_split(0, 8) == []
    with pytest.raises(ValueError):
        pow2_split(5, 3)


def test_plan_groups_cover_every_problem_once_and_share_their_operators():
    ps = W.config4(0)
    groups = plan_groups(ps)
    flat = sorted(i for g in groups for i in g)
    assert flat == list(range(len(ps)))
    for g in groups:
        assert len(g) & (len(g) - 1) == 0
        assert len({share_key(ps[i]) for i in g}) == 1
    # decreasing cost order
    cost = [(ps[g[0]].n + 1) ** 2 * ps[g[0]].N * len(g) for g in groups]
    assert cost == sorted(cost, reverse=True)


def test_plan_groups_respect_the_slot_cap():
    ps = [W.with_size(p, 16, 1024) for p in W.config4(1, 200)]
    groups = plan_groups(ps, max_batch=1024)
    assert all(len(g) * 512 <= 65536 for g in groups)
    assert sum(len(g) for g in groups) == 200


def test_problems_with_other_conductivity_are_not_batched_together():
    ps = [W.with_size(p, 16, 16) for p in W.config4(2, 4)]
    ps[3] = dataclasses.replace(ps[3], sigma_in=2.0)
    groups = plan_groups(ps)
    assert sorted(len(g) for g in groups) == [1, 2, 1] or sorted(len(g) for g in groups) == [1, 1, 2]
