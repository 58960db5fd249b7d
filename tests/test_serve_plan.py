"""Host logic of the serving scheduler (paper_2511_15022_amd/serve.py): the
longest-processing-time-first plan, checked against an exhaustive search of
the best makespan on small batches and against Graham's 4/3 bound."""
import itertools

import numpy as np

from paper_2511_15022_amd import serve


class R:
    def __init__(self, index, cost):
        self.index, self.c = index, cost


def makespan(queues):
    return max(sum(r.c for r in q) for q in queues)


def test_every_request_planned_once_and_queues_shortest_first():
    rng = np.random.default_rng(1)
    reqs = [R(i, float(rng.integers(1, 50))) for i in range(23)]
    queues = serve.plan(reqs, 4, lambda r: r.c)
    assert sorted(r.index for q in queues for r in q) == list(range(23))
    for q in queues:
        assert [r.c for r in q] == sorted(r.c for r in q)


def test_lpt_within_graham_bound_of_the_optimum():
    rng = np.random.default_rng(2)
    for trial in range(20):
        m = int(rng.integers(2, 4))
        reqs = [R(i, float(rng.integers(1, 30))) for i in range(int(rng.integers(3, 8)))]
        best = min(
            max(sum(r.c for r, a in zip(reqs, assign) if a == k) for k in range(m))
            for assign in itertools.product(range(m), repeat=len(reqs)))
        got = makespan(serve.plan(reqs, m, lambda r: r.c))
        assert best <= got <= (4.0 / 3.0 - 1.0 / (3 * m)) * best + 1e-9


def test_single_stream_holds_everything_in_cost_order():
    reqs = [R(i, c) for i, c in enumerate([5.0, 1.0, 3.0, 3.0])]
    (q,) = serve.plan(reqs, 1, lambda r: r.c)
    assert [r.index for r in q] == [1, 2, 3, 0]
