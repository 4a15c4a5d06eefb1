"""Admission policy of the serving loop (host logic, no GPU)."""
import pytest

from paper_2508_19737_amd.serve import Admission


class R:
    def __init__(self, rid):
        self.rid = rid
        self.cancelled = False


def test_fifo_and_budget():
    a = Admission(max_slots=4, budget_bytes=100)
    for i, c in enumerate([40, 50, 30, 5]):
        a.offer(R(i), c)
    got = [r.rid for r, _ in a.admit()]
    assert got == [0, 1]                 # 40 + 50 fit, 30 does not: head blocks (strict FIFO)
    assert a.used == 90 and a.slots == 2
    a.release(40)
    assert [r.rid for r, _ in a.admit()] == [2, 3]
    assert a.used == 85 and a.slots == 3


def test_one_slot_tiny_budget_queues_not_fails():
    a = Admission(max_slots=1, budget_bytes=10)
    for i in range(5):
        a.offer(R(i), 7)
    order = []
    for _ in range(5):
        adm = a.admit()
        assert len(adm) == 1
        order.append(adm[0][0].rid)
        assert a.admit() == []           # slot taken: the rest wait
        a.release(adm[0][1])
    assert order == [0, 1, 2, 3, 4] and not a.rejected


def test_never_fits_is_rejected_and_cancel_frees_position():
    a = Admission(max_slots=2, budget_bytes=10)
    a.offer(R(0), 11)
    assert [r.rid for r in a.rejected] == [0]
    a.offer(R(1), 6)
    a.offer(R(2), 6)
    a.offer(R(3), 4)
    assert a.cancel(2) and not a.cancel(42)
    assert [r.rid for r, _ in a.admit()] == [1, 3]


def test_bad_limits():
    with pytest.raises(ValueError):
        Admission(0, 10)
    with pytest.raises(ValueError):
        Admission(1, 0)


def test_shrink_keeps_the_slot():
    a = Admission(max_slots=2, budget_bytes=100)
    a.offer(R(0), 70)            # 40 resident + 30 while building
    a.offer(R(1), 50)
    assert [r.rid for r, _ in a.admit()] == [0]
    a.shrink(30)                 # build done: only the resident part stays
    assert a.used == 40 and a.slots == 1
    assert [r.rid for r, _ in a.admit()] == [1]
    a.release(40)
    a.release(50)
    assert a.used == 0 and a.slots == 0
