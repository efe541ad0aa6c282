"""Admission logic of the serving loop on the CPU, with a stand-in for the
device pool that keeps the pool's contract (md_validate, md_attach refusing
with MD_E_CAPACITY when the arena is full, md_advance / md_poll with step
targets and status bits): a job that can never fit is rejected with an
error result instead of blocking the queue, a job whose replica stops with
an error bit is retired with an error result, and every other job runs."""
import dataclasses

import numpy as np
import pytest

import md_inputs as I
from paper_0912_3824_amd import mdx
from paper_0912_3824_amd.serve import Server


class FakePool:
    def __init__(self, max_slots, max_particles, fail_n=None):
        self.max_slots, self.cap, self.fail_n = max_slots, max_particles, fail_n
        self.sizes, self.steps, self.target, self.bits = {}, {}, {}, {}

    def validate(self, n, box):
        return mdx.MD_E_CAPACITY if n > self.cap else 0

    def attach(self, slot, n, box, species, pos, vel):
        if slot in self.sizes:
            raise mdx.MdError(-7, "slot busy")
        if sum(self.sizes.values()) + n > self.cap:
            raise mdx.MdError(mdx.MD_E_CAPACITY, "particle arena full")
        self.sizes[slot], self.steps[slot], self.bits[slot] = n, 0, 0

    def set_target(self, slot, t):
        self.target[slot] = t

    def advance(self, k):
        for s in self.sizes:
            if self.bits[s]:
                continue
            self.steps[s] = min(self.target[s], self.steps[s] + k)
            if self.sizes[s] == self.fail_n and self.steps[s] >= 50:
                self.steps[s], self.bits[s] = 50, mdx.MD_ST_LIST_OVERFLOW

    def poll(self):
        steps = np.full(self.max_slots, -1, dtype=np.int64)
        status = np.zeros(self.max_slots, dtype=np.int32)
        for s in self.sizes:
            steps[s] = self.steps[s]
            status[s] = self.bits[s] | (mdx.MD_ST_AT_FULL_STEP if self.steps[s] >= self.target[s] else 0)
        return steps, status

    def get_state(self, slot):
        n = self.sizes[slot]
        return np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3), dtype=np.int32)

    def detach(self, slot):
        for d in (self.sizes, self.steps, self.target, self.bits):
            d.pop(slot)


@dataclasses.dataclass
class _Sys:
    n: int
    box: float = 50.0
    species: object = None
    pos: object = None
    vel: object = None


def _serve(jobs, pool, slots=2):
    built = []
    srv = Server(None, max_slots=slots, chunk_steps=64, pool=pool,
                 make_system=lambda j: built.append(j.job_id) or _Sys(j.n))
    res = srv.run(jobs, time_scale=0.0)
    return res, built


def test_oversize_job_is_rejected_and_does_not_block_the_queue():
    jobs = [I.Job(0, 0.0, 5000, 100, 0.5, 1),   # never fits (arena 4000)
            I.Job(1, 0.0, 1500, 200, 0.5, 2),
            I.Job(2, 0.0, 2500, 300, 0.5, 3),
            I.Job(3, 0.0, 1000, 100, 0.5, 4)]
    res, built = _serve(jobs, FakePool(2, 4000))
    assert res["failed"] == [0]
    done = {r.job_id: r for r in res["results"]}
    assert set(done) == {0, 1, 2, 3}
    assert "does not fit" in done[0].error
    assert all(done[k].error is None and done[k].pos.shape == (jobs[k].n, 3) for k in (1, 2, 3))
    assert res["particle_steps"] == 1500 * 200 + 2500 * 300 + 1000 * 100
    assert sorted(built) == [0, 1, 2, 3]  # each job's system built once


def test_job_refused_by_an_empty_pool_is_rejected():
    """md_validate passes but md_attach refuses with nothing else running
    (e.g. the first lists overflow): rejected, not retried forever."""
    class Refusing(FakePool):
        def attach(self, slot, n, box, species, pos, vel):
            if n == 777:
                raise mdx.MdError(mdx.MD_E_CAPACITY, "neighbour list overflow at attach")
            super().attach(slot, n, box, species, pos, vel)
    jobs = [I.Job(0, 0.0, 777, 100, 0.5, 1), I.Job(1, 0.0, 1000, 100, 0.5, 2)]
    res, _ = _serve(jobs, Refusing(2, 4000))
    assert res["failed"] == [0]
    assert "overflow" in {r.job_id: r for r in res["results"]}[0].error


def test_replica_stopped_by_an_error_bit_is_retired_with_an_error():
    jobs = [I.Job(0, 0.0, 1200, 500, 0.5, 1), I.Job(1, 0.0, 900, 300, 0.5, 2),
            I.Job(2, 0.0, 800, 200, 0.5, 3)]
    res, _ = _serve(jobs, FakePool(2, 4000, fail_n=900))
    assert res["failed"] == [1]
    r1 = {r.job_id: r for r in res["results"]}[1]
    assert "step 50" in r1.error and "0x1" in r1.error
    assert res["particle_steps"] == 1200 * 500 + 800 * 200
